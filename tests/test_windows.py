"""CPU check of the window sampler used by the full-size GPU tests: the
oracle's value at a site from a window around it equals the value from the
whole lattice (the light-cone argument of Sect. 2.2's polynomial)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from windows import chain_sites, ribbon_sample_sites, ribbon_sites


@pytest.mark.parametrize("edge", ["zigzag", "armchair"])
@pytest.mark.parametrize("shape", [(40, 130), (7, 301), (63, 64)])
def test_ribbon_windows_equal_whole_lattice(edge, shape):
    w, l = shape
    eps = W.anderson_disorder(w, l, 1.3, 3)
    psi0 = W.random_state(w * l, 4)
    H = O.honeycomb(w, l, eps, edge=edge)
    lo, hi = H.gershgorin()
    plan = O.Plan(lo, hi, 0.6)
    assert 5 <= plan.M <= 20
    K = 2
    full = O.propagate(H, plan, psi0, K)
    sites = ribbon_sample_sites(w, l, 12, 5)
    # windows must reach the odd-parity origins too (x0 + y0 odd before widening)
    sites += [(y, x) for y in (3, 20, w - 4) for x in (31, 32, l - 30) if 0 <= y < w and 0 <= x < l]
    got = ribbon_sites(w, l, edge, eps, psi0, plan, K, sites)
    ref = np.array([full[y * l + x] for y, x in sites])
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(full).max()


def test_ribbon_window_pins_have_teeth():
    # a window of half the light cone's radius, or one whose origin breaks the
    # brick wall's parity, gives a wrong value: the equalities above are not
    # trivially satisfied
    w, l = 40, 130
    eps = W.anderson_disorder(w, l, 1.3, 3)
    psi0 = W.random_state(w * l, 4)
    H = O.honeycomb(w, l, eps)
    lo, hi = H.gershgorin()
    plan = O.Plan(lo, hi, 0.6)
    full = O.propagate(H, plan, psi0, 1)
    y, x = 20, 60
    e2, p2 = eps.reshape(w, l), psi0.reshape(w, l)

    def window(y0, y1, x0, x1):
        Hw = O.honeycomb(y1 - y0, x1 - x0, np.ascontiguousarray(e2[y0:y1, x0:x1]).reshape(-1))
        out = O.propagate(Hw, plan, np.ascontiguousarray(p2[y0:y1, x0:x1]).reshape(-1), 1)
        return out[(y - y0) * (x1 - x0) + (x - x0)]

    R = plan.M + 1
    assert abs(window(y - R, y + R + 1, x - R, x + R + 1) - full[y * l + x]) <= 1e-14
    h = plan.M // 2
    tol = 1e-10 * np.abs(full).max()  # the GPU tests' site tolerance
    assert abs(window(y - h, y + h + 1, x - h, x + h + 1) - full[y * l + x]) > tol
    # origin (x - R - 1) + (y - R) is odd: the bonds inside the window flip
    assert abs(window(y - R, y + R + 1, x - R - 1, x + R + 1) - full[y * l + x]) > tol


def test_chain_windows_equal_whole_chain():
    n = 3000
    x, dx = W.chain_grid(n, -30, 30)
    V = W.harmonic(x, 0.7)
    psi0 = W.random_state(n, 8)
    H = O.chain1d(V, dx)
    lo, hi = H.gershgorin()
    plan = O.Plan(lo, hi, 0.01)
    full = O.propagate(H, plan, psi0, 3)
    sites = [0, 1, 2, 500, 1499, 2998, 2999]
    got = chain_sites(V, dx, psi0, plan, 3, sites)
    assert np.abs(got - full[sites]).max() <= 1e-13 * np.abs(full).max()
