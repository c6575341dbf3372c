"""The adjoint's default schedule regenerates a step's Chebyshev vectors by
running the Sect. 2.2 three-term recursion backwards from the step's last
pair, v_{k-1} = 2 H~ v_k - v_{k+1}.  Exact in exact arithmetic; this checks on
the CPU, with the oracle's operators and spectral scale, that in floating
point the regenerated vectors match the forward ones to rounding (the
rescaled spectrum lies inside [-1, 1], where the recursion's error growth is
bounded both ways)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W


def forward_and_back(H, lo, hi, dt, psi0):
    plan = O.Plan(lo, hi, dt)
    rowptr, col, val = H.csr()
    A = sp.csr_matrix((val, col, rowptr), shape=(H.n, H.n))
    Ht = (A - plan.b * sp.identity(H.n, format="csr")) / plan.a
    M = plan.M
    v = [psi0, Ht @ psi0]
    for k in range(1, M):
        v.append(2.0 * (Ht @ v[k]) - v[k - 1])
    r = [None] * (M + 1)
    r[M], r[M - 1] = v[M], v[M - 1]
    for k in range(M - 1, 0, -1):
        r[k - 1] = 2.0 * (Ht @ r[k]) - r[k + 1]
    return M, max(np.linalg.norm(r[k] - v[k]) / np.linalg.norm(v[k]) for k in range(M + 1))


@pytest.mark.parametrize("edge", ["zigzag", "armchair"])
@pytest.mark.parametrize("z", [3.0, 31.0, 120.0])
def test_reverse_recursion_ribbon(edge, z):
    eps, psi0 = W.ribbon_inputs(24, 160, 0.5, 3)
    H = O.honeycomb(24, 160, eps, edge=edge)
    lo, hi = H.gershgorin()
    dt = z / (0.5 * 1.01 * (hi - lo))
    M, err = forward_and_back(H, lo, hi, dt, psi0)
    assert M >= 10
    assert err <= 1e-13


def test_reverse_recursion_chain():
    x, dx, V, psi0 = W.double_well_inputs(2000)
    H = O.chain1d(V, dx)
    lo, hi = H.gershgorin()
    dt = 31.0 / (0.5 * 1.01 * (hi - lo))
    M, err = forward_and_back(H, lo, hi, dt, psi0)
    assert M >= 60
    assert err <= 1e-13
