"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: library
Bessel values, closed forms, dense exact diagonalisation (Sect. 2.1), the
printed numbers of Sects. 3.1-3.3, brute force on tiny inputs, and an
independent tensor-product construction of eq. (ghm).  No GPU is needed.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.special as sp
from scipy.spatial import cKDTree

import oracle as O
import workloads as W


def ed_propagate(Hd, psi0, t):
    """Exact propagation exp(-i H t) psi0 by full diagonalisation (Sect. 2.1)."""
    E, U = np.linalg.eigh(Hd)
    return U @ (np.exp(-1j * E * t) * (U.conj().T @ psi0))


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# ---------------------------------------------------------------------------
# Bessel coefficients and truncation (Sect. 2.2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("z", [1e-9, 0.1, 0.91, 1.22, 3.28, 30.5, 100.0, 1000.0, 7068.0])
def test_bessel_matches_library(z):
    M = O.trunc_order(z)
    J = O.bessel_j(z, M + 8)
    ref = sp.jv(np.arange(M + 9), z)
    # the library value itself carries ~4e-15 absolute error for z >= 100
    tol = 1e-15 if z <= 30.5 else 5e-17 * z + 1e-15
    assert np.abs(J - ref).max() <= tol


def test_bessel_high_precision_points():
    import mpmath as mp
    mp.mp.dps = 30
    for z, ks in [(100.0, [0, 1, 57, 100, 148]), (1000.0, [0, 3, 999, 1101])]:
        J = O.bessel_j(z, max(ks))
        for k in ks:
            assert abs(J[k] - float(mp.besselj(k, z))) <= 3e-16


@pytest.mark.parametrize("z", [0.5, 3.28, 30.5, 250.0, 7068.0])
def test_bessel_parseval(z):
    # J_0^2 + 2 sum J_k^2 = 1: independent of the normalisation used
    J = O.bessel_j(z, O.trunc_order(z) + 30)
    s = J[0] ** 2 + 2.0 * np.sum(J[1:] ** 2)
    assert abs(s - 1.0) <= 3e-14


def test_bessel_tiny_and_zero_argument():
    J = O.bessel_j(0.0, 5)
    assert J[0] == 1.0 and np.all(J[1:] == 0.0)
    J = O.bessel_j(1e-12, 4)
    np.testing.assert_allclose(J, sp.jv(np.arange(5), 1e-12), rtol=1e-14, atol=0)


@pytest.mark.parametrize("z,tol", [(0.0, 1e-15), (1e-6, 1e-15), (0.91, 1e-15), (3.28, 1e-15),
                                   (3.28, 1e-8), (30.5, 1e-15), (100.0, 1e-12), (1000.0, 1e-15)])
def test_truncation_order_brute_force(z, tol):
    # M = (first k > z with |J_k(z)| < tol) - 1, found here by scanning library values
    k = 1
    while not (k > z and abs(sp.jv(k, z)) < tol):
        k += 1
    assert O.trunc_order(z, tol) == k - 1


def test_generating_function():
    # exp(-i E dt) = sum_k gamma_k T_k((E-b)/a) with T_k(x) = cos(k arccos x) (Sect. 2.2)
    rng = np.random.default_rng(7)
    for emin, emax, dt in [(-3.1, 3.3, 1.0), (-0.5, 7.0, 9.4), (10.0, 12.5, 40.0), (-100., 50., 0.3)]:
        a, b = O.scale(emin, emax, 0.01)
        M = O.trunc_order(a * dt)
        g = O.coeffs(a, b, dt, M)
        E = rng.uniform(emin, emax, size=64)
        x = (E - b) / a
        T = np.cos(np.outer(np.arange(M + 1), np.arccos(x)))
        approx = g @ T
        # phases of size |E| dt carry rounding of order eps |E| dt on either side
        tol = 2e-14 + 4 * np.finfo(float).eps * (abs(b) + a) * dt
        np.testing.assert_allclose(approx, np.exp(-1j * E * dt), rtol=0, atol=tol)


def test_scale_matches_paper_definition():
    a, b = O.scale(-2.0, 6.0, 0.01)
    assert b == 2.0
    assert a == pytest.approx(0.5 * (8.0 + 0.08), rel=0, abs=1e-15)
    # |E~| <= 1/(1+alpha) on the spectral interval
    assert (6.0 - b) / a == pytest.approx(1 / 1.01, abs=1e-15)


# ---------------------------------------------------------------------------
# Hamiltonian builders
# ---------------------------------------------------------------------------
def test_chain1d_free_particle_spectrum():
    # V = 0, Dirichlet: eigenvalues (1 - cos(pi m/(n+1)))/dx^2, m = 1..n (DST-I)
    n, dx = 200, 0.1
    H = O.chain1d(np.zeros(n), dx).dense().real
    m = np.arange(1, n + 1)
    E = (1.0 - np.cos(np.pi * m / (n + 1))) / dx ** 2
    np.testing.assert_allclose(np.linalg.eigvalsh(H), np.sort(E), rtol=0, atol=1e-10)
    assert np.allclose(H, H.T)


def _honeycomb_embedding(width, length, edge):
    """Plane coordinates (bond length 1) of brick-wall site (x, y)."""
    y, x = np.meshgrid(np.arange(width), np.arange(length), indexing="ij")
    even = ((x + y) % 2 == 0)
    if edge == "zigzag":
        X = x * math.sqrt(3) / 2
        Y = 1.5 * y + 0.5 * even
    else:
        X = 1.5 * x + 0.5 * even
        Y = y * math.sqrt(3) / 2
    return np.stack([X.reshape(-1), Y.reshape(-1)], axis=1)


@pytest.mark.parametrize("edge", ["zigzag", "armchair"])
def test_honeycomb_bonds_are_nearest_neighbour_pairs(edge):
    # The builder's hopping pairs must be exactly the pairs of honeycomb-lattice
    # points at one bond length, and the points must lie on the honeycomb lattice.
    width, length = 7, 12
    eps = np.zeros(width * length)
    rowptr, col, val = O.honeycomb(width, length, eps, edge=edge, t=1.0).csr()
    bonds = set()
    for i in range(width * length):
        for p in range(rowptr[i], rowptr[i + 1]):
            if col[p] != i:
                assert val[p] == -1.0
                bonds.add((min(i, col[p]), max(i, col[p])))
    pts = _honeycomb_embedding(width, length, edge)
    pairs = cKDTree(pts).query_pairs(r=1.0 + 1e-9)
    assert bonds == set(pairs)
    # every point is A + lattice or B + lattice
    if edge == "zigzag":
        a1, a2, A, B = np.array([math.sqrt(3), 0]), np.array([math.sqrt(3) / 2, 1.5]), \
            np.array([0, 0.5]), np.array([math.sqrt(3) / 2, 0])
    else:
        a1, a2, A, B = np.array([0, math.sqrt(3)]), np.array([1.5, math.sqrt(3) / 2]), \
            np.array([0.5, 0]), np.array([0, math.sqrt(3) / 2])
    Lm = np.stack([a1, a2], axis=1)
    for p in pts:
        ok = False
        for base in (A, B):
            c = np.linalg.solve(Lm, p - base)
            ok |= np.allclose(c, np.round(c), atol=1e-9)
        assert ok


def test_armchair_ribbon_matches_paper_device_size(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "paper_values.json")))["graphene_ribbon"]
    w, l, acc = g["atoms_across"], g["atoms_along"], g["carbon_bond_nm"]
    H = O.honeycomb(w, l, np.zeros(w * l), edge="armchair")
    rowptr, col, _ = H.csr()
    pts = _honeycomb_embedding(w, l, "armchair") * acc
    bonds = {(i, int(c)) for i in range(w * l) for c in col[rowptr[i]:rowptr[i + 1]] if c != i}
    d = np.array([np.linalg.norm(pts[i] - pts[j]) for i, j in bonds])
    np.testing.assert_allclose(d, acc, rtol=1e-12)
    assert round(np.ptp(pts[:, 1]), 2) == g["width_nm"]
    # length measured between the centres of the first and last zigzag chain
    centres = pts[:, 0].reshape(w, l).mean(axis=0)
    assert round(np.ptp(centres), 1) == g["length_nm"]


def _holstein_kron(L, nph, t, w0, g, Delta, periodic):
    """eq. (ghm) built as a tensor product (electron x per-site Fock spaces cut
    at nph), then restricted to total phonon number <= nph.  Basis order:
    electron site slowest, then total phonon number, then lexicographic in
    (n_1..n_L)."""
    d = nph + 1
    b = np.diag(np.sqrt(np.arange(1, d)), 1)  # annihilation on one mode
    I = np.eye(d)

    def site_op(op, j):
        mats = [I] * L
        mats[j] = op
        out = np.array([[1.0]])
        for m in mats:
            out = np.kron(out, m)
        return out

    dim_ph = d ** L
    Hph = np.zeros((dim_ph, dim_ph))
    for j in range(L):
        Hph += w0 * site_op(b.T @ b, j)
    He = np.zeros((L, L))
    for i in range(L):
        He[i, i] = Delta[i]
        j = i + 1
        if periodic:
            j %= L
        if j < L:
            He[i, j] += -t
            He[j, i] += -t
    H = np.kron(np.eye(dim_ph), He) + np.kron(Hph, np.eye(L))
    for i in range(L):
        ni = np.zeros((L, L))
        ni[i, i] = 1.0
        H += np.kron(-g[i] * w0 * site_op(b + b.T, i), ni)
    configs = [c for c in itertools.product(range(d), repeat=L) if sum(c) <= nph]
    configs.sort(key=lambda c: (sum(c), c))
    flat = [np.ravel_multi_index(c, (d,) * L) for c in configs]
    idx = np.array([r * L + i for i in range(L) for r in flat])
    return H[np.ix_(idx, idx)], configs


@pytest.mark.parametrize("L,nph,periodic", [(3, 2, True), (4, 2, False), (2, 3, False), (1, 4, False)])
def test_holstein_builder_matches_tensor_product(L, nph, periodic):
    rng = np.random.default_rng(L * 10 + nph)
    g = rng.uniform(0.3, 1.5, L)
    Delta = rng.uniform(-1, 1, L)
    ref, configs = _holstein_kron(L, nph, 1.0, 1.3, g, Delta, periodic)
    Hm = O.holstein(L, nph, 1.0, 1.3, g, Delta, periodic)
    np.testing.assert_allclose(Hm.dense(), ref, rtol=0, atol=1e-14)
    np.testing.assert_array_equal(O.holstein_occupations(L, nph), np.array(configs, dtype=np.uint8))
    assert Hm.n == L * math.comb(L + nph, nph)


def test_holstein_dimension_matches_paper(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "paper_values.json")))["polaron"]
    D = g["L"] * math.comb(g["L"] + g["nph"], g["nph"])
    assert float(f"{D:.{g['significant_digits']}g}") == g["D_tot"]
    assert O.holstein_nconf(10, 10) * 10 == 1_847_560


def test_gershgorin_encloses_spectrum():
    rng = np.random.default_rng(3)
    for H in [O.chain1d(rng.uniform(0, 5, 50), 0.3),
              O.honeycomb(4, 9, rng.uniform(-1, 1, 36)),
              O.holstein(3, 3, 1.0, 1.0, [0.7, 0.7, 0.7], [0, 0.5, 0], True)]:
        lo, hi = H.gershgorin()
        Hd = H.dense()
        E = np.linalg.eigvalsh(Hd)
        assert lo <= E[0] + 1e-12 and E[-1] <= hi + 1e-12
        # brute-force disc bounds
        r = np.abs(Hd).sum(axis=1) - np.abs(np.diag(Hd))
        assert lo == pytest.approx(np.min(np.diag(Hd).real - r), abs=1e-12)
        assert hi == pytest.approx(np.max(np.diag(Hd).real + r), abs=1e-12)


# ---------------------------------------------------------------------------
# Whole propagation against exact diagonalisation and closed forms
# ---------------------------------------------------------------------------
def _plan(H, dt, **kw):
    lo, hi = H.gershgorin()
    return O.Plan(lo, hi, dt, **kw)


def test_paper_double_well_against_ed(golden_dir):
    # Sect. 3.1 worked example: N = 2048, t = 40, dt = 0.4, error < 2e-11
    g = json.load(open(os.path.join(golden_dir, "paper_values.json")))["double_well"]
    x, dx = W.chain_grid(g["N"], -20.0, 20.0)
    V = W.paper_double_well(x, g["omega0"], g["a"], g["V0"], g["m"])
    assert np.allclose(V, 0.0016 * (x * x - 25.0) ** 2, atol=1e-12)
    psi0 = W.gaussian_1d(x, g["q0"], g["sigma"], g["p0"])
    H = O.chain1d(V, dx)
    P = _plan(H, g["dt"])
    steps = int(round(g["t_final"] / g["dt"]))
    psi = O.propagate(H, P, psi0, steps)
    ref = ed_propagate(H.dense().real, psi0, g["t_final"])
    assert np.abs(psi.real - ref.real).max() < g["chebyshev_abs_error_bound"]
    assert np.abs(psi.imag - ref.imag).max() < g["chebyshev_abs_error_bound"]
    # a sizeable fraction tunnels through the barrier (Sect. 3.1)
    assert 0.01 < np.sum(np.abs(ref[x > 0]) ** 2) < 0.5


def test_free_particle_closed_form():
    # V = 0 on the Dirichlet grid: psi(t) = S diag(exp(-i E_m t)) S psi0 with the
    # DST-I eigenvectors S_jm = sqrt(2/(n+1)) sin(pi j m/(n+1)).
    n = 256
    x, dx = W.chain_grid(n, -12.0, 12.0)
    psi0 = W.gaussian_1d(x, -3.0, 1.0, 1.5)
    H = O.chain1d(np.zeros(n), dx)
    P = _plan(H, 0.25)
    psi = O.propagate(H, P, psi0, 12)
    j = np.arange(1, n + 1)
    S = np.sqrt(2.0 / (n + 1)) * np.sin(np.pi * np.outer(j, j) / (n + 1))
    E = (1.0 - np.cos(np.pi * j / (n + 1))) / dx ** 2
    ref = S @ (np.exp(-1j * E * 3.0) * (S @ psi0))
    assert rel_l2(psi, ref) < 1e-12


def test_free_gaussian_spreading_continuum_limit():
    # |psi|^2 of a free packet: centre x0 + k0 t, variance sigma^2 + (t/(2 sigma))^2
    n = 4096
    x, dx = W.chain_grid(n, -40.0, 40.0)
    sigma, x0, k0, T = 1.0, -5.0, 1.0, 6.0
    psi0 = W.gaussian_1d(x, x0, sigma, k0)
    H = O.chain1d(np.zeros(n), dx)
    P = _plan(H, 1.0)
    rho = np.abs(O.propagate(H, P, psi0, int(T))) ** 2
    mean = np.sum(x * rho)
    var = np.sum((x - mean) ** 2 * rho)
    # lattice dispersion shifts the group velocity by O(k0^2 dx^2)
    assert mean == pytest.approx(x0 + k0 * T, abs=5e-3)
    assert var == pytest.approx(sigma ** 2 + (T / (2 * sigma)) ** 2, rel=5e-3)


def test_harmonic_oscillator_coherent_state():
    # <x>(t) = x0 cos(w t) + (p0/w) sin(w t); after one period psi -> -psi.
    # The finite-difference grid adds O(dx^2) errors: check their size and
    # that halving dx cuts them by four.
    w, x0, p0 = 1.0, 2.0, 0.5

    def errors(n):
        x, dx = W.chain_grid(n, -16.0, 16.0)
        psi0 = W.gaussian_1d(x, x0, 1.0 / math.sqrt(2.0 * w), p0)
        H = O.chain1d(W.harmonic(x, w), dx)
        steps = 40
        P = _plan(H, 2.0 * math.pi / w / steps)
        psi, err = psi0.copy(), 0.0
        for s in range(1, steps + 1):
            psi = O.propagate(H, P, psi, 1)
            if s % 5 == 0:
                t = s * P.dt
                mean = np.sum(x * np.abs(psi) ** 2)
                err = max(err, abs(mean - (x0 * math.cos(w * t) + p0 / w * math.sin(w * t))))
        return err, rel_l2(psi, -psi0)

    e1, r1 = errors(1024)
    e2, r2 = errors(2048)
    assert e2 < 1e-3 and r2 < 5e-3
    assert 3.5 < e1 / e2 < 4.5 and 3.5 < r1 / r2 < 4.5


@pytest.mark.parametrize("case", ["chain", "zigzag", "armchair", "holstein_ring", "holstein_open"])
def test_propagation_against_ed(case):
    rng = np.random.default_rng(11)
    if case == "chain":
        x, dx = W.chain_grid(300, -8.0, 8.0)
        H = O.chain1d(W.quartic_well(x, 0.05, 3.0), dx)
        psi0 = W.gaussian_1d(x, -3.0, 0.7, 1.0)
        dt, K = 0.05, 20
    elif case in ("zigzag", "armchair"):
        w, l = 6, 16
        H = O.honeycomb(w, l, W.anderson_disorder(w, l, 1.0, 5), edge=case)
        psi0 = W.gaussian_ribbon(w, l, 4.0, 2.5, 2.0, 1.0)
        dt, K = 1.0, 15
    else:
        L, nph = 4, 3
        H = O.holstein(L, nph, 1.0, 1.0, math.sqrt(0.5), rng.uniform(-0.5, 0.5, L),
                       case == "holstein_ring")
        psi0 = W.holstein_packet(L, O.holstein_nconf(L, nph), 1.0, 0.8, 0.6)
        dt, K = 0.1, 30
    P = _plan(H, dt)
    psi, nrm, en = O.propagate(H, P, psi0, K, want_obs=True)
    Hd = H.dense()
    ref = ed_propagate(Hd, psi0, dt * K)
    assert rel_l2(psi, ref) < 1e-11
    # norm and energy of each step's input state are conserved
    assert np.abs(nrm - 1.0).max() < 1e-12
    E0 = np.vdot(psi0, Hd @ psi0).real
    assert np.abs(en - E0).max() < 1e-12 * max(1.0, abs(P.a))


def test_norm_energy_conservation_long_run():
    w, l = 16, 64
    H = O.honeycomb(w, l, W.anderson_disorder(w, l, 0.5, 0))
    psi0 = W.ribbon_packet(w, l, 4.0, 1.0)
    P = _plan(H, 1.0)
    assert P.M == 20 or P.M == 19 or P.M == 21
    _, nrm, en = O.propagate(H, P, psi0, 400, want_obs=True)
    assert np.abs(nrm - 1.0).max() < 1e-12
    assert np.abs(en - en[0]).max() < 1e-12


def test_zero_and_one_order_steps():
    # M = 0: psi <- gamma_0 psi;  M = 1: psi <- gamma_0 psi + gamma_1 H~ psi
    rng = np.random.default_rng(2)
    H = O.chain1d(rng.uniform(0, 1, 40), 0.5)
    lo, hi = H.gershgorin()
    psi0 = rng.normal(size=40) + 1j * rng.normal(size=40)
    for M in (0, 1, 2):
        P = O.Plan(lo, hi, 1e-3, M=M)
        out = O.propagate(H, P, psi0, 1)
        Ht = (H.dense() - P.b * np.eye(40)) / P.a
        ref = P.gamma[0] * psi0
        if M >= 1:
            ref = ref + P.gamma[1] * (Ht @ psi0)
        if M >= 2:
            ref = ref + P.gamma[2] * (2 * Ht @ Ht @ psi0 - psi0)
        np.testing.assert_allclose(out, ref, rtol=1e-14, atol=1e-14)


# ---------------------------------------------------------------------------
# Holstein special cases and observables (Sect. 3.3, Fig. 3)
# ---------------------------------------------------------------------------
def test_independent_boson_site():
    # t = 0 single site: <b+b>(t) = 2 g^2 (1 - cos w0 t), <b+b^+>(t) = 2 g (1 - cos w0 t)
    g2, w0, nph = 0.5, 1.0, 30
    g = math.sqrt(g2)
    H = O.holstein(1, nph, 0.0, w0, g, 0.0, False)
    psi = W.holstein_vacuum_site(1, 0, O.holstein_nconf(1, nph))
    P = _plan(H, 0.1)
    for s in range(1, 31):
        psi = O.propagate(H, P, psi, 1)
        if s % 5 == 0:
            t = 0.1 * s
            n_i, nph_i, chi = O.holstein_obs(1, nph, psi)
            assert n_i[0] == pytest.approx(1.0, abs=1e-13)
            assert nph_i[0] == pytest.approx(2 * g2 * (1 - math.cos(w0 * t)), abs=1e-11)
            assert chi[0] == pytest.approx(2 * g * (1 - math.cos(w0 * t)), abs=1e-11)


def test_free_ring_without_coupling():
    # g = 0, no phonons: electron on a ring, eigenvalues -2 t cos(2 pi k/L)
    L = 7
    H = O.holstein(L, 0, 1.0, 1.0, 0.0, 0.0, True)
    E = np.linalg.eigvalsh(H.dense())
    ref = np.sort(-2.0 * np.cos(2 * np.pi * np.arange(L) / L))
    np.testing.assert_allclose(E, ref, atol=1e-13)
    psi0 = W.single_site(L, 0)
    psi = O.propagate(H, _plan(H, 0.5), psi0, 6)
    # amplitude on site j: (1/L) sum_k exp(i 2 pi k j/L) exp(2 i t cos(2 pi k/L))
    k = np.arange(L)
    ref_psi = np.array([np.mean(np.exp(2j * np.pi * k * j / L) *
                                np.exp(2j * 3.0 * np.cos(2 * np.pi * k / L))) for j in range(L)])
    assert rel_l2(psi, ref_psi) < 1e-12


def test_holstein_observables_brute_force():
    L, nph = 3, 2
    rng = np.random.default_rng(5)
    occ = O.holstein_occupations(L, nph)
    dim = occ.shape[0] * L
    psi = rng.normal(size=dim) + 1j * rng.normal(size=dim)
    n_i, nph_i, chi = O.holstein_obs(L, nph, psi)
    ref, configs = _holstein_kron(L, nph, 0.0, 1.0, np.zeros(L), np.zeros(L), False)
    # explicit operators in the truncated tensor-product basis
    d = nph + 1
    b = np.diag(np.sqrt(np.arange(1, d)), 1)
    flat = [np.ravel_multi_index(c, (d,) * L) for c in configs]
    idx = np.array([r * L + i for i in range(L) for r in flat])
    for i in range(L):
        ni = np.zeros((L, L))
        ni[i, i] = 1.0
        mats = [np.eye(d)] * L
        mats_b = list(mats)
        mats_b[i] = b + b.T
        mats_n = list(mats)
        mats_n[i] = b.T @ b
        def kron_all(ms):
            out = np.array([[1.0]])
            for m in ms:
                out = np.kron(out, m)
            return out
        Nop = np.kron(np.eye(d ** L), ni)[np.ix_(idx, idx)]
        Bop = np.kron(kron_all(mats_n), np.eye(L))[np.ix_(idx, idx)]
        Xop = np.kron(kron_all(mats_b), ni)[np.ix_(idx, idx)]
        assert n_i[i] == pytest.approx(np.vdot(psi, Nop @ psi).real, rel=1e-13)
        assert nph_i[i] == pytest.approx(np.vdot(psi, Bop @ psi).real, rel=1e-13)
        # the truncated (b + b^+) keeps only in-basis transitions
        assert chi[i] == pytest.approx(np.vdot(psi, Xop @ psi).real, rel=1e-12, abs=1e-12)


def test_density_and_region_sum():
    rng = np.random.default_rng(1)
    psi = rng.normal(size=100) + 1j * rng.normal(size=100)
    rho = O.density(psi)
    np.testing.assert_allclose(rho, np.abs(psi) ** 2, rtol=1e-15)
    mask = (np.arange(100) > 40).astype(np.uint8)
    assert O.region_sum(psi, mask) == pytest.approx(np.sum(np.abs(psi[41:]) ** 2), rel=1e-14)


# ---------------------------------------------------------------------------
# Crank-Nicolson, eq. (CN)
# ---------------------------------------------------------------------------
def test_crank_nicolson_second_order():
    x, dx = W.chain_grid(200, -8.0, 8.0)
    V = W.quartic_well(x, 0.05, 3.0)
    psi0 = W.gaussian_1d(x, -3.0, 0.7, 1.0)
    H = O.chain1d(V, dx)
    T = 0.5
    ref = ed_propagate(H.dense().real, psi0, T)
    errs = []
    for S in (50, 100, 200):
        psi = O.crank_nicolson_1d(V, dx, psi0, T / S, S)
        errs.append(np.linalg.norm(psi - ref))
        assert abs(np.linalg.norm(psi) - 1.0) < 1e-12  # CN is unitary
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(order - 2.0) < 0.1)


# ---------------------------------------------------------------------------
# Reverse mode (dL/dV for L = sum mask |psi_K|^2)
# ---------------------------------------------------------------------------
def _chain_case(n=48, seed=4):
    rng = np.random.default_rng(seed)
    x, dx = W.chain_grid(n, -6.0, 6.0)
    V = W.quartic_well(x, 0.05, 2.0) + rng.uniform(0, 0.2, n)
    psi0 = W.gaussian_1d(x, -1.5, 0.8, 1.2)
    mask = (x > 0).astype(np.float64)
    return V, dx, psi0, mask


def test_adjoint_matches_dense_autograd():
    torch = pytest.importorskip("torch")
    V, dx, psi0, mask = _chain_case()
    n = V.size
    H = O.chain1d(V, dx)
    lo, hi = H.gershgorin()
    dt, K = 0.2, 5
    P = O.Plan(lo, hi, dt)
    L, g, _ = O.adjoint(H, P, psi0, K, mask)
    Vt = torch.tensor(V, dtype=torch.float64, requires_grad=True)
    T = torch.zeros(n, n, dtype=torch.float64)
    idx = torch.arange(n - 1)
    T[idx, idx + 1] = -0.5 / dx ** 2
    T[idx + 1, idx] = -0.5 / dx ** 2
    Hm = T + torch.diag(Vt + 1.0 / dx ** 2)
    U = torch.linalg.matrix_exp(-1j * dt * Hm.to(torch.complex128))
    psi = torch.tensor(psi0)
    for _ in range(K):
        psi = U @ psi
    Lt = (torch.tensor(mask) * psi.abs() ** 2).sum()
    Lt.backward()
    assert L == pytest.approx(Lt.item(), rel=1e-12)
    np.testing.assert_allclose(g, Vt.grad.numpy(), rtol=0, atol=1e-11 * np.abs(g).max())


def test_adjoint_central_differences():
    V, dx, psi0, mask = _chain_case(n=64, seed=9)
    H = O.chain1d(V, dx)
    lo, hi = H.gershgorin()
    dt, K, h = 0.3, 4, 1e-6
    P = O.Plan(lo, hi, dt)
    _, g, _ = O.adjoint(H, P, psi0, K, mask)
    for i in [3, 17, 30, 41, 60]:
        Vp, Vm = V.copy(), V.copy()
        Vp[i] += h
        Vm[i] -= h
        Lp = np.sum(mask * np.abs(O.propagate(O.chain1d(Vp, dx), P, psi0, K)) ** 2)
        Lm = np.sum(mask * np.abs(O.propagate(O.chain1d(Vm, dx), P, psi0, K)) ** 2)
        assert g[i] == pytest.approx((Lp - Lm) / (2 * h), abs=1e-8)


def test_adjoint_of_state_is_inverse_propagator():
    # one step: u_0 = p(H~)^H gbar ~ exp(+i H dt) gbar for gbar = 2 mask psi_1
    V, dx, psi0, mask = _chain_case(n=40, seed=2)
    H = O.chain1d(V, dx)
    lo, hi = H.gershgorin()
    P = O.Plan(lo, hi, 0.4)
    _, _, u0 = O.adjoint(H, P, psi0, 1, mask)
    psi1 = O.propagate(H, P, psi0, 1)
    E, U = np.linalg.eigh(H.dense().real)
    ref = U @ (np.exp(1j * E * 0.4) * (U.T @ (2 * mask * psi1)))
    assert rel_l2(u0, ref) < 1e-12


def test_adjoint_honeycomb_central_differences():
    w, l = 5, 10
    eps = W.anderson_disorder(w, l, 0.5, 3)
    psi0 = W.gaussian_ribbon(w, l, 2.5, 2.0, 1.5, 1.0)
    mask = W.right_half_mask_ribbon(w, l)
    H = O.honeycomb(w, l, eps)
    lo, hi = H.gershgorin()
    P = O.Plan(lo, hi, 2.0)
    K, h = 3, 1e-6
    _, g, _ = O.adjoint(H, P, psi0, K, mask)
    for i in [0, 7, 23, 38, 49]:
        ep, em = eps.copy(), eps.copy()
        ep[i] += h
        em[i] -= h
        Lp = np.sum(mask * np.abs(O.propagate(O.honeycomb(w, l, ep), P, psi0, K)) ** 2)
        Lm = np.sum(mask * np.abs(O.propagate(O.honeycomb(w, l, em), P, psi0, K)) ** 2)
        assert g[i] == pytest.approx((Lp - Lm) / (2 * h), abs=1e-8)


# ---------------------------------------------------------------------------
# Time-dependent H(t) held constant within each step (Sect. 2.2, last paragraph)
# ---------------------------------------------------------------------------
def _td_oracle(V_of_step, dx, psi0, plan, K):
    psi = psi0.copy()
    for s in range(K):
        psi = O.propagate(O.chain1d(V_of_step(s), dx), plan, psi, 1)
    return psi


def test_time_dependent_uniform_shift_is_a_global_phase():
    # V(x, t) = V0(x) + f0 + f1 t: the shift only multiplies psi by
    # exp(-i int f dt); mid-step values make the sum exact for linear f
    x, dx = W.chain_grid(200, -8.0, 8.0)
    V0 = W.quartic_well(x, 0.05, 3.0)
    psi0 = W.gaussian_1d(x, -3.0, 0.7, 1.0)
    f0, f1, dt, K = 0.3, 0.8, 0.05, 24
    H0 = O.chain1d(V0, dx)
    lo, hi = H0.gershgorin()
    plan = O.Plan(lo - 1.0, hi + f0 + f1 * dt * K + 1.0, dt)
    psi = _td_oracle(lambda s: V0 + f0 + f1 * (s + 0.5) * dt, dx, psi0, plan, K)
    T = dt * K
    ref = np.exp(-1j * (f0 * T + 0.5 * f1 * T * T)) * O.propagate(H0, plan, psi0, K)
    assert rel_l2(psi, ref) < 1e-12


def test_time_dependent_midpoint_is_second_order():
    # driven particle V(x, t) = V0(x) + E sin(w t) x: error vs a fine-step run
    x, dx = W.chain_grid(160, -8.0, 8.0)
    V0 = W.harmonic(x, 0.5)
    psi0 = W.gaussian_1d(x, -1.0, 1.0, 0.5)
    E, w, T = 0.4, 1.3, 2.0
    lo, hi = O.chain1d(V0, dx).gershgorin()
    bound = E * np.abs(x).max()

    def run(K):
        dt = T / K
        plan = O.Plan(lo - bound, hi + bound, dt)
        return _td_oracle(lambda s: V0 + E * np.sin(w * (s + 0.5) * dt) * x, dx, psi0, plan, K)

    ref = run(512)
    errs = [np.linalg.norm(run(K) - ref) for K in (16, 32, 64)]
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(order - 2.0) < 0.15)
