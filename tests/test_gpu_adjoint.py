"""GPU adjoint (dL/dV) against the CPU oracle's reverse mode and against
central finite differences of the GPU forward pass."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from test_gpu_parity import assert_state_close

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available()
    return T


@pytest.fixture(scope="module")
def cheb():
    import paper_0907_3022_amd as P
    P.load_library()
    return P


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def chain_inputs(n, a=0.05, b=5.0, dense=False):
    """dense: a random state and random weights w_i in L = sum w_i |psi_i|^2,
    so that gbar, every adjoint vector and dL/dV are nonzero on every site."""
    x, dx, V, psi0 = W.double_well_inputs(n, -20.0, 20.0, a, b, -5.0, 1.0, 1.0)
    mask = (x > 0).astype(np.float64)
    if dense:
        psi0, mask = W.random_state(n, 500 + n), W.random_weights(n, 600 + n)
    return dx, V, psi0, mask


def ribbon_inputs(width, length, Wd=0.5, seed=0, dense=False):
    eps, psi0 = W.ribbon_inputs(width, length, Wd, seed)
    mask = W.right_half_mask_ribbon(width, length)
    if dense:
        n = width * length
        psi0, mask = W.random_state(n, 700 + seed), W.random_weights(n, 800 + seed)
    return eps, psi0, mask


def assert_grad_close(g, gr, tol=1e-8):
    """rel-L2 <= tol and every site within tol * max|gr|."""
    assert rel_l2(g, gr) <= tol
    assert np.abs(g - gr).max() <= tol * np.abs(gr).max()


def gpu_adjoint(torch, cheb, kind, geom, V, psi0, mask, bounds, dt, K, mode):
    prop = cheb.Propagator(kind, dt, K, bounds, adjoint_mode=mode, **geom)
    Vt = torch.from_numpy(V.copy()).cuda().requires_grad_(True)
    p0 = torch.from_numpy(psi0.copy()).cuda().requires_grad_(True)
    say(f"[gpu] adjoint {kind} n={V.size} K={K} mode={mode}")
    psi = cheb.ChebPropagate.apply(Vt, p0, prop)
    m = torch.from_numpy(mask).cuda()
    L = (m * psi.abs() ** 2).sum()
    L.backward()
    torch.cuda.synchronize()
    return float(L.item()), Vt.grad.cpu().numpy(), p0.grad.cpu().numpy(), prop


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("case", ["chain", "zigzag", "armchair", "chain_large"])
@pytest.mark.parametrize("dense", [False, True])
def test_adjoint_matches_oracle(torch, cheb, case, mode, dense):
    if case.startswith("chain"):
        n = 300 if case == "chain" else 9001
        dx, V, psi0, mask = chain_inputs(n, dense=dense)
        H = O.chain1d(V, dx)
        geom = dict(dx=dx)
        kind = "chain"
        lo, hi = H.gershgorin()
        dt = 30.0 / (0.5 * 1.01 * (hi - lo))   # order ~ 64
    else:
        w, l = 8, 60
        V, psi0, mask = ribbon_inputs(w, l, dense=dense)
        H = O.honeycomb(w, l, V, edge=case)
        geom = dict(width=w, length=l, edge=case)
        kind = "honeycomb"
        lo, hi = H.gershgorin()
        dt = 2.5
    K = 4
    Lg, g, u0, prop = gpu_adjoint(torch, cheb, kind, geom, V, psi0, mask, (lo, hi), dt, K, mode)
    plan = O.Plan(lo, hi, dt)
    assert prop.M == plan.M
    Lr, gr, ur = O.adjoint(H, plan, psi0, K, mask)
    assert Lg == pytest.approx(Lr, rel=1e-10)
    assert_grad_close(g, gr)
    assert_state_close(u0, ur)


# degenerate lattices: one site (bounds widened around its one eigenvalue),
# two and three chain sites, single rows and columns of a ribbon, a 2 x 2 cell
@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("kind,size", [("chain", 1), ("chain", 2), ("chain", 3), ("honeycomb", (1, 1)),
                                       ("honeycomb", (1, 5)), ("honeycomb", (5, 1)), ("honeycomb", (2, 2))])
def test_adjoint_degenerate_lattices_match_oracle(torch, cheb, kind, size, mode):
    if kind == "chain":
        n, dx = size, 1.0
        V = W.uniform01(900 + n, n) - 0.5
        H = O.chain1d(V, dx)
        geom = dict(dx=dx)
    else:
        w, l = size
        n = w * l
        V = W.anderson_disorder(w, l, 0.5, 9)
        H = O.honeycomb(w, l, V, edge="zigzag")
        geom = dict(width=w, length=l, edge="zigzag")
    psi0, mask = W.random_state(n, 950 + n), W.random_weights(n, 960 + n)
    lo, hi = H.gershgorin()
    if hi == lo:
        lo, hi = lo - 1.0, hi + 1.0
    dt, K = 2.0, 3
    Lg, g, u0, prop = gpu_adjoint(torch, cheb, kind, geom, V, psi0, mask, (lo, hi), dt, K, mode)
    plan = O.Plan(lo, hi, dt)
    assert prop.M == plan.M
    Lr, gr, ur = O.adjoint(H, plan, psi0, K, mask)
    assert Lg == pytest.approx(Lr, rel=1e-10)
    if n == 1:  # |psi|^2 of one site does not depend on V: dL/dV is zero up to rounding
        assert abs(g).max() <= 1e-13 and abs(gr).max() <= 1e-13
    else:
        assert_grad_close(g, gr)
    assert_state_close(u0, ur)


# z = a dt from 1e-9 to 0.3 gives M = 1, 2, 3, 4, 5, 6, 10: the reverse sweep
# pairs levels two by two where it can and leaves single levels (odd counts,
# level 0, the level next to u_M) to the one-level kernel; the downward
# schedule (mode 2) splits the M levels into passes of 2 .. 5 ending at level 0
@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("case", ["chain", "zigzag", "armchair"])
@pytest.mark.parametrize("z", [1e-9, 1e-7, 3e-4, 1e-3, 0.01, 0.02, 0.3])
def test_adjoint_low_orders(torch, cheb, case, mode, z):
    if case == "chain":
        dx, V, psi0, mask = chain_inputs(257)
        H = O.chain1d(V, dx)
        geom, kind = dict(dx=dx), "chain"
    else:
        V, psi0, mask = ribbon_inputs(9, 70)
        H = O.honeycomb(9, 70, V, edge=case)
        geom, kind = dict(width=9, length=70, edge=case), "honeycomb"
    lo, hi = H.gershgorin()
    dt = z / (0.5 * 1.01 * (hi - lo))
    K = 3
    Lg, g, u0, prop = gpu_adjoint(torch, cheb, kind, geom, V, psi0, mask, (lo, hi), dt, K, mode)
    plan = O.Plan(lo, hi, dt)
    assert prop.M == plan.M
    Lr, gr, ur = O.adjoint(H, plan, psi0, K, mask)
    assert Lg == pytest.approx(Lr, rel=1e-10)
    # at tiny dt dL/dV is O(dt^2) while its terms are O(1): both sides carry
    # rounding noise of ~1e-16 per term, hence the absolute floor
    assert np.linalg.norm(g - gr) <= 1e-8 * np.linalg.norm(gr) + 1e-12
    assert rel_l2(u0, ur) <= 1e-10


def test_adjoint_modes_agree(torch, cheb):
    # the two memory schedules group the levels into passes differently (the
    # segment schedule cannot run deep passes across segment boundaries), so
    # they agree to rounding
    w, l = 16, 200
    V, psi0, mask = ribbon_inputs(w, l)
    H = O.honeycomb(w, l, V)
    b = H.gershgorin()
    _, g0, u0, _ = gpu_adjoint(torch, cheb, "honeycomb", dict(width=w, length=l), V, psi0, mask, b, 9.4, 3, 0)
    _, g1, u1, _ = gpu_adjoint(torch, cheb, "honeycomb", dict(width=w, length=l), V, psi0, mask, b, 9.4, 3, 1)
    assert rel_l2(g0, g1) <= 1e-12
    assert rel_l2(u0, u1) <= 1e-13
    # the downward schedule regenerates the forward vectors by the recursion
    # run backwards: equal to rounding as well
    _, g2, u2, _ = gpu_adjoint(torch, cheb, "honeycomb", dict(width=w, length=l), V, psi0, mask, b, 9.4, 3, 2)
    assert rel_l2(g2, g0) <= 1e-12
    assert rel_l2(u2, u0) <= 1e-13


# the downward schedule at every pass depth and at chunk heights that put
# chunk boundaries at every offset of the 6-iteration body; 37 x 130 has
# chunks and strips clear of the border
# (a chain is one row: no chunk heights to force)
@pytest.mark.parametrize("case,rows", [("chain", None)] + [(c, r) for c in ("zigzag", "armchair")
                                                           for r in (None, 1, 5, 16)])
@pytest.mark.parametrize("rev_depth", [2, 3, 4, 5])
def test_adjoint_reverse_depths_match_oracle(torch, cheb, monkeypatch, rev_depth, case, rows):
    monkeypatch.setenv("CHEBTD_REV_DEPTH", str(rev_depth))
    if rows is not None:
        monkeypatch.setenv("CHEBTD_REV_ROWS", str(rows))
    if case == "chain":
        dx, V, psi0, mask = chain_inputs(5003, dense=True)
        H = O.chain1d(V, dx)
        geom, kind = dict(dx=dx), "chain"
        lo, hi = H.gershgorin()
        dt = 12.0 / (0.5 * 1.01 * (hi - lo))
    else:
        w, l = 37, 130
        V, psi0, mask = ribbon_inputs(w, l, dense=True)
        H = O.honeycomb(w, l, V, edge=case)
        geom, kind = dict(width=w, length=l, edge=case), "honeycomb"
        lo, hi = H.gershgorin()
        dt = 1.37
    K = 2
    Lg, g, u0, prop = gpu_adjoint(torch, cheb, kind, geom, V, psi0, mask, (lo, hi), dt, K, 2)
    plan = O.Plan(lo, hi, dt)
    assert prop.M == plan.M and plan.M >= 14
    Lr, gr, ur = O.adjoint(H, plan, psi0, K, mask)
    assert Lg == pytest.approx(Lr, rel=1e-10)
    assert_grad_close(g, gr)
    assert_state_close(u0, ur)


# the forward run keeps each step's (v_{M-1}, v_M) for the downward schedule:
# written by the step's last multi-order pass, or copied after a last single
# order or the one-order-per-pass path
@pytest.mark.parametrize("single", [False, True])
@pytest.mark.parametrize("case", ["chain", "zigzag"])
@pytest.mark.parametrize("z", [0.02, 1.0, 7.0])
def test_adjoint_reverse_step_ends(torch, cheb, case, single, z):
    if case == "chain":
        dx, V, psi0, mask = chain_inputs(257)
        H = O.chain1d(V, dx)
    else:
        V, psi0, mask = ribbon_inputs(9, 70)
        H = O.honeycomb(9, 70, V)
    lo, hi = H.gershgorin()
    dt = z / (0.5 * 1.01 * (hi - lo))
    K = 3
    ctx = cheb.Context()
    Vd = torch.from_numpy(V.copy()).cuda()
    if case == "chain":
        ctx.chain1d(Vd, dx)
    else:
        ctx.honeycomb(9, 70, Vd)
    ctx.set_bounds(lo, hi)
    M = ctx.plan(dt)
    ctx.reserve_adjoint(K, cheb.ADJ_REVERSE)
    say(f"[gpu] reverse step ends {case} M={M} passes={ctx.plan_passes()} single={single}")
    psi = torch.from_numpy(psi0.copy()).cuda()
    flags = cheb.NO_CHECK | cheb.KEEP_CHECKPOINTS | (cheb.SINGLE_ORDER if single else 0)
    ctx.propagate(psi, K, None, None, flags)
    m = torch.from_numpy(mask).cuda()
    gbar = (2.0 * m * psi).contiguous()
    dV = torch.zeros_like(Vd)
    ctx.adjoint(gbar, dV)
    torch.cuda.synchronize()
    plan = O.Plan(lo, hi, dt)
    assert M == plan.M
    Lr, gr, ur = O.adjoint(H, plan, psi0, K, mask)
    assert np.linalg.norm(dV.cpu().numpy() - gr) <= 1e-8 * np.linalg.norm(gr) + 1e-12
    assert rel_l2(gbar.cpu().numpy(), ur) <= 1e-10
    ctx.close()


# D adjoint levels per pass (2 .. 6) with the forward vectors recomputed two
# or six orders per pass; 37 x 130 has chunks and strips clear of the border
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("case", ["chain", "zigzag", "armchair"])
@pytest.mark.parametrize("rec_depth", [2, 6])
@pytest.mark.parametrize("adj_depth", [2, 3, 4, 5, 6])
def test_adjoint_depths_match_oracle(torch, cheb, monkeypatch, adj_depth, rec_depth, case, mode):
    monkeypatch.setenv("CHEBTD_ADJ_DEPTH", str(adj_depth))
    monkeypatch.setenv("CHEBTD_REC_DEPTH", str(rec_depth))
    if case == "chain":
        dx, V, psi0, mask = chain_inputs(5003, dense=True)
        H = O.chain1d(V, dx)
        geom, kind = dict(dx=dx), "chain"
        lo, hi = H.gershgorin()
        dt = 12.0 / (0.5 * 1.01 * (hi - lo))
    else:
        w, l = 37, 130
        V, psi0, mask = ribbon_inputs(w, l, dense=True)
        H = O.honeycomb(w, l, V, edge=case)
        geom, kind = dict(width=w, length=l, edge=case), "honeycomb"
        lo, hi = H.gershgorin()
        dt = 1.37
    K = 2
    Lg, g, u0, prop = gpu_adjoint(torch, cheb, kind, geom, V, psi0, mask, (lo, hi), dt, K, mode)
    plan = O.Plan(lo, hi, dt)
    assert prop.M == plan.M and plan.M >= 14
    Lr, gr, ur = O.adjoint(H, plan, psi0, K, mask)
    assert Lg == pytest.approx(Lr, rel=1e-10)
    assert_grad_close(g, gr)
    assert_state_close(u0, ur)


def _fd_check(torch, cheb, kind, geom, V, psi0, mask, bounds, dt, K, sites, h, rtol_floor):
    Lg, g, _, prop = gpu_adjoint(torch, cheb, kind, geom, V, psi0, mask, bounds, dt, K, None)
    Vd = torch.from_numpy(V.copy()).cuda()
    m = torch.from_numpy(mask).cuda()
    p0 = torch.from_numpy(psi0).cuda()

    def loss(Vx):
        with torch.no_grad():
            psi = prop.forward(Vx, p0, keep=False)
            return float((m * psi.abs() ** 2).sum().item())

    fd = []
    for i in sites:
        Vd[i] += h
        Lp = loss(Vd)
        Vd[i] -= 2 * h
        Lm = loss(Vd)
        Vd[i] += h
        fd.append((Lp - Lm) / (2 * h))
    fd = np.array(fd)
    ga = g[sites]
    say(f"[gpu] FD {kind}: L={Lg:.6e} max|g|={np.abs(g).max():.3e} max|g-fd|={np.abs(ga - fd).max():.3e}")
    assert np.all(np.abs(ga - fd) <= rtol_floor * np.abs(g).max() + 1e-13)
    return g


def test_adjoint_config_ribbon_256x4096_fd(torch, cheb):
    p = W.ADJOINT.params
    w, l = p["width"], p["length"]
    V, psi0, mask = ribbon_inputs(w, l, p["W"], 0)
    ctx = cheb.Context()
    ctx.honeycomb(w, l, torch.from_numpy(V).cuda())
    lo, hi = ctx.gershgorin()
    a = 0.5 * 1.01 * (hi - lo)
    dt = 30.5 / a
    # sites inside the packet's reach
    sites = W.fd_sites(w * l, p["fd_sites"], 77, candidates=np.arange(w * l)[(np.tile(np.arange(l), w) > l // 8)])
    g = _fd_check(torch, cheb, "honeycomb", dict(width=w, length=l), V, psi0, mask, (lo, hi), dt,
                  p["K"], sites, p["h"], 1e-5)
    assert np.abs(g).max() > 0


def test_adjoint_config_chain_65536_fd(torch, cheb):
    p = W.ADJOINT.params
    dx, V, psi0, mask = chain_inputs(p["n1d"])
    ctx = cheb.Context()
    ctx.chain1d(torch.from_numpy(V).cuda(), dx)
    lo, hi = ctx.gershgorin()
    dt = 30.5 / (0.5 * 1.01 * (hi - lo))
    x = np.linspace(-20, 20, p["n1d"])
    sites = W.fd_sites(p["n1d"], p["fd_sites"], 78, candidates=np.nonzero(np.abs(x) < 1.0)[0])
    _fd_check(torch, cheb, "chain", dict(dx=dx), V, psi0, mask, (lo, hi), dt, p["K"], sites, p["h"], 1e-4)


@pytest.mark.parametrize("mode,state", [(0, "packet"), (2, "packet"), (2, "dense"), (1, "dense")])
def test_adjoint_full_size_vs_oracle_short(torch, cheb, mode, state):
    # full 256 x 4096 ribbon, order ~64, 2 steps: GPU reverse sweep vs the oracle's
    p = W.ADJOINT.params
    w, l = p["width"], p["length"]
    if state == "dense":
        V, psi0, mask = ribbon_inputs(w, l, p["W"], 0, dense=True)
    else:
        V, psi0, _ = ribbon_inputs(w, l, p["W"], 0)
        # two steps barely move the packet: weigh the half of it ahead of x0 = l/4
        mask = (np.tile(np.arange(l), w) > l / 4).astype(np.float64)
    H = O.honeycomb(w, l, V)
    lo, hi = H.gershgorin()
    dt = 30.5 / (0.5 * 1.01 * (hi - lo))
    Lg, g, u0, prop = gpu_adjoint(torch, cheb, "honeycomb", dict(width=w, length=l), V, psi0, mask,
                                  (lo, hi), dt, 2, mode)
    plan = O.Plan(lo, hi, dt)
    assert prop.M == plan.M and 60 <= plan.M <= 70
    Lr, gr, ur = O.adjoint(H, plan, psi0, 2, mask)
    assert_grad_close(g, gr)
    assert_state_close(u0, ur)


def test_reverse_schedule_past_offset_limit(torch, cheb):
    # (1 + 14) n 16 B > 2^31 for a 9M-site chain: the downward schedule is
    # refused with CHEBTD_E_ARG, and the autograd wrapper's default falls back
    # to the recompute schedule
    n = 9_000_000
    x, dx = W.chain_grid(n, -0.01 * n, 0.01 * n)
    V = torch.from_numpy(W.harmonic(x, 1e-3)).cuda()
    ctx = cheb.Context()
    ctx.chain1d(V, dx)
    lo, hi = ctx.gershgorin()
    ctx.set_bounds(lo, hi, 0.01)
    ctx.plan(0.002)
    with pytest.raises(cheb.ChebError) as err:
        ctx.reserve_adjoint(2, cheb.ADJ_REVERSE)
    assert err.value.code == -1  # CHEBTD_E_ARG
    ctx.reserve_adjoint(2, cheb.ADJ_STEP)
    ctx.close()
    prop = cheb.Propagator("chain", 0.002, 2, (lo, hi), dx=dx)
    Vt = V.clone().requires_grad_(True)
    p0 = torch.from_numpy(W.gaussian_1d(x, 0.0, 50.0, 0.5)).cuda()
    psi = cheb.ChebPropagate.apply(Vt, p0, prop)
    L = (psi.abs() ** 2 * (torch.from_numpy(x).cuda() > 0)).sum()
    L.backward()
    torch.cuda.synchronize()
    g = Vt.grad.cpu().numpy()
    assert np.all(np.isfinite(g)) and np.abs(g).max() > 0


def test_adjoint_refuses_overwritten_run(torch, cheb):
    # each checkpointing run is numbered; the adjoint of an overwritten run is
    # refused (CHEBTD_E_STATE) and the stored run's adjoint is the oracle's
    w, l = 9, 70
    V, psi0, mask = ribbon_inputs(w, l, dense=True)
    H = O.honeycomb(w, l, V)
    lo, hi = H.gershgorin()
    ctx = cheb.Context()
    Vd = torch.from_numpy(V.copy()).cuda()
    ctx.honeycomb(w, l, Vd)
    ctx.set_bounds(lo, hi)
    ctx.plan(1.3)
    ctx.reserve_adjoint(3, cheb.ADJ_REVERSE)
    assert ctx.checkpoint_run() == 0
    psi_b0 = W.random_state(w * l, 1234)
    runs = []
    for p0 in (psi_b0, psi0):
        psi = torch.from_numpy(p0.copy()).cuda()
        ctx.propagate(psi, 3, flags=cheb.KEEP_CHECKPOINTS)
        runs.append(ctx.checkpoint_run())
    assert 0 < runs[0] < runs[1]
    m = torch.from_numpy(mask).cuda()
    gbar = (2.0 * m * psi).contiguous()
    dV = torch.zeros_like(Vd)
    with pytest.raises(cheb.ChebError) as err:
        ctx.adjoint(gbar.clone(), dV, run=runs[0])
    assert err.value.code == -5  # CHEBTD_E_STATE
    assert float(dV.abs().max()) == 0.0
    ctx.adjoint(gbar, dV, run=runs[1])
    torch.cuda.synchronize()
    _, gr, ur = O.adjoint(H, O.Plan(lo, hi, 1.3), psi0, 3, mask)
    assert_grad_close(dV.cpu().numpy(), gr)
    assert_state_close(gbar.cpu().numpy(), ur)
    # a new plan drops the stored run
    ctx.plan(1.3)
    assert ctx.checkpoint_run() == 0
    ctx.close()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_zero_step_run_replaces_the_stored_run(torch, cheb, mode):
    # a checkpointing run of K = 0 steps is a run of its own: it becomes the
    # stored run (the earlier one's adjoint is refused) and its adjoint is the
    # identity (gbar passes through, dL/dV gains nothing)
    w, l = 9, 70
    V, psi0, _ = ribbon_inputs(w, l, dense=True)
    lo, hi = O.honeycomb(w, l, V).gershgorin()
    ctx = cheb.Context()
    Vd = torch.from_numpy(V.copy()).cuda()
    ctx.honeycomb(w, l, Vd)
    ctx.set_bounds(lo, hi)
    ctx.plan(1.3)
    ctx.reserve_adjoint(3, mode)
    psi = torch.from_numpy(psi0.copy()).cuda()
    ctx.propagate(psi, 3, flags=cheb.KEEP_CHECKPOINTS)
    run3 = ctx.checkpoint_run()
    before = psi.clone()
    ctx.propagate(psi, 0, flags=cheb.KEEP_CHECKPOINTS)
    run0 = ctx.checkpoint_run()
    assert 0 < run3 < run0
    assert torch.equal(psi, before)
    gbar = torch.from_numpy(W.random_state(w * l, 4321)).cuda()
    g0 = gbar.clone()
    dV = torch.full((w * l,), 0.25, dtype=torch.float64, device="cuda")
    with pytest.raises(cheb.ChebError) as err:
        ctx.adjoint(gbar, dV, run=run3)
    assert err.value.code == -5  # CHEBTD_E_STATE
    ctx.adjoint(gbar, dV, run=run0)
    torch.cuda.synchronize()
    assert torch.equal(gbar, g0) and bool((dV == 0.25).all())
    ctx.close()


def test_autograd_zero_steps_is_the_identity(torch, cheb):
    # K = 0: psi_K = psi_0, so dL/dpsi_0 = dL/dpsi_K and dL/dV = 0
    w, l = 9, 70
    V, psi0, mask = ribbon_inputs(w, l, dense=True)
    lo, hi = O.honeycomb(w, l, V).gershgorin()
    L0, g, u0, _ = gpu_adjoint(torch, cheb, "honeycomb", dict(width=w, length=l), V, psi0, mask,
                               (lo, hi), 1.3, 0, None)
    assert L0 == pytest.approx(float((mask * np.abs(psi0) ** 2).sum()), rel=1e-14)
    assert float(np.abs(g).max()) == 0.0
    np.testing.assert_allclose(u0, 2.0 * mask * psi0, rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("mode", [None, 0, 1])
def test_autograd_two_applies_before_backward(torch, cheb, mode):
    # one Propagator applied to two disorder realisations before one backward
    # through their summed loss: each graph node gets the gradient of its own
    # trajectory (the second forward overwrote the first's checkpoints, so the
    # first node's backward runs its forward again)
    w, l = 8, 60
    V1, psi1, mask = ribbon_inputs(w, l, 0.5, 0, dense=True)
    V2 = W.anderson_disorder(w, l, 0.9, 5)
    psi2 = W.random_state(w * l, 55)
    lo = min(V1.min(), V2.min()) - 3.0
    hi = max(V1.max(), V2.max()) + 3.0
    dt, K = 1.7, 3
    prop = cheb.Propagator("honeycomb", dt, K, (lo, hi), width=w, length=l, adjoint_mode=mode)
    m = torch.from_numpy(mask).cuda()
    Vt1 = torch.from_numpy(V1.copy()).cuda().requires_grad_(True)
    Vt2 = torch.from_numpy(V2.copy()).cuda().requires_grad_(True)
    out1 = cheb.ChebPropagate.apply(Vt1, torch.from_numpy(psi1.copy()).cuda(), prop)
    out2 = cheb.ChebPropagate.apply(Vt2, torch.from_numpy(psi2.copy()).cuda(), prop)
    loss = (m * out1.abs() ** 2).sum() + 0.5 * (m * out2.abs() ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    plan = O.Plan(lo, hi, dt)
    _, g1, _ = O.adjoint(O.honeycomb(w, l, V1), plan, psi1, K, mask)
    _, g2, _ = O.adjoint(O.honeycomb(w, l, V2), plan, psi2, K, mask)
    assert_grad_close(Vt1.grad.cpu().numpy(), g1)
    assert_grad_close(Vt2.grad.cpu().numpy(), 0.5 * g2)
