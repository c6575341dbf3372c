"""Time-dependent H(t) held constant within each step: the GPU path
(chebtd_propagate_td) against the oracle stepping with the same per-step
Hamiltonians, for the chain, a ribbon and the Holstein model."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from test_gpu_parity import assert_state_close

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("state", ["packet", "dense"])
@pytest.mark.parametrize("n", [300, 5003])
def test_chain_driven(torch, cheb, n, state):
    x, dx = W.chain_grid(n, -8.0, 8.0)
    V0 = W.quartic_well(x, 0.05, 3.0)
    psi0 = W.gaussian_1d(x, -3.0, 0.7, 1.0) if state == "packet" else W.random_state(n, 90 + n)
    E, w, dt, K = 0.5, 2.0, 0.01, 9
    sched = np.stack([V0 + E * np.sin(w * (s + 0.5) * dt) * x for s in range(K)])
    lo, hi = O.chain1d(V0, dx).gershgorin()
    b = E * np.abs(x).max()
    plan = O.Plan(lo - b, hi + b, dt)
    ref = psi0.copy()
    for s in range(K):
        ref = O.propagate(O.chain1d(sched[s], dx), plan, ref, 1)
    ctx = cheb.Context()
    V_d = torch.from_numpy(V0).cuda()
    ctx.chain1d(V_d, dx)
    ctx.set_bounds(lo - b, hi + b)
    assert ctx.plan(dt) == plan.M
    psi = torch.from_numpy(psi0.copy()).cuda()
    ctx.propagate_td(psi, torch.from_numpy(sched).cuda())
    torch.cuda.synchronize()
    assert_state_close(psi.cpu().numpy(), ref)
    # the built Hamiltonian is restored: a plain step uses V0 again
    p2 = torch.from_numpy(psi0.copy()).cuda()
    ctx.propagate(p2, 2)
    torch.cuda.synchronize()
    assert rel_l2(p2.cpu().numpy(), O.propagate(O.chain1d(V0, dx), plan, psi0, 2)) <= 1e-10


@pytest.mark.parametrize("state", ["packet", "dense"])
def test_ribbon_ramped_disorder(torch, cheb, state):
    w, l, K, dt = 12, 333, 7, 1.0
    eps0, psi0 = W.ribbon_inputs(w, l, 0.5, 3)
    if state == "dense":
        psi0 = W.random_state(w * l, 93)
    sched = np.stack([eps0 * (1.0 + 0.1 * s) + 0.05 * s for s in range(K)])
    lo = min(O.honeycomb(w, l, e).gershgorin()[0] for e in sched)
    hi = max(O.honeycomb(w, l, e).gershgorin()[1] for e in sched)
    plan = O.Plan(lo, hi, dt)
    ref = psi0.copy()
    for s in range(K):
        ref = O.propagate(O.honeycomb(w, l, sched[s]), plan, ref, 1)
    ctx = cheb.Context()
    e_d = torch.from_numpy(eps0).cuda()
    ctx.honeycomb(w, l, e_d)
    ctx.set_bounds(lo, hi)
    ctx.plan(dt)
    psi = torch.from_numpy(psi0.copy()).cuda()
    nrm = torch.zeros(K, dtype=torch.float64, device="cuda")
    en = torch.zeros(K, dtype=torch.float64, device="cuda")
    ctx.propagate_td(psi, torch.from_numpy(sched).cuda(), nrm, en)
    torch.cuda.synchronize()
    assert_state_close(psi.cpu().numpy(), ref)
    # energy of the state entering step s under that step's H
    p = psi0.copy()
    for s in range(K):
        Hs = O.honeycomb(w, l, sched[s])
        _, rn, re = O.propagate(Hs, plan, p, 1, want_obs=True)
        assert en[s].item() == pytest.approx(re[0], rel=1e-11, abs=1e-12)
        p = O.propagate(Hs, plan, p, 1)


@pytest.mark.parametrize("state", ["packet", "dense"])
@pytest.mark.parametrize("rank", ["0", "1"])
def test_holstein_biased_barrier(torch, cheb, monkeypatch, state, rank):
    # rank "1": the walk that forms the phonon partners' ranks itself (its
    # default past 8M states) with the per-step Delta_i; "0": the table walk
    monkeypatch.setenv("CHEBTD_HOL_RANK", rank)
    L, nph, K, dt = 6, 4, 8, 0.2
    g = np.full(L, np.sqrt(0.5))
    D0 = np.zeros(L)
    sched = np.stack([np.linspace(0.0, 0.3 * np.sin(0.7 * (s + 0.5) * dt), L) for s in range(K)])
    lo = min(O.holstein(L, nph, 1.0, 1.0, g, d, False).gershgorin()[0] for d in sched)
    hi = max(O.holstein(L, nph, 1.0, 1.0, g, d, False).gershgorin()[1] for d in sched)
    plan = O.Plan(lo, hi, dt)
    psi0 = W.holstein_packet(L, O.holstein_nconf(L, nph), 2.0, 1.0, 0.4)
    if state == "dense":
        psi0 = W.random_state(psi0.size, 94)
    ref = psi0.copy()
    for s in range(K):
        ref = O.propagate(O.holstein(L, nph, 1.0, 1.0, g, sched[s], False), plan, ref, 1)
    ctx = cheb.Context()
    ctx.holstein(L, nph, 1.0, 1.0, g, D0, False)
    ctx.set_bounds(lo, hi)
    ctx.plan(dt)
    psi = torch.from_numpy(psi0.copy()).cuda()
    ctx.propagate_td(psi, torch.from_numpy(sched).cuda())
    torch.cuda.synchronize()
    assert_state_close(psi.cpu().numpy(), ref)


def test_td_rejects_short_stride_and_checkpoints(torch, cheb):
    ctx = cheb.Context()
    V = torch.zeros(50, dtype=torch.float64, device="cuda")
    ctx.chain1d(V, 0.1)
    ctx.set_bounds(-1.0, 500.0)
    ctx.plan(0.01)
    psi = torch.zeros(50, dtype=torch.complex128, device="cuda")
    with pytest.raises(cheb.ChebError):
        ctx.propagate_td(psi, torch.zeros(3, 49, dtype=torch.float64, device="cuda"))
    with pytest.raises(cheb.ChebError):
        ctx.propagate_td(psi, torch.zeros(3, 50, dtype=torch.float64, device="cuda"),
                         flags=cheb.KEEP_CHECKPOINTS)
