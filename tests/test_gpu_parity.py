"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Every comparison feeds both sides the same seeded inputs (workloads) and the
same spectral bounds (the oracle's Gershgorin discs), then checks the
relative L2 error of psi against 1e-10; integer/structural results must
match exactly and repeated GPU runs must agree bit for bit.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-10


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a visible GPU"
    return T


@pytest.fixture(scope="module")
def cheb():
    import paper_0907_3022_amd as P
    P.load_library()  # fails loudly when the HIP library is missing
    return P


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def assert_state_close(got, ref, tol=TOL):
    """rel-L2 <= tol, and every site within tol * max|ref| (an error where
    the state is small cannot hide in the norm of the whole vector)."""
    got, ref = np.asarray(got), np.asarray(ref)
    err = rel_l2(got, ref)
    assert err <= tol, f"rel-L2 {err:.3e}"
    d = np.abs(got - ref)
    worst = int(np.argmax(d))
    assert d[worst] <= tol * np.abs(ref).max(), \
        f"site {worst}: |diff| {d[worst]:.3e} vs max|ref| {np.abs(ref).max():.3e}"


def dev(torch, x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()


# ---------------------------------------------------------------------------
# helpers building the same problem on both sides
# ---------------------------------------------------------------------------
def chain_case(n, xmin=-20.0, xmax=20.0, a=0.05, b=5.0, x0=-5.0, sigma=1.0, k0=1.0,
               state="packet", seed=11):
    """state "packet": the Sect. 3.1 Gaussian; "dense": a seeded random state
    with amplitude on every site."""
    if n == 1:  # single point: H = 1/dx^2 + V
        V, dx, psi0 = np.array([0.3]), 1.0, np.array([1.0 + 0.0j])
        return dict(kind="chain", n=1, dx=dx, V=V, psi0=psi0, H=O.chain1d(V, dx))
    x, dx, V, psi0 = W.double_well_inputs(n, xmin, xmax, a, b, x0, sigma, k0)
    if state == "dense":
        psi0 = W.random_state(n, seed)
    return dict(kind="chain", n=n, dx=dx, V=V, psi0=psi0, H=O.chain1d(V, dx))


def honey_case(width, length, edge="zigzag", Wd=0.5, seed=0, sigma=None, k0=1.0,
               state="packet"):
    """state "packet": the injected Gaussian of the ribbon workload; "dense": a
    seeded random state with amplitude on every site (borders, far strips and
    chunks included)."""
    eps = W.anderson_disorder(width, length, Wd, seed)
    if state == "dense":
        psi0 = W.random_state(width * length, seed + 101)
    else:
        sig = sigma if sigma is not None else min(20.0, width / 4.0)
        psi0 = W.ribbon_packet(width, length, sig, k0)
    return dict(kind="honey", width=width, length=length, edge=edge, eps=eps, psi0=psi0,
                H=O.honeycomb(width, length, eps, edge=edge))


def holstein_case(L, nph, g2, periodic=True, Delta=0.0, state="vacuum"):
    """state "vacuum": the electron on site 0 with no phonons; "dense": a
    seeded random state over the whole basis."""
    g = math.sqrt(g2)
    nconf = O.holstein_nconf(L, nph)
    if state == "dense":
        psi0 = W.random_state(L * nconf, 31 + L + nph)
    else:
        psi0 = W.holstein_vacuum_site(L, 0, nconf)
    return dict(kind="holstein", L=L, nph=nph, g=g, Delta=Delta, periodic=periodic, psi0=psi0,
                H=O.holstein(L, nph, 1.0, 1.0, g, Delta, periodic))


def gpu_context(torch, cheb, case):
    ctx = cheb.Context()
    if case["kind"] == "chain":
        case["V_dev"] = dev(torch, case["V"])
        ctx.chain1d(case["V_dev"], case["dx"])
    elif case["kind"] == "honey":
        case["eps_dev"] = dev(torch, case["eps"])
        ctx.honeycomb(case["width"], case["length"], case["eps_dev"], edge=case["edge"])
    else:
        ctx.holstein(case["L"], case["nph"], 1.0, 1.0, case["g"], case["Delta"], case["periodic"])
    return ctx


def run_both(torch, cheb, case, dt, K, flags=0, M=None):
    H = case["H"]
    emin, emax = H.gershgorin()
    if emax == emin:  # a 1x1 Hamiltonian: any interval around its value
        emin, emax = emin - 1.0, emax + 1.0
    plan = O.Plan(emin, emax, dt, M=M)
    ctx = gpu_context(torch, cheb, case)
    ctx.set_bounds(emin, emax, 0.01)
    Mg = ctx.plan(dt) if M is None else (ctx.plan_order(dt, M) and M)
    assert Mg == plan.M
    psi = dev(torch, case["psi0"])
    nrm = torch.zeros(K, dtype=torch.float64, device="cuda")
    en = torch.zeros(K, dtype=torch.float64, device="cuda")
    say(f"[gpu] propagate {case['kind']} n={ctx.n} M={Mg} K={K} flags={flags}")
    ctx.propagate(psi, K, nrm, en, flags)
    torch.cuda.synchronize()
    ref, rn, re = O.propagate(H, plan, case["psi0"], K, want_obs=True)
    return ctx, host(psi), ref, host(nrm), rn, host(en), re, plan


# ---------------------------------------------------------------------------
# plan
# ---------------------------------------------------------------------------
def test_plan_weights_match_oracle(torch, cheb):
    case = chain_case(600)
    emin, emax = case["H"].gershgorin()
    ctx = gpu_context(torch, cheb, case)
    ctx.set_bounds(emin, emax)
    for dt in (1e-3, 0.05, 0.5):
        M = ctx.plan(dt)
        p = ctx.get_plan()
        ref = O.Plan(emin, emax, dt)
        assert M == ref.M and p["a"] == ref.a and p["b"] == ref.b
        # two independent Miller recurrences: rounding grows like sqrt(z) eps
        z = ref.a * dt
        np.testing.assert_allclose(p["gamma"], ref.gamma, rtol=0,
                                   atol=1e-15 + 4e-16 * np.sqrt(max(z, 1.0)))


@pytest.mark.parametrize("which", ["chain", "zigzag", "armchair", "holstein"])
def test_gershgorin_matches_oracle(torch, cheb, which):
    case = {"chain": lambda: chain_case(5000), "zigzag": lambda: honey_case(9, 301),
            "armchair": lambda: honey_case(9, 301, "armchair"),
            "holstein": lambda: holstein_case(5, 4, 0.5, False, 0.3)}[which]()
    ctx = gpu_context(torch, cheb, case)
    lo, hi = ctx.gershgorin()
    rlo, rhi = case["H"].gershgorin()
    assert lo == pytest.approx(rlo, rel=1e-14, abs=1e-14)
    assert hi == pytest.approx(rhi, rel=1e-14, abs=1e-14)


# ---------------------------------------------------------------------------
# propagation parity
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,flags", [(1, 0), (17, 0), (700, 0), (1024, 0), (1500, 0), (4096, 0),
                                     (4096, 8), (5003, 0), (70001, 0)])
@pytest.mark.parametrize("state", ["packet", "dense"])
def test_chain_parity(torch, cheb, n, flags, state):
    case = chain_case(n, state=state) if n > 64 else chain_case(n, -2.0, 2.0, state=state)
    dt, K = (0.02, 4) if n >= 4096 else (0.05, 5)
    if n == 1:
        dt = 0.3
    _, psi, ref, nrm, rn, en, re, plan = run_both(torch, cheb, case, dt, K, flags)
    assert_state_close(psi, ref)
    np.testing.assert_allclose(nrm, rn, rtol=1e-12)
    np.testing.assert_allclose(en, re, rtol=1e-11, atol=1e-11 * plan.a)


# Chains of 129 .. 4096 sites run in one launch over several one-wavefront
# workgroups that swap halo strips every H orders; every site's arithmetic is
# that of the one-workgroup kernel, so psi is bitwise equal to it (the step
# norm and energy add the same terms in another order).  The shapes include an
# exchange every two orders ("2,64,2"), a last workgroup owning fewer sites
# than its halo (n = 129 with 128 own sites per workgroup; n = 777) and
# workgroups of four wavefronts ("2,256,96").
def _chain_run(torch, cheb, monkeypatch, case, env, K=3, dt=0.05):
    if env is None:
        monkeypatch.delenv("CHEBTD_CHAIN_MULTI", raising=False)
    else:
        monkeypatch.setenv("CHEBTD_CHAIN_MULTI", env)
    emin, emax = case["H"].gershgorin()
    ctx = gpu_context(torch, cheb, case)
    ctx.set_bounds(emin, emax, 0.01)
    ctx.plan(dt)
    psi = dev(torch, case["psi0"])
    nrm = torch.zeros(K, dtype=torch.float64, device="cuda")
    en = torch.zeros(K, dtype=torch.float64, device="cuda")
    say(f"[gpu] chain n={case['n']} workgroups={env}")
    ctx.propagate(psi, K, nrm, en, 0)
    torch.cuda.synchronize()
    out = host(psi), host(nrm), host(en)
    ctx.close()
    return out


@pytest.mark.parametrize("n", [129, 385, 777, 1500, 4096])
@pytest.mark.parametrize("cfg", ["default", "2,64,2", "4,64,64", "8,64,128", "2,256,96"])
def test_chain_workgroups_equal_one_workgroup(torch, cheb, monkeypatch, n, cfg):
    case = chain_case(n, state="dense")
    one = _chain_run(torch, cheb, monkeypatch, case, "0")
    many = _chain_run(torch, cheb, monkeypatch, case, None if cfg == "default" else cfg)
    assert np.array_equal(many[0], one[0])
    np.testing.assert_allclose(many[1], one[1], rtol=1e-13)
    np.testing.assert_allclose(many[2], one[2], rtol=1e-12, atol=1e-12 * np.abs(one[2]).max())


@pytest.mark.parametrize("mode", [1, 2])  # CHEBTD_ADJ_STEP, CHEBTD_ADJ_SQRTM: psi checkpoints from the chain run
def test_chain_workgroups_keep_the_same_checkpoints(torch, cheb, monkeypatch, mode):
    n, K = 1000, 3
    case = chain_case(n, state="dense")
    emin, emax = case["H"].gershgorin()

    def grad(env):
        if env is None:
            monkeypatch.delenv("CHEBTD_CHAIN_MULTI", raising=False)
        else:
            monkeypatch.setenv("CHEBTD_CHAIN_MULTI", env)
        ctx = gpu_context(torch, cheb, case)
        ctx.set_bounds(emin, emax, 0.01)
        ctx.plan(0.05)
        ctx.reserve_adjoint(K, mode)
        psi = dev(torch, case["psi0"])
        ctx.propagate(psi, K, flags=cheb.KEEP_CHECKPOINTS)
        gbar = torch.from_numpy(W.random_state(n, 77)).cuda()
        dV = torch.zeros(n, dtype=torch.float64, device="cuda")
        ctx.adjoint(gbar, dV)
        torch.cuda.synchronize()
        out = host(psi), host(gbar), host(dV)
        ctx.close()
        return out

    one, many = grad("0"), grad(None)
    for a, b in zip(one, many):
        assert np.array_equal(a, b)


def test_chain_workgroups_two_streams_at_once(torch, cheb, monkeypatch):
    # two contexts on two streams run the several-workgroup chain at the same
    # time: each has its own exchange scratch and both fit the GPU together;
    # each result equals the same run alone
    monkeypatch.delenv("CHEBTD_CHAIN_MULTI", raising=False)
    case = chain_case(4096, state="dense")
    emin, emax = case["H"].gershgorin()
    Vd = dev(torch, case["V"])
    starts = [case["psi0"], W.random_state(4096, 5)]
    ctxs = []
    for st in (torch.cuda.Stream(), torch.cuda.Stream()):
        ctx = cheb.Context(stream=st)
        ctx.chain1d(Vd, case["dx"])
        ctx.set_bounds(emin, emax, 0.01)
        ctx.plan(0.5)
        ctxs.append(ctx)
    alone = []
    for ctx, p0 in zip(ctxs, starts):
        psi = dev(torch, p0)
        torch.cuda.synchronize()
        ctx.propagate(psi, 3, flags=cheb.NO_CHECK)
        torch.cuda.synchronize()
        alone.append(host(psi))
    both = [dev(torch, p0) for p0 in starts]
    torch.cuda.synchronize()
    say("[gpu] two chain runs on two streams")
    for ctx, psi in zip(ctxs, both):
        ctx.propagate(psi, 3, flags=cheb.NO_CHECK)
    torch.cuda.synchronize()
    for a, b in zip(alone, both):
        assert np.array_equal(a, host(b))
    for ctx in ctxs:
        ctx.close()


def test_chain_workgroups_report_a_wait_that_runs_out(torch, cheb, monkeypatch):
    # a wait limit of zero, set from the host, makes every workgroup give up at
    # its first wait: the kernel still ends, leaves psi NaN and the call
    # reports the time-out; the next call, with the normal limit, is right again
    case = chain_case(4096, state="dense")
    emin, emax = case["H"].gershgorin()
    monkeypatch.delenv("CHEBTD_CHAIN_MULTI", raising=False)
    monkeypatch.setenv("CHEBTD_CHAIN_SPIN", "0")
    ctx = gpu_context(torch, cheb, case)
    ctx.set_bounds(emin, emax, 0.01)
    ctx.plan(0.5)
    psi = dev(torch, case["psi0"])
    with pytest.raises(cheb.ChebError) as err:
        ctx.propagate(psi, 2)
    assert err.value.code == -6  # CHEBTD_E_TIMEOUT
    assert bool(torch.isnan(psi).all())
    monkeypatch.delenv("CHEBTD_CHAIN_SPIN")
    psi = dev(torch, case["psi0"])
    ctx.propagate(psi, 2)
    torch.cuda.synchronize()
    ref = O.propagate(case["H"], O.Plan(emin, emax, 0.5), case["psi0"], 2)
    assert_state_close(host(psi), ref)
    ctx.close()


@pytest.mark.parametrize("edge,width,length", [("zigzag", 6, 300), ("zigzag", 1, 513),
                                               ("zigzag", 31, 257), ("armchair", 6, 300),
                                               ("armchair", 10, 1000), ("zigzag", 128, 200)])
@pytest.mark.parametrize("state", ["packet", "dense"])
def test_honeycomb_parity(torch, cheb, edge, width, length, state):
    case = honey_case(width, length, edge, state=state)
    _, psi, ref, nrm, rn, en, re, plan = run_both(torch, cheb, case, 1.0, 6)
    assert_state_close(psi, ref)
    np.testing.assert_allclose(nrm, rn, rtol=1e-12)
    np.testing.assert_allclose(en, re, rtol=1e-11, atol=1e-11)


# Table 2 shape (Sect. 3.2): the 10 x 1000 armchair ribbon from one occupied
# site at its centre, at dt = 1, 10 and 100 (M = 20, 67, 399) to t = 100 (the
# paper runs to t = 1e4), replayed as a graph
@pytest.mark.parametrize("dt", [1.0, 10.0, 100.0])
def test_table2_ribbon_single_site(torch, cheb, dt):
    p = W.TABLE2.params
    w, l = p["width"], p["length"]
    eps, psi0 = W.table2_inputs(w, l, p["W"], p["seed"])
    case = dict(kind="honey", width=w, length=l, edge=p["edge"], eps=eps, psi0=psi0,
                H=O.honeycomb(w, l, eps, edge=p["edge"]))
    K = int(round(100.0 / dt))
    _, psi, ref, nrm, rn, en, re, plan = run_both(torch, cheb, case, dt, K, flags=cheb.GRAPH)
    assert_state_close(psi, ref)
    np.testing.assert_allclose(nrm, rn, rtol=1e-12)
    np.testing.assert_allclose(en, re, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("L,nph,g2,periodic", [(4, 3, 0.5, True), (6, 4, 2.0, True), (5, 5, 0.5, False),
                                               (3, 6, 2.0, True), (1, 7, 0.5, False), (2, 5, 0.5, False),
                                               (5, 0, 2.0, True)])
@pytest.mark.parametrize("state", ["vacuum", "dense"])
@pytest.mark.parametrize("rank", [None, True])
def test_holstein_parity_and_observables(torch, cheb, hol_spt_env, L, nph, g2, periodic, state, rank):
    # rank True: the walk ranks the phonon partners itself (its default
    # only past 8M states); None: the size rule (the partner tables here)
    case = holstein_case(L, nph, g2, periodic, Delta=np.linspace(0, 0.5, L), state=state)
    hol_spt_env(None, rank)
    ctx, psi, ref, nrm, rn, en, re, _ = run_both(torch, cheb, case, 0.1, 8)
    assert_state_close(psi, ref)
    np.testing.assert_allclose(nrm, rn, rtol=1e-12)
    _, name, orders = ctx.time_recursion_kernel(1)  # the walk that ran
    assert orders == 1 and name == ("k_iter_hol<true, false>" if rank else "k_iter_hol<false, false>")
    n_i, nph_i, chi = (host(t) for t in ctx.holstein_obs(dev(torch, ref)))
    rn_i, rnph_i, rchi = O.holstein_obs(L, nph, ref)
    np.testing.assert_allclose(n_i, rn_i, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(nph_i, rnph_i, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(chi, rchi, rtol=1e-11, atol=1e-14)


def test_polaron_figure3_parameters_reduced(torch, cheb):
    # the Fig. 3 setting (open chain, barrier with extra local coupling, packet
    # moving right with k = pi/9) on 12 sites with at most 5 phonons, to the
    # figure's last time
    p = W.POLARON_PAPER.params
    L, nph = 12, 5
    g, Delta = W.polaron_couplings(L, p["w0"], p["eps_p"], p["eps_p_barrier"], 8, p["barrier"])
    H = O.holstein(L, nph, p["t"], p["w0"], g, Delta, False)
    psi0 = W.holstein_packet(L, O.holstein_nconf(L, nph), p["packet_site"], p["width"], p["k"])
    emin, emax = H.gershgorin()
    ctx = cheb.Context()
    ctx.holstein(L, nph, p["t"], p["w0"], g, Delta, False)
    ctx.set_bounds(emin, emax)
    plan = O.Plan(emin, emax, p["dt"])
    assert ctx.plan(p["dt"]) == plan.M
    # the figure's times t = 6, 10, 14, reached step by step on both sides
    psi, ref, t_prev = dev(torch, psi0), psi0, 0.0
    for ts in p["snapshots"]:
        K = int(round((ts - t_prev) / p["dt"]))
        ctx.propagate(psi, K)
        torch.cuda.synchronize()
        ref = O.propagate(H, plan, ref, K)
        assert_state_close(host(psi), ref)
        for a, b in zip((host(t) for t in ctx.holstein_obs(psi)), O.holstein_obs(L, nph, ref)):
            np.testing.assert_allclose(a, b, rtol=1e-11, atol=1e-14)
        t_prev = ts


@pytest.fixture
def hol_spt_env():
    """setter(spt, rank=None): sites per thread of the Holstein walk (None:
    its default) and whether it ranks the phonon partners itself (True) or
    reads the per-state partner tables (False); None: its size rule."""
    import os
    saved = {k: os.environ.get(k) for k in ("CHEBTD_HOL_SPT", "CHEBTD_HOL_RANK")}

    def setter(spt, rank=None):
        if spt is None:
            os.environ.pop("CHEBTD_HOL_SPT", None)
        else:
            os.environ["CHEBTD_HOL_SPT"] = str(spt)
        if rank is None:
            os.environ.pop("CHEBTD_HOL_RANK", None)
        else:
            os.environ["CHEBTD_HOL_RANK"] = "1" if rank else "0"
    yield setter
    for k, v in saved.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v


def _polaron_fig3(L, nph, barrier_site, periodic, state):
    p = W.POLARON_PAPER.params
    g, Delta = W.polaron_couplings(L, p["w0"], p["eps_p"], p["eps_p_barrier"], barrier_site,
                                   p["barrier"])
    H = O.holstein(L, nph, p["t"], p["w0"], g, Delta, periodic)
    nconf = O.holstein_nconf(L, nph)
    if state == "dense":
        psi0 = W.random_state(L * nconf, 400 + L)
    else:
        psi0 = W.holstein_packet(L, nconf, p["packet_site"], p["width"], p["k"])
    return p, g, Delta, H, psi0


# the walk takes every electron site of a configuration in one thread by
# default; CHEBTD_HOL_SPT groups them instead, which exercises group
# boundaries inside the chain (left neighbour from the previous group),
# groups that do not divide L and the ring's wrap from the last group to the
# first, for both walks (partner ranks formed in the walk or read)
@pytest.mark.parametrize("spt,rank", [(1, True), (2, True), (3, True), (5, True), (7, True), (9, True),
                                      (12, True), (1, False), (5, False), (12, False)])
@pytest.mark.parametrize("periodic,state", [(False, "packet"), (False, "dense"), (True, "dense")])
def test_holstein_grouped_walk_matches_oracle(torch, cheb, hol_spt_env, spt, rank, periodic, state):
    # rank: the walk ranks the phonon partners itself (combinatorial number
    # system, digit by digit as it walks the sites; a group starting past
    # site 0 first takes the digits before it) or reads the partner tables
    L, nph = 12, 5
    p, g, Delta, H, psi0 = _polaron_fig3(L, nph, 8, periodic, state)
    hol_spt_env(spt, rank)
    ctx = cheb.Context()
    ctx.holstein(L, nph, p["t"], p["w0"], g, Delta, periodic)
    hol_spt_env(None)
    emin, emax = H.gershgorin()
    ctx.set_bounds(emin, emax)
    plan = O.Plan(emin, emax, p["dt"])
    assert ctx.plan(p["dt"]) == plan.M
    psi = dev(torch, psi0)
    nrm = torch.zeros(6, dtype=torch.float64, device="cuda")
    say(f"[gpu] Holstein grouped walk spt={spt} periodic={periodic} {state}")
    ctx.propagate(psi, 6, nrm)
    torch.cuda.synchronize()
    ref, rn, _ = O.propagate(H, plan, psi0, 6, want_obs=True)
    assert_state_close(host(psi), ref)
    np.testing.assert_allclose(host(nrm), rn, rtol=1e-12)
    for a, b in zip((host(t) for t in ctx.holstein_obs(psi)), O.holstein_obs(L, nph, ref)):
        np.testing.assert_allclose(a, b, rtol=1e-11, atol=1e-14)


def test_holstein_open_chain_16M_states_matches_oracle(torch, cheb, hol_spt_env):
    # 12 open sites with up to 11 phonons: 1,352,078 configurations (16.2M
    # states, past 8M: the defaults of the Fig. 3 polaron's size, every site
    # in one thread and the partner ranks formed in the walk), then grouped
    # by five, and reading the partner tables
    L, nph = 12, 11
    p, g, Delta, H, psi0 = _polaron_fig3(L, nph, 8, False, "packet")
    assert O.holstein_nconf(L, nph) == 1_352_078
    emin, emax = H.gershgorin()
    plan = O.Plan(emin, emax, p["dt"])
    ref = O.propagate(H, plan, psi0, 2)
    ref_obs = O.holstein_obs(L, nph, ref)
    for spt, rank in ((None, None), (5, True), (None, False)):
        hol_spt_env(spt, rank)
        ctx = cheb.Context()
        ctx.holstein(L, nph, p["t"], p["w0"], g, Delta, False)
        hol_spt_env(None)
        ctx.set_bounds(emin, emax)
        assert ctx.plan(p["dt"]) == plan.M
        psi = dev(torch, psi0)
        say(f"[gpu] Holstein L=12 nph=11 (16.2M states), sites per thread {spt or L}, own ranks {rank}")
        ctx.propagate(psi, 2)
        torch.cuda.synchronize()
        ranks = rank is None or rank  # past 8M states the default ranks the partners
        assert ctx.time_recursion_kernel(1)[1].startswith("k_iter_hol<true" if ranks else "k_iter_hol<false")
        assert_state_close(host(psi), ref)
        for a, b in zip((host(t) for t in ctx.holstein_obs(psi)), ref_obs):
            np.testing.assert_allclose(a, b, rtol=1e-11, atol=1e-14)
        ctx.close()


def test_holstein_matrix_free_matches_csr_path(torch, cheb):
    # the matrix-free Holstein operator and the general CSR kernel on the
    # library's own host-built CSR of the same eq. (ghm) matrix
    L, nph = 6, 5
    g = np.linspace(0.4, 1.1, L)
    Delta = np.linspace(-0.3, 0.4, L)
    for periodic in (True, False):
        rowptr, col, val = cheb.holstein_csr_host(L, nph, 1.0, 1.3, g, Delta, periodic)
        mf = cheb.Context()
        mf.holstein(L, nph, 1.0, 1.3, g, Delta, periodic)
        cs = cheb.Context()
        r_d, c_d, v_d = dev(torch, rowptr), dev(torch, col), dev(torch, val)
        cs.csr(r_d, c_d, v_d)
        lo, hi = mf.gershgorin()
        lo2, hi2 = cs.gershgorin()
        assert lo == pytest.approx(lo2, rel=1e-14) and hi == pytest.approx(hi2, rel=1e-14)
        psi0 = W.holstein_packet(L, mf.n // L, 2.0, 1.0, 0.5)
        outs = []
        for ctx in (mf, cs):
            ctx.set_bounds(lo, hi)
            ctx.plan(0.3)
            p = dev(torch, psi0)
            ctx.propagate(p, 6)
            torch.cuda.synchronize()
            outs.append(host(p))
        assert rel_l2(outs[0], outs[1]) <= 1e-13


def test_generic_csr_parity(torch, cheb):
    # a complex Hermitian matrix through chebtd_h_csr (device CSR from the caller)
    rng = np.random.default_rng(3)
    n = 777
    A = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        for j in rng.choice(n, 4, replace=False):
            v = rng.normal() + 1j * rng.normal()
            A[i, j] += v
            A[j, i] += np.conj(v)
    A[np.diag_indices(n)] = rng.normal(size=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    cols, vals = [], []
    for i in range(n):
        nz = np.nonzero(A[i])[0]
        cols += list(nz)
        vals += list(A[i, nz])
        rowptr[i + 1] = len(cols)
    H = O.import_csr(rowptr, np.array(cols), np.array(vals))
    emin, emax = H.gershgorin()
    psi0 = (rng.normal(size=n) + 1j * rng.normal(size=n))
    psi0 /= np.linalg.norm(psi0)
    plan = O.Plan(emin, emax, 0.7)
    ctx = cheb.Context()
    r_d, c_d, v_d = dev(torch, rowptr), dev(torch, np.array(cols, np.int32)), dev(torch, np.array(vals))
    ctx.csr(r_d, c_d, v_d)
    lo, hi = ctx.gershgorin()
    assert lo == pytest.approx(emin, rel=1e-13) and hi == pytest.approx(emax, rel=1e-13)
    ctx.set_bounds(emin, emax)
    assert ctx.plan(0.7) == plan.M
    psi = dev(torch, psi0)
    ctx.propagate(psi, 5)
    assert_state_close(host(psi), O.propagate(H, plan, psi0, 5))


def _hermitian_csr(A):
    n = A.shape[0]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    cols, vals = [], []
    for i in range(n):
        nz = np.nonzero(A[i])[0]
        cols += list(nz)
        vals += list(A[i, nz])
        rowptr[i + 1] = len(cols)
    return rowptr, np.array(cols, dtype=np.int32), np.array(vals, dtype=np.complex128)


# CSR edge cases: a single entry, empty rows (eigenvalue 0, no neighbours),
# and rows with 1 .. 13 entries (the kernel takes entries four at a time, so
# every remainder of that loop), under lazy accumulation over 7 steps
@pytest.mark.parametrize("case", ["single", "empty_rows", "ragged_rows"])
def test_csr_edge_cases_match_oracle(torch, cheb, case):
    rng = np.random.default_rng(17)
    if case == "single":
        A = np.array([[0.3 + 0.0j]])
    else:
        n = 60
        A = np.zeros((n, n), dtype=np.complex128)
        if case == "empty_rows":
            live = np.arange(10, n)  # rows 0 .. 9 stay empty
            for i in live:
                j = rng.choice(live)
                v = rng.normal() + 1j * rng.normal()
                A[i, j] += v
                A[j, i] += np.conj(v)
        else:  # row 0 holds its diagonal alone
            for i in range(1, n):
                for j in rng.choice(np.arange(1, n), 1 + i % 7, replace=False):
                    if j != i:
                        v = rng.normal() + 1j * rng.normal()
                        A[i, j] += v
                        A[j, i] += np.conj(v)
            A[np.diag_indices(n)] = rng.normal(size=n)
        counts = np.count_nonzero(A, axis=1)
        if case == "ragged_rows":
            assert counts[0] == 1 and counts.max() >= 9 and set((counts % 4).tolist()) == {0, 1, 2, 3}
        else:
            assert (counts[:10] == 0).all()
    rowptr, cols, vals = _hermitian_csr(A)
    H = O.import_csr(rowptr, cols.astype(np.int64), vals)
    emin, emax = H.gershgorin()
    if emax == emin:
        emin, emax = emin - 1.0, emax + 1.0
    n = A.shape[0]
    psi0 = W.random_state(n, 77 + n)
    plan = O.Plan(emin, emax, 0.9)
    ctx = cheb.Context()
    r_d, c_d, v_d = dev(torch, rowptr), dev(torch, cols), dev(torch, vals)
    ctx.csr(r_d, c_d, v_d)
    ctx.set_bounds(emin, emax)
    assert ctx.plan(0.9) == plan.M
    psi = dev(torch, psi0)
    nrm = torch.zeros(7, dtype=torch.float64, device="cuda")
    say(f"[gpu] CSR edge case {case}, n={n}, nnz={len(vals)}, M={plan.M}")
    ctx.propagate(psi, 7, nrm)
    torch.cuda.synchronize()
    ref, rn, _ = O.propagate(H, plan, psi0, 7, want_obs=True)
    assert_state_close(host(psi), ref)
    np.testing.assert_allclose(host(nrm), rn, rtol=1e-12)


@pytest.mark.parametrize("M", [0, 1, 2, 3])
def test_low_orders(torch, cheb, M):
    for case in (chain_case(300, state="dense"), chain_case(9000, state="dense"),
                 honey_case(5, 100, state="dense")):
        # a forced low order is not unitary: skip the norm check
        _, psi, ref, *_ = run_both(torch, cheb, case, 1e-4, 3, flags=cheb.NO_CHECK, M=M)
        assert_state_close(psi, ref)


# ---------------------------------------------------------------------------
# two orders per pass vs one order per pass
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("rows", ["1", "3", "8", "16", "200"])
def test_two_orders_per_pass_matches_single_order_and_oracle(torch, cheb, rows, monkeypatch):
    monkeypatch.setenv("CHEBTD_PAIR_ROWS", rows)
    cases = [(honey_case(19, 211, state="dense"), 1.0),
             (honey_case(12, 130, "armchair", state="dense"), 1.0),
             (honey_case(1, 300, state="dense"), 1.0), (chain_case(9001, state="dense"), 0.002),
             (honey_case(64, 640, state="dense"), 1.4), (honey_case(64, 640), 1.4)]
    for case, dt in cases:
        H = case["H"]
        emin, emax = H.gershgorin()
        ctx = gpu_context(torch, cheb, case)
        ctx.set_bounds(emin, emax)
        M = ctx.plan(dt)
        a = dev(torch, case["psi0"])
        b = dev(torch, case["psi0"])
        na = torch.zeros(3, dtype=torch.float64, device="cuda")
        nb = torch.zeros(3, dtype=torch.float64, device="cuda")
        say(f"[gpu] pairs rows={rows} {case['kind']} n={ctx.n} M={M}")
        ctx.propagate(a, 3, na)
        ctx.propagate(b, 3, nb, flags=cheb.SINGLE_ORDER)
        torch.cuda.synchronize()
        ref = O.propagate(H, O.Plan(emin, emax, dt), case["psi0"], 3)
        assert_state_close(host(a), ref)
        assert_state_close(host(b), ref)
        assert rel_l2(host(a), host(b)) <= 1e-13
        np.testing.assert_allclose(host(na), host(nb), rtol=1e-13)


@pytest.mark.parametrize("M", [2, 3, 4, 5, 8, 9])
def test_two_orders_per_pass_at_small_orders(torch, cheb, M):
    for case in (honey_case(10, 300, state="dense"), chain_case(7000, state="dense")):
        _, psi, ref, nrm, rn, *_ = run_both(torch, cheb, case, 0.01, 3, flags=cheb.NO_CHECK, M=M)
        assert_state_close(psi, ref)
        np.testing.assert_allclose(nrm, rn, rtol=1e-12)


# ---------------------------------------------------------------------------
# launch-mode equivalence, determinism, resume
# ---------------------------------------------------------------------------
def test_graph_replay_matches_direct_launches(torch, cheb):
    case = honey_case(16, 700)
    emin, emax = case["H"].gershgorin()
    ctx = gpu_context(torch, cheb, case)
    ctx.set_bounds(emin, emax)
    ctx.plan(1.0)
    outs = []
    for flags in (0, cheb.GRAPH, cheb.GRAPH, 0):
        for K in (7, 8):
            psi = dev(torch, case["psi0"])
            nrm = torch.zeros(K, dtype=torch.float64, device="cuda")
            say(f"[gpu] graph flags={flags} K={K}")
            ctx.propagate(psi, K, nrm, None, flags)
            torch.cuda.synchronize()
            outs.append((K, host(psi), host(nrm)))
    by_k = {}
    for K, p, n_ in outs:
        if K in by_k:
            np.testing.assert_array_equal(p, by_k[K][0])
            np.testing.assert_array_equal(n_, by_k[K][1])
        else:
            by_k[K] = (p, n_)


def test_bitwise_determinism_and_resume(torch, cheb):
    for case in (honey_case(12, 400), chain_case(3000), chain_case(6000),
                 holstein_case(5, 4, 2.0)):
        emin, emax = case["H"].gershgorin()
        ctx = gpu_context(torch, cheb, case)
        ctx.set_bounds(emin, emax)
        ctx.plan(0.3)
        a = dev(torch, case["psi0"])
        b = dev(torch, case["psi0"])
        ctx.propagate(a, 9)
        ctx.propagate(b, 4)
        ctx.propagate(b, 5)
        c = dev(torch, case["psi0"])
        ctx.propagate(c, 9)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(a), host(b))
        np.testing.assert_array_equal(host(a), host(c))


def test_persistent_matches_per_iteration_launches(torch, cheb):
    case = chain_case(4096)
    emin, emax = case["H"].gershgorin()
    ctx = gpu_context(torch, cheb, case)
    ctx.set_bounds(emin, emax)
    ctx.plan(0.05)
    a = dev(torch, case["psi0"])
    b = dev(torch, case["psi0"])
    ctx.propagate(a, 3)
    ctx.propagate(b, 3, flags=cheb.NO_PERSISTENT)
    torch.cuda.synchronize()
    assert rel_l2(host(a), host(b)) <= 1e-13


# ---------------------------------------------------------------------------
# observables and failure detection
# ---------------------------------------------------------------------------
def test_density_region_norm_energy(torch, cheb):
    case = honey_case(8, 300)
    emin, emax = case["H"].gershgorin()
    ctx = gpu_context(torch, cheb, case)
    ctx.set_bounds(emin, emax)
    psi = dev(torch, case["psi0"])
    np.testing.assert_allclose(host(ctx.density(psi)), O.density(case["psi0"]), rtol=1e-15)
    mask = W.right_half_mask_ribbon(8, 300).astype(np.uint8)
    mask[::7] = 1
    out = host(ctx.region_sum(psi, dev(torch, mask)))[0]
    assert out == pytest.approx(O.region_sum(case["psi0"], mask), rel=1e-13)
    ne = host(ctx.norm_energy(psi))
    Hd = case["H"].dense()
    assert ne[0] == pytest.approx(1.0, rel=1e-13)
    assert ne[1] == pytest.approx(np.vdot(case["psi0"], Hd @ case["psi0"]).real, rel=1e-12, abs=1e-13)


@pytest.mark.parametrize("kind", ["chain", "csr", "holstein_tables", "holstein_ranks"])
def test_norm_energy_of_every_operator(torch, cheb, hol_spt_env, kind):
    # <psi|psi> and <psi|H|psi> of a dense state through chebtd_norm_energy:
    # for the Holstein model the walk's head mode without outputs (partial
    # sums only), with the partner tables and with the ranks formed in the walk
    rank = None
    if kind == "chain":
        case = chain_case(777, state="dense")
    elif kind == "csr":
        case = holstein_case(5, 4, 2.0, True, state="dense")
        rowptr, col, val = case["H"].csr()
        case = dict(case, kind="csr", csr=(rowptr, col.astype(np.int32), val))
    else:
        case = holstein_case(6, 5, 0.5, False, Delta=np.linspace(0, 0.3, 6), state="dense")
        rank = kind == "holstein_ranks"
    hol_spt_env(None, rank)
    emin, emax = case["H"].gershgorin()
    if kind == "csr":
        ctx = cheb.Context()
        r_d, c_d, v_d = (dev(torch, a) for a in case["csr"])
        ctx.csr(r_d, c_d, v_d)
    else:
        ctx = gpu_context(torch, cheb, case)
    ctx.set_bounds(emin, emax)
    psi0 = case["psi0"]
    ne = host(ctx.norm_energy(dev(torch, psi0)))
    e_ref = np.vdot(psi0, case["H"].dense() @ psi0).real
    assert ne[0] == pytest.approx(float(np.vdot(psi0, psi0).real), rel=1e-13)
    assert ne[1] == pytest.approx(e_ref, rel=1e-12, abs=1e-12 * (abs(emin) + abs(emax)))
    ctx.close()


def test_region_sum_and_norm_past_the_reduction_grid(torch, cheb):
    # 1.5M sites: each thread of the norm and region sums walks several sites
    # (at most 2048 blocks of 256 threads); both against numpy sums
    n = 1_500_001
    psi0 = W.random_state(n, 4242)
    mask = (W.uniform01(77, n) < 0.3).astype(np.uint8)
    x, dx = W.chain_grid(n, -30.0, 30.0)
    ctx = cheb.Context()
    V = torch.from_numpy(W.harmonic(x, 1e-3)).cuda()
    ctx.chain1d(V, dx)
    ctx.set_bounds(*ctx.gershgorin())
    psi = dev(torch, psi0)
    rho = np.abs(psi0) ** 2
    got = host(ctx.region_sum(psi, dev(torch, mask)))[0]
    assert got == pytest.approx(float(rho[mask == 1].sum()), rel=1e-12)
    ne = host(ctx.norm_energy(psi))
    assert ne[0] == pytest.approx(float(rho.sum()), rel=1e-12)
    ctx.close()


def test_divergence_is_reported(torch, cheb):
    # bounds that miss most of the spectrum make T_k(H~) grow: the end-of-call
    # check must report it instead of returning garbage
    case = chain_case(2000)
    ctx = gpu_context(torch, cheb, case)
    ctx.set_bounds(0.0, 1.0, 0.01)
    ctx.plan(0.5)
    psi = dev(torch, case["psi0"])
    with pytest.raises(cheb.ChebError) as ei:
        ctx.propagate(psi, 3, flags=cheb.NO_PERSISTENT)
    assert ei.value.code == -3


def test_argument_errors_on_gpu(torch, cheb):
    ctx = cheb.Context()
    with pytest.raises(cheb.ChebError):
        ctx.plan(1.0)  # no Hamiltonian
    V = torch.zeros(10, dtype=torch.float64, device="cuda")
    ctx.chain1d(V, 0.1)
    with pytest.raises(cheb.ChebError):
        ctx.plan(1.0)  # no bounds
    with pytest.raises(cheb.ChebError):
        ctx.set_bounds(1.0, 0.0)
    with pytest.raises(TypeError):
        ctx.propagate(torch.zeros(10, dtype=torch.complex64, device="cuda"), 1)


# ---------------------------------------------------------------------------
# full-size workloads, in the launch configuration the benchmark times
# ---------------------------------------------------------------------------
def test_full_double_well_4096(torch, cheb):
    p = W.DOUBLE_WELL.params
    case = chain_case(p["n"], p["xmin"], p["xmax"], p["a"], p["b"], p["x0"], p["sigma"], p["k0"])
    _, psi, ref, nrm, rn, en, re, plan = run_both(torch, cheb, case, p["dt"], 2)
    assert plan.M > 7000
    assert_state_close(psi, ref)
    np.testing.assert_allclose(en, re, rtol=1e-11)


@pytest.mark.parametrize("state", ["packet", "dense"])
def test_full_zigzag_ribbon_128x8192(torch, cheb, state):
    p = W.GRAPHENE.params
    case = honey_case(p["width"], p["length"], p["edge"], p["W"], p["seed"], p["sigma"], p["k0"],
                      state=state)
    _, psi, ref, nrm, rn, en, re, plan = run_both(torch, cheb, case, p["dt"], 3)
    assert plan.M == 20
    assert_state_close(psi, ref)
    np.testing.assert_allclose(nrm, rn, rtol=1e-12)


@pytest.mark.parametrize("g2,state", [(0.5, "vacuum"), (2.0, "vacuum"), (2.0, "dense")])
def test_full_holstein_ring(torch, cheb, g2, state):
    p = W.HOLSTEIN.params
    case = holstein_case(p["L"], p["nph"], g2, p["periodic"], state=state)
    ctx, psi, ref, nrm, rn, en, re, plan = run_both(torch, cheb, case, p["dt"], 2)
    assert ctx.n == 1_847_560
    assert plan.M == (13 if g2 == 0.5 else 14)
    assert_state_close(psi, ref)


@pytest.mark.parametrize("g2", [0.5, 2.0])
def test_full_holstein_ring_as_general_csr(torch, cheb, g2):
    # the L = 10, N_ph <= 10 ring (1,847,560 rows, 7.39M entries) through the
    # general CSR kernel, from the library's host-built CSR, against the
    # oracle's own eq. (ghm) matrix, from a dense state
    p = W.HOLSTEIN.params
    case = holstein_case(p["L"], p["nph"], g2, p["periodic"], state="dense")
    rowptr, col, val = cheb.holstein_csr_host(p["L"], p["nph"], 1.0, 1.0, math.sqrt(g2), 0.0, p["periodic"])
    assert rowptr[-1] == 4 * 1_847_560
    ctx = cheb.Context()
    r_d, c_d, v_d = dev(torch, rowptr), dev(torch, col), dev(torch, val)
    ctx.csr(r_d, c_d, v_d)
    emin, emax = case["H"].gershgorin()
    ctx.set_bounds(emin, emax)
    plan = O.Plan(emin, emax, p["dt"])
    assert ctx.plan(p["dt"]) == plan.M
    psi = dev(torch, case["psi0"])
    nrm = torch.zeros(3, dtype=torch.float64, device="cuda")
    say(f"[gpu] Holstein ring as CSR, g2={g2}, M={plan.M}")
    ctx.propagate(psi, 3, nrm)
    torch.cuda.synchronize()
    ref, rn, _ = O.propagate(case["H"], plan, case["psi0"], 3, want_obs=True)
    assert_state_close(host(psi), ref)
    np.testing.assert_allclose(host(nrm), rn, rtol=1e-12)
