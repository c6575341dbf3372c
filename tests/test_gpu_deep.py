"""D = 3 .. 6 Chebyshev orders per pass (the deep walk) against the CPU
oracle, and against the two-orders-per-pass path, for ribbons and chains."""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from test_gpu_parity import (assert_state_close, chain_case, dev, gpu_context, honey_case, host,
                             rel_l2, run_both, say)
from windows import chain_sites, ribbon_sample_sites, ribbon_sites

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


@pytest.fixture
def depth_env():
    saved = {k: os.environ.get(k) for k in ("CHEBTD_DEPTH", "CHEBTD_DEEP_ROWS")}

    def setter(depth, rows=None):
        if depth is None:  # the library's own choice of passes
            os.environ.pop("CHEBTD_DEPTH", None)
        else:
            os.environ["CHEBTD_DEPTH"] = str(depth)
        if rows is None:
            os.environ.pop("CHEBTD_DEEP_ROWS", None)
        else:
            os.environ["CHEBTD_DEEP_ROWS"] = str(rows)
    yield setter
    for k, v in saved.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v


def run(torch, cheb, case, dt, K, M=None, flags=0):
    H = case["H"]
    emin, emax = H.gershgorin()
    plan = O.Plan(emin, emax, dt, M=M)
    ctx = gpu_context(torch, cheb, case)
    ctx.set_bounds(emin, emax, 0.01)
    Mg = ctx.plan(dt) if M is None else (ctx.plan_order(dt, M) and M)
    assert Mg == plan.M
    psi = dev(torch, case["psi0"])
    nrm = torch.zeros(K, dtype=torch.float64, device="cuda")
    en = torch.zeros(K, dtype=torch.float64, device="cuda")
    # forced low orders are not unitary: skip the end-of-call norm check
    ctx.propagate(psi, K, nrm, en, flags | (cheb.NO_CHECK if M is not None else 0))
    torch.cuda.synchronize()
    return ctx, host(psi), host(nrm), host(en), plan


# ragged ribbons: fewer rows than a chunk, partial strips, one column past a strip
@pytest.mark.parametrize("depth", [None, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("shape", [(1, 300, "zigzag"), (3, 59, "zigzag"), (8, 200, "armchair"),
                                   (17, 117, "zigzag"), (24, 61, "armchair")])
@pytest.mark.parametrize("M,state", [(3, "dense"), (4, "dense"), (5, "dense"), (6, "dense"), (7, "dense"),
                                     (11, "dense"), (20, "dense"), (5, "packet"), (20, "packet")])
def test_deep_ribbon_matches_oracle(torch, cheb, depth_env, depth, shape, M, state):
    # the dense state puts amplitude on every site: the right-hand partial
    # strip, the last chunk and the border walks are compared site by site
    w, l, edge = shape
    depth_env(depth)
    case = honey_case(w, l, edge, state=state)
    say(f"[gpu] deep D={depth} ribbon {w}x{l} {edge} M={M} {state}")
    _, psi, nrm, en, plan = run(torch, cheb, case, 1.0, 3, M=M)
    ref, rn, re = O.propagate(case["H"], plan, case["psi0"], 3, want_obs=True)
    assert_state_close(psi, ref)
    np.testing.assert_allclose(nrm, rn, rtol=1e-12)
    np.testing.assert_allclose(en, re, rtol=1e-10, atol=1e-12)


# degenerate ribbons: one site, one row or one column, a 2 x 2 cell, fewer
# columns or rows than any strip's or chunk's halo, at every pass depth
@pytest.mark.parametrize("depth", [None, 2, 3, 6])
@pytest.mark.parametrize("shape", [(1, 1), (1, 2), (2, 1), (5, 1), (2, 2), (64, 3), (3, 64)])
@pytest.mark.parametrize("edge", ["zigzag", "armchair"])
def test_degenerate_ribbons_match_oracle(torch, cheb, depth_env, depth, shape, edge):
    w, l = shape
    depth_env(depth)
    case = honey_case(w, l, edge, state="dense")
    say(f"[gpu] degenerate ribbon {w}x{l} {edge} D={depth}")
    _, psi, ref, nrm, rn, en, re, plan = run_both(torch, cheb, case, 1.0, 3)
    assert_state_close(psi, ref)
    np.testing.assert_allclose(nrm, rn, rtol=1e-12)
    np.testing.assert_allclose(en, re, rtol=1e-10, atol=1e-12)


# 37 x 130 has chunks and strips clear of the border for every depth and height
@pytest.mark.parametrize("edge", ["zigzag", "armchair"])
@pytest.mark.parametrize("depth", [3, 4, 5, 6])
@pytest.mark.parametrize("rows", [1, 2, 4, 5, 8, 16, 32])
def test_deep_chunk_heights(torch, cheb, depth_env, edge, depth, rows):
    depth_env(depth, rows)
    case = honey_case(37, 130, edge, state="dense")
    say(f"[gpu] deep D={depth} rows={rows} 37x130 {edge} dense")
    _, psi, _, _, plan = run(torch, cheb, case, 1.0, 2)
    ref = O.propagate(case["H"], plan, case["psi0"], 2)
    assert_state_close(psi, ref)


@pytest.mark.parametrize("depth", [3, 4, 5, 6])
@pytest.mark.parametrize("n", [4097, 20011])
def test_deep_chain_matches_oracle(torch, cheb, depth_env, depth, n):
    # longer than the one-workgroup chain kernel: the chain runs as a ribbon of one row
    depth_env(depth)
    case = chain_case(n, state="dense")
    say(f"[gpu] deep D={depth} chain n={n} dense")
    _, psi, _, _, plan = run(torch, cheb, case, 0.002, 2)
    ref = O.propagate(case["H"], plan, case["psi0"], 2)
    assert_state_close(psi, ref)


@pytest.mark.parametrize("depth", [3, 4, 5, 6])
def test_deep_graph_replays_bitwise_and_agrees_with_pairs(torch, cheb, depth_env, depth):
    case = honey_case(16, 700)
    depth_env(2)
    _, p2, _, _, _ = run(torch, cheb, case, 1.0, 6)
    depth_env(depth)
    _, pd, nd, _, _ = run(torch, cheb, case, 1.0, 6)
    _, pg, ng, _, _ = run(torch, cheb, case, 1.0, 6, flags=cheb.GRAPH)
    np.testing.assert_array_equal(pd, pg)
    np.testing.assert_array_equal(nd, ng)
    # the same arithmetic in another order: agreement to rounding
    assert rel_l2(pd, p2) <= 1e-13


@pytest.mark.parametrize("state", ["packet", "dense"])
def test_deep_headline_ribbon_full_size(torch, cheb, depth_env, state):
    p = W.GRAPHENE.params
    case = honey_case(p["width"], p["length"], p["edge"], p["W"], p["seed"], p["sigma"], p["k0"],
                      state=state)
    ref = rn = None
    for depth in (None, 3, 4, 5, 6):
        depth_env(depth)
        say(f"[gpu] headline ribbon 128x8192 D={depth} {state}")
        _, psi, nrm, _, plan = run(torch, cheb, case, p["dt"], 2)
        if ref is None:
            ref, rn, _ = O.propagate(case["H"], plan, case["psi0"], 2, want_obs=True)
        assert plan.M == 20
        assert_state_close(psi, ref)
        np.testing.assert_allclose(nrm, rn, rtol=1e-12)


def check_passes(passes, M, allowed):
    assert sum(passes) == M
    assert passes[0] >= 2  # the head forms v_1 .. v_D
    assert passes.count(1) <= 1 and (1 not in passes or passes[-1] == 1)
    assert all(p in allowed for p in passes)


@pytest.mark.parametrize("kind", ["ribbon", "chain"])
def test_plan_passes(torch, cheb, depth_env, kind):
    case = honey_case(16, 200) if kind == "ribbon" else chain_case(5000)
    ctx = gpu_context(torch, cheb, case)
    emin, emax = case["H"].gershgorin()
    ctx.set_bounds(emin, emax, 0.01)
    depth_env(None)
    for M in range(2, 64):
        ctx.plan_order(1.0, M)
        check_passes(ctx.plan_passes(), M, {1, 2, 3, 4, 5, 6})
    if kind == "ribbon":
        ctx.plan_order(1.0, 20)
        # the headline order splits into four deep passes
        passes = ctx.plan_passes()
        assert len(passes) == 4 and min(passes) >= 3, passes
    for depth in (2, 3, 4, 5, 6):
        depth_env(depth)
        for M in range(2, 40):
            ctx.plan_order(1.0, M)
            check_passes(ctx.plan_passes(), M, {1, 2, depth})
    depth_env(None)
    ctx.plan_order(1.0, 1)
    assert ctx.plan_passes() == []


def test_plan_passes_default_schedules_match_oracle(torch, cheb, depth_env):
    # every M from 2 to 30 under the library's own split, on one ragged ribbon
    depth_env(None)
    case = honey_case(21, 131, "armchair", state="dense")
    for M in range(2, 31):
        _, psi, nrm, en, plan = run(torch, cheb, case, 1.0, 2, M=M)
        ref, rn, re = O.propagate(case["H"], plan, case["psi0"], 2, want_obs=True)
        assert_state_close(psi, ref)
        np.testing.assert_allclose(nrm, rn, rtol=1e-12)
        np.testing.assert_allclose(en, re, rtol=1e-10, atol=1e-12)


def test_long_chain_beyond_deep_offsets_uses_pairs(torch, cheb, depth_env):
    # (1 + 14) * n * 16 B exceeds 2^31: the deep kernel's 32-bit offsets would
    # wrap, so the plan keeps to two-order passes, also when a depth is forced
    n = 9_000_000
    x, dx = W.chain_grid(n, -0.01 * n, 0.01 * n)
    V = torch.from_numpy(W.harmonic(x, 1e-3)).cuda()
    for depth in (None, 3, 6):
        depth_env(depth)
        ctx = cheb.Context()
        ctx.chain1d(V, dx)
        lo, hi = ctx.gershgorin()
        ctx.set_bounds(lo, hi, 0.01)
        M = ctx.plan(0.002)
        passes = ctx.plan_passes()
        assert sum(passes) == M and set(passes) <= {1, 2}
        ms, name, orders = ctx.time_recursion_kernel(2)
        assert name.startswith("k_pair") and orders == 2
        psi0 = W.random_state(n, 9)
        psi = torch.from_numpy(psi0).cuda()
        nrm = torch.zeros(2, dtype=torch.float64, device="cuda")
        say(f"[gpu] 9M chain, pairs path, forced depth {depth}")
        ctx.propagate(psi, 2, nrm, None, 0)
        torch.cuda.synchronize()
        assert abs(host(nrm)[1] / host(nrm)[0] - 1.0) < 1e-12
        # sampled sites against the oracle (windows around each site): both
        # ends, the last pair-walk strip and seeded interior sites
        plan = O.Plan(lo, hi, 0.002)
        assert plan.M == M
        sites = np.unique(np.concatenate([[0, 1, 61, 62, n // 2, n - 63, n - 2, n - 1],
                                          (W.uniform01(5, 40) * n).astype(np.int64)]))
        ref = chain_sites(W.harmonic(x, 1e-3), dx, psi0, plan, 2, sites)
        got = host(psi)[sites]
        assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
        ctx.close()


def test_deep_tall_chunks_from_16M_sites(torch, cheb, depth_env):
    # from 16M sites five- and six-order passes walk 52- and 56-row chunks
    # with streaming stores: one step of a 512 x 32768 ribbon from a dense
    # state against the oracle, site by site
    case = honey_case(512, 32768, "zigzag", 0.5, 4, state="dense")
    ref = None
    for depth in (None, 6):
        depth_env(depth)
        say(f"[gpu] 512x32768 dense, depth {depth}")
        ctx, psi, nrm, _, plan = run(torch, cheb, case, 1.0, 1)
        passes = ctx.plan_passes()
        assert plan.M == 20 and sum(passes) == 20
        if depth is None:
            assert passes == [5, 5, 5, 5]
            ref = O.propagate(case["H"], plan, case["psi0"], 1)
        else:
            assert 6 in passes
        ctx.close()
        assert_state_close(psi, ref)
        assert abs(nrm[0] - 1.0) < 1e-12


@pytest.mark.parametrize("edge", ["zigzag", "armchair"])
def test_deep_64M_sites_sampled(torch, cheb, depth_env, edge):
    # the 1024 x 65536 point of the ribbon size sweep (64M sites, 1 GiB per
    # vector) in the passes the plan picks there, from a dense state: sampled
    # sites (corners, borders, strip boundaries, seeded interior) against the
    # oracle on windows around each, and the norm
    w, l = 1024, 65536
    depth_env(None)
    eps = W.anderson_disorder(w, l, 0.5, 6)
    psi0 = W.random_state(w * l, 606)
    ctx = cheb.Context()
    eps_d = torch.from_numpy(eps).cuda()
    ctx.honeycomb(w, l, eps_d, edge=edge)
    lo, hi = ctx.gershgorin()
    ctx.set_bounds(lo, hi, 0.01)
    M = ctx.plan(1.0)
    psi = torch.from_numpy(psi0).cuda()
    nrm = torch.zeros(2, dtype=torch.float64, device="cuda")
    say(f"[gpu] 1024x65536 {edge} dense, passes {ctx.plan_passes()}")
    ctx.propagate(psi, 2, nrm, None, 0)
    torch.cuda.synchronize()
    n2 = host(nrm)
    assert abs(n2[0] - 1.0) < 1e-12 and abs(n2[1] - 1.0) < 1e-12
    sites = ribbon_sample_sites(w, l, 48, 17)
    idx = np.array([y * l + x for y, x in sites])
    got = host(psi)[idx]
    del psi
    ctx.close()
    plan = O.Plan(lo, hi, 1.0)
    assert plan.M == M
    ref = ribbon_sites(w, l, edge, eps, psi0, plan, 2, sites)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("edge", ["zigzag", "armchair"])
def test_deep_at_the_offset_limit_sampled(torch, cheb, depth_env, edge):
    # the largest ribbon the deep walk's 32-bit buffer offsets allow:
    # (W + 14) L 16 B = 2^31 exactly at 2034 x 65536 (133M sites), where the
    # rows past the lattice that the border walks address reach the top of
    # the offset range; two steps from a dense state in the passes the plan
    # picks, sampled sites (the last rows among them) against the oracle on
    # windows around each. One row more and the plan keeps to two-order passes.
    w, l = 2034, 65536
    assert (w + 14) * l * 16 == 1 << 31
    depth_env(None)
    eps = W.anderson_disorder(w, l, 0.5, 7)
    psi0 = W.random_state(w * l, 707)
    ctx = cheb.Context()
    eps_d = torch.from_numpy(eps).cuda()
    ctx.honeycomb(w, l, eps_d, edge=edge)
    lo, hi = ctx.gershgorin()
    ctx.set_bounds(lo, hi, 0.01)
    M = ctx.plan(1.0)
    passes = ctx.plan_passes()
    assert max(passes) >= 3 and sum(passes) == M
    psi = torch.from_numpy(psi0).cuda()
    nrm = torch.zeros(2, dtype=torch.float64, device="cuda")
    say(f"[gpu] 2034x65536 (offset limit) {edge} dense, passes {passes}")
    ctx.propagate(psi, 2, nrm, None, 0)
    torch.cuda.synchronize()
    n2 = host(nrm)
    assert abs(n2[0] - 1.0) < 1e-12 and abs(n2[1] - 1.0) < 1e-12
    sites = set(ribbon_sample_sites(w, l, 32, 23))
    u = W.uniform01(29, 12)
    for k in range(6):  # the last six rows, where the offsets are largest
        sites.add((w - 1 - k, int(u[2 * k] * l)))
        sites.add((w - 1 - k, l - 1 - int(u[2 * k + 1] * 64)))
    sites = sorted(sites)
    idx = np.array([y * l + x for y, x in sites])
    got = host(psi)[idx]
    del psi
    ctx.close()
    plan = O.Plan(lo, hi, 1.0)
    assert plan.M == M
    ref = ribbon_sites(w, l, edge, eps, psi0, plan, 2, sites)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
    # one row more: past the limit the plan keeps to two-order passes
    del eps_d
    torch.cuda.empty_cache()
    eps1 = torch.zeros((w + 1) * l, dtype=torch.float64, device="cuda")
    ctx = cheb.Context()
    ctx.honeycomb(w + 1, l, eps1, edge=edge)
    ctx.set_bounds(-3.0, 3.0, 0.01)
    assert ctx.plan(1.0) == 20
    assert set(ctx.plan_passes()) <= {1, 2}
    ctx.close()
