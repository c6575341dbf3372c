"""Batched ribbons on the GPU: the three schedules, graph replay and the
autotuner against the CPU oracle (system by system) and against the
single-system path (bit for bit: the per-site arithmetic is the same)."""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from test_gpu_parity import assert_state_close
from windows import ribbon_sites

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


def make_systems(specs, torch, state="dense"):
    """specs: (width, length, W, seed, edge); bounds from the oracle's discs.
    state "dense": a seeded random state on every site of each ribbon;
    "packet": the injected Gaussian."""
    out = []
    for (w, l, Wd, seed, edge) in specs:
        eps, psi0 = W.ribbon_inputs(w, l, Wd, seed)
        if state == "dense":
            psi0 = W.random_state(w * l, 7000 + seed)
        H = O.honeycomb(w, l, eps, edge=edge)
        lo, hi = H.gershgorin()
        out.append(dict(width=w, length=l, edge=edge, eps_np=eps, psi0=psi0, H=H, emin=lo, emax=hi,
                        eps=torch.from_numpy(eps).cuda(), psi=torch.from_numpy(psi0.copy()).cuda()))
    return out


SMALL = [(1, 50, 0.3, 1, "zigzag"), (7, 300, 1.0, 2, "armchair"), (33, 129, 2.0, 3, "zigzag"),
         (40, 700, 0.1, 4, "zigzag"), (5, 1025, 0.5, 5, "armchair"), (16, 64, 1.5, 6, "zigzag"),
         (128, 40, 0.7, 7, "zigzag"), (2, 2, 0.9, 8, "armchair"), (64, 513, 1.2, 9, "zigzag"),
         (9, 999, 0.2, 10, "zigzag"), (31, 257, 1.9, 11, "armchair"), (3, 4097, 0.6, 12, "zigzag")]


def reset(systems, torch):
    for s in systems:
        s["psi"].copy_(torch.from_numpy(s["psi0"]).cuda())


@pytest.mark.parametrize("mode,tile,block,wg", [(0, 1024, 256, 1), (0, 512, 512, 1), (1, 1024, 256, 2),
                                                (1, 4096, 512, 4), (1, 256, 256, 8), (2, 1024, 256, 1),
                                                (2, 512, 512, 1), (3, 1024, 256, 1), (3, 512, 512, 1)])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_oracle(torch, cheb, mode, tile, block, wg, graph):
    systems = make_systems(SMALL, torch)
    ctx = cheb.Context()
    dt, K = 1.0, 5
    ctx.batch_create(systems, dt)
    ctx.batch_set_schedule(mode, tile, block, wg)
    say(f"[gpu] batch mode={mode} tile={tile} block={block} wg={wg} graph={graph}")
    ctx.batch_propagate(K, cheb.GRAPH if graph else 0)
    torch.cuda.synchronize()
    Ms = ctx.batch_info()
    for s, M in zip(systems, Ms):
        plan = O.Plan(s["emin"], s["emax"], dt)
        assert M == plan.M
        ref = O.propagate(s["H"], plan, s["psi0"], K)
        assert_state_close(s["psi"].cpu().numpy(), ref)


# degenerate systems beside ordinary ones: a single site (its bounds widened
# around its one eigenvalue), single columns and rows, a 2 x 2 cell; M differs
# between them, so the schedules' per-system pass counts differ too
DEGENERATE = [(1, 1, 0.4, 21, "zigzag"), (6, 1, 1.0, 22, "zigzag"), (5, 1, 1.0, 23, "armchair"),
              (1, 3, 0.8, 24, "armchair"), (2, 2, 1.3, 25, "zigzag"), (40, 300, 0.5, 26, "zigzag")]


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_batch_degenerate_systems_match_oracle(torch, cheb, mode):
    systems = make_systems(DEGENERATE, torch)
    for s in systems:
        if s["emax"] == s["emin"]:
            s["emin"], s["emax"] = s["emin"] - 1.0, s["emax"] + 1.0
    ctx = cheb.Context()
    dt, K = 1.0, 4
    ctx.batch_create(systems, dt)
    ctx.batch_set_schedule(mode, 1024, 256, 1)
    say(f"[gpu] batch of degenerate systems, mode={mode}")
    ctx.batch_propagate(K, cheb.GRAPH)
    torch.cuda.synchronize()
    Ms = ctx.batch_info()
    for s, M in zip(systems, Ms):
        plan = O.Plan(s["emin"], s["emax"], dt)
        assert M == plan.M
        ref = O.propagate(s["H"], plan, s["psi0"], K)
        assert_state_close(s["psi"].cpu().numpy(), ref)


def test_batch_packets_match_oracle(torch, cheb):
    # the injected packets of the batched workload through the default deep
    # schedule
    systems = make_systems(SMALL, torch, state="packet")
    ctx = cheb.Context()
    ctx.batch_create(systems, 1.0)
    ctx.batch_set_schedule(cheb.SCHED_DEEP, 1024, 256, 1)
    ctx.batch_propagate(3, cheb.GRAPH)
    torch.cuda.synchronize()
    for s in systems:
        ref = O.propagate(s["H"], O.Plan(s["emin"], s["emax"], 1.0), s["psi0"], 3)
        assert_state_close(s["psi"].cpu().numpy(), ref)


def single_system(torch, cheb, s, K, depth, passes=None):
    """One system through the single-system path; depth 2 keeps it on the
    two-orders and one-order kernels the batch shares, None lets the plan
    split the orders as it does by default.  passes (a list) receives the
    plan's orders per pass."""
    saved = os.environ.get("CHEBTD_DEPTH")
    if depth is None:
        os.environ.pop("CHEBTD_DEPTH", None)
    else:
        os.environ["CHEBTD_DEPTH"] = str(depth)
    try:
        one = cheb.Context()
        one.honeycomb(s["width"], s["length"], s["eps"], edge=s["edge"])
        one.set_bounds(s["emin"], s["emax"])
        one.plan(1.0)
        if passes is not None:
            passes.extend(one.plan_passes())
    finally:
        if saved is None:
            os.environ.pop("CHEBTD_DEPTH", None)
        else:
            os.environ["CHEBTD_DEPTH"] = saved
    p = torch.from_numpy(s["psi0"].copy()).cuda()
    one.propagate(p, K)
    torch.cuda.synchronize()
    return p.cpu().numpy()


def test_batch_equals_single_system_path_bitwise(torch, cheb):
    systems = make_systems(SMALL[:6], torch)
    ctx = cheb.Context()
    ctx.batch_create(systems, 1.0)
    ctx.batch_set_schedule(1, 2048, 256, 2)
    ctx.batch_propagate(4)
    torch.cuda.synchronize()
    for s in systems:
        got = s["psi"].cpu().numpy()
        np.testing.assert_array_equal(single_system(torch, cheb, s, 4, 2), got)
        # the default split (deep passes) rounds in another order
        ref = single_system(torch, cheb, s, 4, None)
        assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


def test_batch_autotune_restores_state_and_caches(torch, cheb, tmp_path):
    systems = make_systems(SMALL, torch)
    ctx = cheb.Context()
    ctx.batch_create(systems, 1.0)
    cache = str(tmp_path / "tune.txt")
    best = ctx.batch_autotune(cache)
    assert best[0] in (0, 1, 2, 3)
    for s in systems:
        np.testing.assert_array_equal(s["psi"].cpu().numpy(), s["psi0"])
    assert os.path.exists(cache) and len(open(cache).read().split()) == 5
    best2 = ctx.batch_autotune(cache)  # read back from the cache
    assert tuple(best2) == tuple(best)
    ctx.batch_propagate(3, cheb.GRAPH)
    torch.cuda.synchronize()
    s = systems[3]
    ref = O.propagate(s["H"], O.Plan(s["emin"], s["emax"], 1.0), s["psi0"], 3)
    assert_state_close(s["psi"].cpu().numpy(), ref)


def test_batch_rejects_bad_schedule(torch, cheb):
    systems = make_systems(SMALL[:2], torch)
    ctx = cheb.Context()
    ctx.batch_create(systems, 1.0)
    with pytest.raises(cheb.ChebError):
        ctx.batch_set_schedule(1, 1000, 256, 2)  # tile not a multiple of block
    with pytest.raises(cheb.ChebError):
        ctx.batch_set_schedule(5, 1024, 256, 2)


def batch_deep_split(M, D=5):
    """Orders per pass the batched deep schedule gives a system: the fewest
    passes of D or D + 1 orders (D + 1 first) when they cover M exactly,
    else M // D passes taking up to one extra order each, then two-order
    passes and a one-order tail."""
    E = D + 1 if D < 6 else 0
    if E and D * (-(-M // E)) <= M:
        npass = -(-M // E)
        ext = M - D * npass
    else:
        npass = M // D
        ext = min(M - D * npass, npass) if E else 0
    rest = M - D * npass - ext
    return [E] * ext + [D] * (npass - ext) + [2] * (rest // 2) + [1] * (rest % 2)


@pytest.mark.parametrize("rows", [None, "3", "22", "40"])
@pytest.mark.parametrize("K", [1, 2, 3])
def test_batch_deep_equals_single_system_path_bitwise(torch, cheb, monkeypatch, K, rows):
    # the fewest passes of five or six orders per system (M = 17 .. 22 here:
    # 6+6+5, 5+5+5+5, 6+5+5+5, 6+6+5+5), which is also how the single
    # system's default plan splits these M: the same passes in the same
    # order, hence the same bits.  A site's arithmetic does not depend on the
    # chunk heights (the batch's default, overrides, the single system's own)
    if rows is not None:
        monkeypatch.setenv("CHEBTD_BATCH_DEEP_ROWS", rows)
    systems = make_systems(SMALL, torch)
    ctx = cheb.Context()
    ctx.batch_create(systems, 1.0)
    ctx.batch_set_schedule(cheb.SCHED_DEEP, 1024, 256, 1)
    ctx.batch_propagate(K, cheb.GRAPH)
    torch.cuda.synchronize()
    Ms = ctx.batch_info()
    assert {6, 5} <= {d for M in Ms for d in batch_deep_split(int(M))}
    for s, M in zip(systems, Ms):
        passes = []
        got = single_system(torch, cheb, s, K, None, passes)
        assert passes == batch_deep_split(int(M))
        np.testing.assert_array_equal(got, s["psi"].cpu().numpy())


@pytest.mark.parametrize("depth", ["4", "6"])
def test_batch_deep_other_depths_match_oracle(torch, cheb, monkeypatch, depth):
    # CHEBTD_BATCH_DEPTH=4: passes of four or five orders; =6: passes of six
    # orders only (no deeper walk), then two-order passes and the tail
    monkeypatch.setenv("CHEBTD_BATCH_DEPTH", depth)
    systems = make_systems(SMALL, torch)
    ctx = cheb.Context()
    ctx.batch_create(systems, 1.0)
    ctx.batch_set_schedule(cheb.SCHED_DEEP, 1024, 256, 1)
    ctx.batch_propagate(3, cheb.GRAPH)
    torch.cuda.synchronize()
    for s in systems:
        ref = O.propagate(s["H"], O.Plan(s["emin"], s["emax"], 1.0), s["psi0"], 3)
        assert_state_close(s["psi"].cpu().numpy(), ref)


@pytest.mark.parametrize("K", [1, 2, 3])
def test_batch_pairs_equals_single_system_path_bitwise(torch, cheb, K):
    # both walk the ribbon with the same two-orders-per-pass code and finish
    # odd orders with the same one-order stencil; odd K ends in the copy back
    systems = make_systems(SMALL, torch)
    ctx = cheb.Context()
    ctx.batch_create(systems, 1.0)
    ctx.batch_set_schedule(cheb.SCHED_PAIRS, 1024, 256, 1)
    ctx.batch_propagate(K, cheb.GRAPH)
    torch.cuda.synchronize()
    Ms = ctx.batch_info()
    assert any(M % 2 for M in Ms) and any(M % 2 == 0 for M in Ms)
    for s in systems:
        np.testing.assert_array_equal(single_system(torch, cheb, s, K, 2), s["psi"].cpu().numpy())


def test_batch_pairs_needs_two_orders(torch, cheb):
    # a tiny dt gives M = 1 for a system: the pairs schedule is refused, the
    # others still run
    systems = make_systems(SMALL[:3], torch)
    ctx = cheb.Context()
    ctx.batch_create(systems, 1e-9)
    assert min(ctx.batch_info()) < 2
    with pytest.raises(cheb.ChebError, match="M >= 2"):
        ctx.batch_set_schedule(cheb.SCHED_PAIRS, 1024, 256, 1)
    ctx.batch_set_schedule(cheb.SCHED_LEVELS, 1024, 256, 1)
    ctx.batch_propagate(2)
    torch.cuda.synchronize()


def test_full_batched_config_sampled(torch, cheb):
    # 256 ribbons, widths 32-128, lengths 512-4096, W in [0.1, 2], each from a
    # dense random state: the levels and persistent schedules agree bit for
    # bit everywhere, the pairs and deep schedules to rounding site by site;
    # every system is checked against the oracle at sampled sites (corners,
    # far borders, seeded interior) from windows around them, and three whole
    # systems against the oracle
    p = W.BATCHED.params
    descs = W.batched_ribbons(p["nsys"], p["seed_base"])
    total = sum(d.n for d in descs)
    assert 3e7 < total < 7e7
    systems, inputs = [], []
    for d in descs:
        eps = W.anderson_disorder(d.width, d.length, d.W, d.seed)
        psi0 = W.random_state(d.n, 9000 + d.seed)
        inputs.append((eps, psi0))
        # Gershgorin discs of a zigzag brick wall (interior sites have 3 bonds)
        systems.append(dict(width=d.width, length=d.length, eps=torch.from_numpy(eps).cuda(),
                            psi=torch.from_numpy(psi0).cuda(), emin=float(eps.min()) - 3.0,
                            emax=float(eps.max()) + 3.0))

    def reset():
        for s, (_, psi0) in zip(systems, inputs):
            s["psi"].copy_(torch.from_numpy(psi0).cuda())

    ctx = cheb.Context()
    ctx.batch_create(systems, p["dt"])
    Ms = ctx.batch_info()
    assert 18 <= Ms.min() and Ms.max() <= 24
    say(f"[gpu] full batch: {len(descs)} systems, {total} sites, levels schedule")
    ctx.batch_set_schedule(0, 2048, 256, 1)
    ctx.batch_propagate(2)
    torch.cuda.synchronize()
    lev = [s["psi"].cpu().numpy() for s in systems]
    reset()
    say("[gpu] full batch: persistent schedule")
    ctx.batch_set_schedule(1, 4096, 256, 2)
    ctx.batch_propagate(2, cheb.GRAPH)
    torch.cuda.synchronize()
    for s, ref in zip(systems, lev):
        np.testing.assert_array_equal(s["psi"].cpu().numpy(), ref)
    for mode, tile, block, name in ((2, 2048, 256, "pairs"), (cheb.SCHED_DEEP, 1024, 512, "deep")):
        reset()
        say(f"[gpu] full batch: {name} schedule")
        ctx.batch_set_schedule(mode, tile, block, 1)
        ctx.batch_propagate(2, cheb.GRAPH)
        torch.cuda.synchronize()
        for s, ref in zip(systems, lev):
            assert_state_close(s["psi"].cpu().numpy(), ref, 1e-13)
    say("[gpu] full batch: oracle windows on every system")
    u = W.uniform01(321, 2 * len(descs))
    for j, d in enumerate(descs):
        eps, psi0 = inputs[j]
        plan = O.Plan(systems[j]["emin"], systems[j]["emax"], p["dt"])
        assert plan.M == Ms[j]
        sites = [(0, 0), (d.width - 1, d.length - 1), (d.width - 1, 0), (0, d.length - 1),
                 (int(u[2 * j] * d.width), int(u[2 * j + 1] * d.length))]
        ref = ribbon_sites(d.width, d.length, "zigzag", eps, psi0, plan, 2, sites)
        got = np.array([lev[j][y * d.length + x] for y, x in sites])
        assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max(), j
    sizes = np.array([d.n for d in descs])
    for j in (int(np.argmin(sizes)), int(np.argsort(sizes)[len(sizes) // 2]), 17):
        d = descs[j]
        eps, psi0 = inputs[j]
        H = O.honeycomb(d.width, d.length, eps)
        plan = O.Plan(systems[j]["emin"], systems[j]["emax"], p["dt"])
        ref = O.propagate(H, plan, psi0, 2)
        assert_state_close(lev[j], ref)


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_batch_rebinds_states_without_replanning(torch, cheb, mode):
    # the batch is built on one set of states; new states are passed per call
    # (the signature chebtd_batch_propagate(ctx, psi[], K, flags)), replayed
    # through the graph captured before the re-bind, and stay bound for the
    # next call
    systems = make_systems(SMALL, torch)
    ctx = cheb.Context()
    ctx.batch_create(systems, 1.0)
    ctx.batch_set_schedule(mode, 1024, 256, 2)
    ctx.batch_propagate(2, cheb.GRAPH)  # captures the graph on the first states
    torch.cuda.synchronize()
    first = [s["psi"].cpu().numpy() for s in systems]
    new0 = [W.random_state(s["width"] * s["length"], 31337 + j) for j, s in enumerate(systems)]
    new = [torch.from_numpy(p.copy()).cuda() for p in new0]
    say(f"[gpu] batch re-bind mode={mode}")
    ctx.batch_propagate(2, cheb.GRAPH, psi=new)
    ctx.batch_propagate(1, cheb.GRAPH)  # still bound to the new states
    torch.cuda.synchronize()
    for j, s in enumerate(systems):
        # the first states were left where the first call put them
        np.testing.assert_array_equal(s["psi"].cpu().numpy(), first[j])
        ref = O.propagate(s["H"], O.Plan(s["emin"], s["emax"], 1.0), new0[j], 3)
        assert_state_close(new[j].cpu().numpy(), ref)
    # and back to the first states
    ctx.batch_propagate(0, 0, psi=[s["psi"] for s in systems])
    ctx.batch_propagate(1)
    torch.cuda.synchronize()
    for j, s in enumerate(systems):
        ref = O.propagate(s["H"], O.Plan(s["emin"], s["emax"], 1.0), s["psi0"], 3)
        assert_state_close(s["psi"].cpu().numpy(), ref)
