#!/usr/bin/env python3
"""Benchmark: Chebyshev time propagation on one MI355X.

The headline line times K time steps of the 128 x 8192 zigzag graphene
ribbon (1,048,576 sites, Anderson disorder W = 0.5, dt = 1, Chebyshev order
M = 20 from the 1e-15 Bessel cutoff).  One step is the whole hot path: the
step head (v_1 = H~ psi, acc = gamma_0 psi + gamma_1 v_1, norm and energy
reductions) and the recursion v_{k+1} = 2 H~ v_k - v_{k-1},
acc += gamma_{k+1} v_{k+1} up to order M, several orders per pass over memory
(the split the library plans, reported as config.orders_per_pass).  The plan (bounds,
Bessel weights, passes) is computed once per dt, outside the timed region, as
the method prescribes.

value = Hamiltonian applications (H~ v products) per second.
roofline: the dominant recursion kernel's algorithmic bytes (104 B per site
and pass, whatever the orders per pass: v_{k-1}, v_k, on-site term and acc
read, the last two vectors and acc written; 88 B per site for a
single-order pass) over its mean launch time measured with HIP events on the
library's stream.
cpu_baseline: the serial CPU oracle on a few steps of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
STENCIL_BYTES = 88       # per site and order: v_k, v_{k-1}, v_{k+1}, acc r/w, on-site term
PAIR_BYTES = 104         # per site and multi-order pass: v_{k-1}, v_k, on-site, acc r/w, last two vectors
CSR_VEC_BYTES = 80       # vector traffic per row and order for CSR
CSR_NNZ_BYTES = 20       # complex128 value + int32 column
CSR_ROW_BYTES = 8        # rowptr
HOL_CSR_BYTES = CSR_VEC_BYTES + 4 * CSR_NNZ_BYTES + CSR_ROW_BYTES  # the same rows stored as CSR


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash():
    """Hash of the multi-order kernels' source (the deep and pair walks, their
    launchers and the shared device helpers) with comments and whitespace
    removed: what the committed byte counters were measured on."""
    import re
    h = hashlib.sha256()
    for f in ("device_ops.h", "pair.hip", "pair_walk.h", "deep_walk.h", "pair.h"):
        with open(os.path.join(ROOT, "paper_0907_3022_amd", "csrc", f), encoding="utf-8") as fh:
            code = fh.read()
        code = re.sub(r"/\*.*?\*/", " ", code, flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()[:16]


def traffic_record(kernel):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    ent = rec.get(kernel)
    if not ent or ent.get("source_sha") != source_hash():
        return None
    return ent.get("bytes_per_launch")


def ribbon_context(torch, P, width, length, Wd, seed, edge="zigzag", dt=1.0):
    eps, psi0 = W.ribbon_inputs(width, length, Wd, seed, 20.0, 1.0)
    eps_d = torch.from_numpy(eps).cuda()
    psi = torch.from_numpy(psi0).cuda()
    ctx = P.Context()
    ctx.honeycomb(width, length, eps_d, edge=edge)
    lo, hi = ctx.gershgorin()
    ctx.set_bounds(lo, hi, 0.01)
    M = ctx.plan(dt)
    return ctx, eps_d, psi, M


def timed(torch, fn, reps=1):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


# ---------------------------------------------------------------------------
def bench_main(torch, P, steps, warmup, mode_flags):
    p = W.GRAPHENE.params
    ctx, eps_d, psi, M = ribbon_context(torch, P, p["width"], p["length"], p["W"], p["seed"],
                                        p["edge"], p["dt"])
    n = p["width"] * p["length"]
    nrm = torch.zeros(max(steps, warmup, 1), dtype=torch.float64, device="cuda")
    en = torch.zeros_like(nrm)
    flags = P.NO_CHECK | mode_flags
    if warmup:
        ctx.propagate(psi, warmup, nrm, en, flags)
    # timed region: exactly `steps` time steps with per-step norm and energy
    t = timed(torch, lambda: ctx.propagate(psi, steps, nrm, en, flags))
    nr = nrm[:steps].cpu().numpy()
    drift = float(np.abs(nr - nr[0]).max()) if steps else 0.0
    # dominant kernel timed alone with HIP events on the library's stream
    ms_iter, kname, orders = ctx.time_recursion_kernel(200)
    ms_single, kname_single, _ = ctx.time_recursion_kernel(200, P.SINGLE_ORDER)
    # the same run with one order per pass, for comparison
    psi2 = psi.clone()
    t_single = timed(torch, lambda: ctx.propagate(psi2, steps, nrm, en, flags | P.SINGLE_ORDER))
    return dict(ctx=ctx, n=n, M=M, seconds=t, ms_iter=ms_iter, kernel=kname, orders=orders,
                passes=ctx.plan_passes(),
                ms_single=ms_single, kernel_single=kname_single, seconds_single=t_single,
                norm_drift=drift, psi=psi, eps=eps_d)


def bench_mode_choice(torch, P):
    """Pick direct launches or hipGraph replay for the main run."""
    p = W.GRAPHENE.params
    ctx, eps_d, psi, M = ribbon_context(torch, P, p["width"], p["length"], p["W"], p["seed"],
                                        p["edge"], p["dt"])
    best = None
    for name, fl in (("direct", 0), ("graph", P.GRAPH)):
        ctx.propagate(psi, 10, None, None, P.NO_CHECK | fl)
        t = timed(torch, lambda: ctx.propagate(psi, 100, None, None, P.NO_CHECK | fl))
        log(f"[bench] launch mode {name}: {t / 100 * 1e3:.3f} ms/step")
        if best is None or t < best[1]:
            best = (name, t, fl)
    ctx.close()
    return best[0], best[2]


def bench_double_well(torch, P, K):
    p = W.DOUBLE_WELL.params
    x, dx, V, psi0 = W.double_well_inputs(p["n"], p["xmin"], p["xmax"], p["a"], p["b"], p["x0"],
                                          p["sigma"], p["k0"])
    ctx = P.Context()
    V_d = torch.from_numpy(V).cuda()
    ctx.chain1d(V_d, dx)
    lo, hi = ctx.gershgorin()
    ctx.set_bounds(lo, hi, 0.01)
    M = ctx.plan(p["dt"])
    psi = torch.from_numpy(psi0).cuda()
    nrm = torch.zeros(K, dtype=torch.float64, device="cuda")
    en = torch.zeros(K, dtype=torch.float64, device="cuda")
    ctx.propagate(psi, 2, nrm, en, P.NO_CHECK)  # warm-up
    psi = torch.from_numpy(psi0).cuda()
    t = timed(torch, lambda: ctx.propagate(psi, K, nrm, en, P.NO_CHECK))
    mask = torch.from_numpy((x > 0).astype(np.uint8)).cuda()
    T = float(ctx.region_sum(psi, mask).item())
    nr, e = nrm.cpu().numpy(), en.cpu().numpy()
    iters = K * M
    return dict(workload="double_well_1d_N4096", M=M, steps=K, seconds=t,
                orders_per_s=iters / t, us_per_order=t / iters * 1e6, transmission_x_gt_0=T,
                norm_drift=float(np.abs(nr - nr[0]).max()),
                energy_rel_drift=float(np.abs(e - e[0]).max() / abs(e[0])),
                bound="one wavefront per workgroup: per-order fp64 issue, plus a halo exchange every H orders")


def bench_table1(torch, P, t_end=40.0, target=1e-9, cn_dts=(2e-4, 1e-4), run_limit_s=30.0):
    """Table 1 comparison on the Sect. 3.1 double well (N = 4096): run time to
    t = 40 of the Chebyshev propagator (dt = 0.5) and of Crank-Nicolson at the
    step that keeps the wave function's real and imaginary parts within
    `target` of the Chebyshev result (continuum normalisation, the integral
    of |psi|^2 over x equal to 1).  CN's step follows from two coarse runs
    and its second order; the run at that step is timed when it is expected
    to take at most `run_limit_s`, else its time is the measured per-step
    time times the step count."""
    p = W.DOUBLE_WELL.params
    x, dx, V, psi0 = W.double_well_inputs(p["n"], p["xmin"], p["xmax"], p["a"], p["b"], p["x0"],
                                          p["sigma"], p["k0"])
    ctx = P.Context()
    V_d = torch.from_numpy(V).cuda()
    ctx.chain1d(V_d, dx)
    lo, hi = ctx.gershgorin()
    ctx.set_bounds(lo, hi, 0.01)
    dt_c = p["dt"]
    K = int(round(t_end / dt_c))
    M = ctx.plan(dt_c)
    psi = torch.from_numpy(psi0).cuda()
    ctx.propagate(psi, 1, None, None, P.NO_CHECK)  # warm-up
    psi = torch.from_numpy(psi0).cuda()
    t_cheb = timed(torch, lambda: ctx.propagate(psi, K, None, None, P.NO_CHECK))
    ref = psi.cpu().numpy()
    scale = 1.0 / np.sqrt(dx)

    def err(a):
        d = (a - ref) * scale
        return float(max(np.abs(d.real).max(), np.abs(d.imag).max()))

    # the Chebyshev result against itself at half the step
    M2 = ctx.plan(dt_c / 2)
    ph = torch.from_numpy(psi0).cuda()
    ctx.propagate(ph, 2 * K, None, None, P.NO_CHECK)
    cheb_self = err(ph.cpu().numpy())
    cn = []
    for dt in cn_dts:
        S = int(round(t_end / dt))
        pc = torch.from_numpy(psi0).cuda()
        ctx.crank_nicolson(pc, dt, 1)  # warm-up
        pc = torch.from_numpy(psi0).cuda()
        t = timed(torch, lambda: ctx.crank_nicolson(pc, dt, S))
        cn.append(dict(dt=dt, steps=S, seconds=t, us_per_step=t / S * 1e6,
                       max_abs_err=err(pc.cpu().numpy())))
    e1, e2 = cn[0]["max_abs_err"], cn[1]["max_abs_err"]
    order = float(np.log(e1 / e2) / np.log(cn_dts[0] / cn_dts[1]))
    dt_star = cn_dts[1] * (target / e2) ** 0.5
    S_star = int(np.ceil(t_end / dt_star))
    us_step = min(c["us_per_step"] for c in cn)
    est = S_star * us_step * 1e-6
    out = dict(workload="double_well_1d_N4096_t40", chebyshev=dict(dt=dt_c, M=M, steps=K,
               seconds=t_cheb, self_err_half_step=cheb_self, M_half_step=M2),
               crank_nicolson_runs=cn, cn_order=order, cn_dt_for_target=dt_star,
               cn_steps_for_target=S_star, target_abs_err=target, cn_us_per_step=us_step)
    if est <= run_limit_s:
        dt_star = t_end / S_star
        pc = torch.from_numpy(psi0).cuda()
        t = timed(torch, lambda: ctx.crank_nicolson(pc, dt_star, S_star))
        out.update(cn_seconds=t, cn_seconds_kind="measured", cn_err_at_target_step=err(pc.cpu().numpy()))
    else:
        out.update(cn_seconds=est, cn_seconds_kind="per-step time x steps")
    out["cn_over_chebyshev"] = out["cn_seconds"] / t_cheb
    out["paper_cn_over_chebyshev"] = 1871.0 / 4.8
    ctx.close()
    return out


def bench_holstein(torch, P, K):
    p = W.HOLSTEIN.params
    out = {}
    for g2 in p["g2"]:
        ctx = P.Context()
        ctx.holstein(p["L"], p["nph"], p["t"], p["w0"], np.sqrt(g2), 0.0, p["periodic"])
        lo, hi = ctx.gershgorin()
        ctx.set_bounds(lo, hi, 0.01)
        M = ctx.plan(p["dt"])
        n = ctx.n
        nconf = n // p["L"]
        psi = torch.from_numpy(W.holstein_vacuum_site(p["L"], 0, nconf)).cuda()
        ctx.propagate(psi, 5, None, None, P.NO_CHECK)
        psi = torch.from_numpy(W.holstein_vacuum_site(p["L"], 0, nconf)).cuda()
        t = timed(torch, lambda: ctx.propagate(psi, K, None, None, P.NO_CHECK))
        ms_iter, kname, _ = ctx.time_recursion_kernel(300)
        bytes_row, bytes_row_eager = hol_bytes(p["L"], kname)
        n_i, nph_i, chi = (v.cpu().numpy() for v in ctx.holstein_obs(psi))
        out[f"g2={g2}"] = dict(n=n, M=M, steps=K, seconds=t, hv_per_s=K * M / t,
                               kernel=kname, kernel_ms=ms_iter,
                               kernel_GBs=bytes_row * n / (ms_iter * 1e-3) / 1e9,
                               step_equivalent_GBs=bytes_row_eager * n / (ms_iter * 1e-3) / 1e9,
                               bytes_per_row_order=bytes_row, bytes_per_row_order_acc_every_order=bytes_row_eager,
                               csr_bytes_per_row_order=HOL_CSR_BYTES,
                               total_phonons=float(nph_i.sum()), electron_density_sum=float(n_i.sum()))
        ctx.close()
        # the same matrix stored as CSR, through the general CSR kernel
        rowptr, col, val = P.holstein_csr_host(p["L"], p["nph"], p["t"], p["w0"], np.sqrt(g2), 0.0,
                                               p["periodic"])
        r_d, c_d, v_d = (torch.from_numpy(a).cuda() for a in (rowptr, col, val))
        cs = P.Context()
        cs.csr(r_d, c_d, v_d)
        cs.set_bounds(lo, hi, 0.01)
        cs.plan(p["dt"])
        psi = torch.from_numpy(W.holstein_vacuum_site(p["L"], 0, nconf)).cuda()
        cs.propagate(psi, 5, None, None, P.NO_CHECK)
        psi = torch.from_numpy(W.holstein_vacuum_site(p["L"], 0, nconf)).cuda()
        t_csr = timed(torch, lambda: cs.propagate(psi, K, None, None, P.NO_CHECK))
        ms_csr, kname_csr, _ = cs.time_recursion_kernel(300)
        csr_bytes = HOL_CSR_BYTES - 32 + 32.0 / 3.0  # acc on one order in three
        out[f"g2={g2}"]["csr"] = dict(nnz=int(rowptr[-1]), seconds=t_csr, hv_per_s=K * M / t_csr,
                                      kernel=kname_csr, kernel_ms=ms_csr, bytes_per_row_order=csr_bytes,
                                      kernel_GBs=csr_bytes * n / (ms_csr * 1e-3) / 1e9,
                                      step_equivalent_GBs=HOL_CSR_BYTES * n / (ms_csr * 1e-3) / 1e9)
        cs.close()
    return out


def hol_bytes(L, kname):
    """Algorithmic bytes per state and order of the matrix-free Holstein walk
    as it runs: v_k, v_{k-1} read and v_{k+1} written (48), acc read and
    written (32) on one order in three (the walk adds three orders' weights at
    once), and, in the walk that reads them (k_iter_hol<false, ...>, chosen
    where the last-level cache holds them), the raise/lower tables (2 x
    int32), the occupation (uint8) and the configuration total (uint8 per L
    states); the walk that ranks the phonon partners itself
    (k_iter_hol<true, ...>) reads no table.  Second: the table walk updating
    acc every order, for comparison."""
    tables = 4 + 4 + 1 + 1.0 / L
    lazy = 48 + 32.0 / 3.0 + (0.0 if kname.startswith("k_iter_hol<true") else tables)
    eager = 48 + tables + 32
    return lazy, eager


def bench_polaron_paper(torch, P):
    """Sect. 3.3 / Fig. 3 at the paper's size: D = 622,751,220 states, the
    matrix-free Holstein operator, observables at the figure's times."""
    p = W.POLARON_PAPER.params
    L = p["L"]
    g, Delta = W.polaron_couplings(L, p["w0"], p["eps_p"], p["eps_p_barrier"], p["barrier_site"],
                                   p["barrier"])
    t0 = time.perf_counter()
    ctx = P.Context()
    ctx.holstein(L, p["nph"], p["t"], p["w0"], g, Delta, False)
    build_s = time.perf_counter() - t0
    n = ctx.n
    nconf = n // L
    psi = torch.zeros(n, dtype=torch.complex128, device="cuda")
    # bare electron packet with the phonon vacuum (configuration rank 0 of
    # every site's block of states, index site * nconf)
    packet = W.holstein_packet(L, 1, p["packet_site"], p["width"], p["k"])
    psi[::nconf] = torch.from_numpy(packet).cuda()
    lo, hi = ctx.gershgorin()
    ctx.set_bounds(lo, hi)
    M = ctx.plan(p["dt"])
    snaps = []
    t_prev, run_s = 0.0, 0.0
    n_i, nph_i, chi = (v.cpu().numpy() for v in ctx.holstein_obs(psi))
    snaps.append(dict(t=0.0, n=n_i.round(6).tolist(), nph=nph_i.round(6).tolist(), chi=chi.round(6).tolist()))
    norms = []
    for ts in p["snapshots"]:
        K = int(round((ts - t_prev) / p["dt"]))
        nrm = torch.zeros(K, dtype=torch.float64, device="cuda")
        run_s += timed(torch, lambda: ctx.propagate(psi, K, nrm, None, 0))
        norms.append(float(nrm.max().item()))
        t_prev = ts
        n_i, nph_i, chi = (v.cpu().numpy() for v in ctx.holstein_obs(psi))
        snaps.append(dict(t=ts, n=n_i.round(6).tolist(), nph=nph_i.round(6).tolist(),
                          chi=chi.round(6).tolist(), sum_n=float(n_i.sum())))
    ms_iter, kname, _ = ctx.time_recursion_kernel(30)
    orders = int(round(p["snapshots"][-1] / p["dt"])) * M
    bytes_row, bytes_row_eager = hol_bytes(L, kname)
    ctx.close()
    del psi
    torch.cuda.empty_cache()
    return dict(workload="polaron_L18_nph11", states=n, M=M, dt=p["dt"], build_seconds=build_s,
                propagate_seconds=run_s, orders=orders, hv_per_s=orders / run_s,
                kernel=kname, kernel_ms=ms_iter, kernel_GBs=bytes_row * n / (ms_iter * 1e-3) / 1e9,
                step_equivalent_GBs=bytes_row_eager * n / (ms_iter * 1e-3) / 1e9,
                bytes_per_row_order=bytes_row, bytes_per_row_order_acc_every_order=bytes_row_eager,
                device_GB=(3 * 16 + 9) * n / 1e9, snapshots=snaps, max_norm_deviation=max(abs(x - 1) for x in norms))


def bench_sweep(torch, P, sizes):
    res = []
    for width, length in sizes:
        ctx, eps_d, psi, M = ribbon_context(torch, P, width, length, 0.5, 1)
        ms, kname, orders = ctx.time_recursion_kernel(50)
        ms1, kname1, _ = ctx.time_recursion_kernel(50, P.SINGLE_ORDER)
        n = width * length
        per = PAIR_BYTES if orders >= 2 else STENCIL_BYTES
        res.append(dict(sites=n, shape=f"{width}x{length}", kernel=kname, kernel_ms=ms, passes=ctx.plan_passes(),
                        orders_per_launch=orders, GBs=per * n / (ms * 1e-3) / 1e9,
                        ns_per_site_order=ms * 1e6 / n / orders,
                        single_order_kernel_ms=ms1, single_order_GBs=STENCIL_BYTES * n / (ms1 * 1e-3) / 1e9))
        ctx.close()
        del eps_d, psi
        torch.cuda.empty_cache()
    return res


def bench_batched(torch, P, K, seq_steps=10):
    """256 uneven ribbons: one batched propagation vs the same systems one by one."""
    p = W.BATCHED.params
    descs = W.batched_ribbons(p["nsys"], p["seed_base"])
    systems, inputs = [], []
    probe = P.Context()
    for d in descs:
        eps, psi0 = W.ribbon_inputs(d.width, d.length, d.W, d.seed)
        eps_d = torch.from_numpy(eps).cuda()
        probe.honeycomb(d.width, d.length, eps_d)
        lo, hi = probe.gershgorin()
        systems.append(dict(width=d.width, length=d.length, eps=eps_d,
                            psi=torch.from_numpy(psi0).cuda(), emin=lo, emax=hi))
        inputs.append(psi0)
    probe.close()
    ctx = P.Context()
    ctx.batch_create(systems, p["dt"])
    Ms = ctx.batch_info()
    t0 = time.perf_counter()
    best = ctx.batch_autotune(os.path.join(tempfile.gettempdir(), "chebtd_batch_tune.txt"))
    tune_s = time.perf_counter() - t0
    site_orders = float(sum(s["width"] * s["length"] * int(M) for s, M in zip(systems, Ms)))
    ctx.batch_propagate(2, P.GRAPH | P.NO_CHECK)  # warm-up
    t = timed(torch, lambda: ctx.batch_propagate(K, P.GRAPH))
    # the same systems one after another through the single-system path
    one = P.Context()
    seq_t = 0.0
    for s in systems:
        one.honeycomb(s["width"], s["length"], s["eps"])
        one.set_bounds(s["emin"], s["emax"])
        one.plan(p["dt"])
        one.propagate(s["psi"], 1, None, None, P.NO_CHECK)
        seq_t += timed(torch, lambda: one.propagate(s["psi"], seq_steps, None, None, P.NO_CHECK))
    one.close()
    ctx.close()
    batched_rate = site_orders * K / t
    seq_rate = site_orders * seq_steps / seq_t
    mode = ["levels", "persistent", "pairs", "deep"][best[0]]
    # algorithmic bytes of one step: 88 per site and order, or 104 per site
    # and multi-order pass plus 88 for an odd tail (the deep schedule: the
    # fewest passes of `depth` or `depth` + 1 orders that cover M, else
    # M // depth passes taking up to one extra order each, then pairs)
    if mode in ("pairs", "deep"):
        depth = int(os.environ.get("CHEBTD_BATCH_DEPTH", "5")) if mode == "deep" else 2

        def passes(M):
            nd, ext = 0, 0
            if mode == "deep":
                E = depth + 1 if depth < 6 else 0
                if E and depth * (-(-M // E)) <= M:
                    nd = -(-M // E)
                    ext = M - depth * nd
                else:
                    nd = M // depth
                    ext = min(M - depth * nd, nd) if E else 0
            rest = M - nd * depth - ext
            return nd + rest // 2, rest % 2
        step_bytes = sum(s["width"] * s["length"] * (PAIR_BYTES * passes(int(M))[0] + STENCIL_BYTES * passes(int(M))[1])
                         for s, M in zip(systems, Ms))
    else:
        step_bytes = STENCIL_BYTES * site_orders
    return dict(workload="batched_256_ribbons", systems=len(systems),
                sites=int(sum(s["width"] * s["length"] for s in systems)),
                M_min=int(Ms.min()), M_max=int(Ms.max()), steps=K, seconds=t,
                schedule=dict(mode=mode, tile=best[1], block=best[2], wg_per_cu=best[3]),
                autotune_seconds=tune_s, site_orders_per_s=batched_rate,
                GBs=step_bytes * K / t / 1e9, GBs_at_88B_per_site_order=STENCIL_BYTES * batched_rate / 1e9,
                sequential_site_orders_per_s=seq_rate, sequential_steps=seq_steps,
                speedup_vs_sequential=batched_rate / seq_rate)


def bench_adjoint(torch, P, K):
    """dL/dV of the transmitted probability: backward time vs plain forward time."""
    p = W.ADJOINT.params
    out = {}
    cases = [("ribbon_256x4096", "honeycomb"), ("chain_65536", "chain")]
    for name, kind in cases:
        ctx = P.Context()
        if kind == "honeycomb":
            V, psi0 = W.ribbon_inputs(p["width"], p["length"], p["W"], 0)
            mask = W.right_half_mask_ribbon(p["width"], p["length"])
            Vd = torch.from_numpy(V).cuda()
            ctx.honeycomb(p["width"], p["length"], Vd)
        else:
            x, dx, V, psi0 = W.double_well_inputs(p["n1d"])
            mask = (x > 0).astype(np.float64)
            Vd = torch.from_numpy(V).cuda()
            ctx.chain1d(Vd, dx)
        lo, hi = ctx.gershgorin()
        ctx.set_bounds(lo, hi)
        a = 0.5 * 1.01 * (hi - lo)
        M = ctx.plan(30.5 / a)
        ctx.reserve_adjoint(K, P.ADJ_STEP)
        psi = torch.from_numpy(psi0).cuda()
        ctx.propagate(psi, 2, None, None, P.NO_CHECK)  # warm-up
        psi.copy_(torch.from_numpy(psi0).cuda())
        t_plain = timed(torch, lambda: ctx.propagate(psi, K, None, None, P.NO_CHECK))
        psi.copy_(torch.from_numpy(psi0).cuda())
        t_fwd = timed(torch, lambda: ctx.propagate(psi, K, None, None, P.NO_CHECK | P.KEEP_CHECKPOINTS))
        m = torch.from_numpy(mask).cuda()
        gbar = (2.0 * m * psi).contiguous()
        dV = torch.zeros_like(Vd)
        t_bwd = timed(torch, lambda: ctx.adjoint(gbar, dV))
        # memory-lean schedule on the same run
        ctx.reserve_adjoint(K, P.ADJ_SQRTM)
        psi.copy_(torch.from_numpy(psi0).cuda())
        ctx.propagate(psi, K, None, None, P.NO_CHECK | P.KEEP_CHECKPOINTS)
        gbar2 = (2.0 * m * psi).contiguous()
        dV2 = torch.zeros_like(Vd)
        t_bwd2 = timed(torch, lambda: ctx.adjoint(gbar2, dV2))
        # forward vectors regenerated downwards from each step's last two
        ctx.reserve_adjoint(K, P.ADJ_REVERSE)
        psi.copy_(torch.from_numpy(psi0).cuda())
        t_fwd3 = timed(torch, lambda: ctx.propagate(psi, K, None, None, P.NO_CHECK | P.KEEP_CHECKPOINTS))
        gbar3 = (2.0 * m * psi).contiguous()
        dV3 = torch.zeros_like(Vd)
        t_bwd3 = timed(torch, lambda: ctx.adjoint(gbar3, dV3))
        # the schedules group levels into passes differently: equal to rounding
        nv = float(dV.norm())
        sched_diff = float((dV - dV2).norm()) / nv if nv > 0 else 0.0
        rev_diff = float((dV - dV3).norm()) / nv if nv > 0 else 0.0
        # backward_s: the default schedule (forward vectors run downwards)
        out[name] = dict(n=int(Vd.numel()), M=M, steps=K, forward_s=t_plain,
                         forward_with_checkpoints_s=t_fwd3, backward_s=t_bwd3,
                         backward_over_forward=t_bwd3 / t_plain,
                         backward_step_s=t_bwd, backward_step_over_forward=t_bwd / t_plain,
                         forward_with_psi_checkpoints_s=t_fwd,
                         backward_sqrtM_s=t_bwd2, backward_sqrtM_over_forward=t_bwd2 / t_plain,
                         step_sqrtM_rel_diff=sched_diff, step_reverse_rel_diff=rev_diff,
                         transmission=float((m * psi.abs() ** 2).sum().item()))
        ctx.close()
    return out


def bench_table2(torch, P):
    """Table 2 shape: the armchair ribbon of 10 x 1000 atoms with one occupied
    site at its centre, propagated to t = 1e4 at dt = 1, 10 and 100.  Reports
    each run's time beside the paper's single-core times (context only), the
    order the 1e-15 cutoff gives (the paper's M are the empirical orders for
    agreement with exact results, not comparable), the three final states
    against each other (each step is exact to the cutoff, so they differ by
    rounding accumulated over the steps), the norm and how far the state
    spread (rms distance from the start column, participation fraction)."""
    p = W.TABLE2.params
    w, l = p["width"], p["length"]
    eps, psi0 = W.table2_inputs(w, l, p["W"], p["seed"])
    ctx = P.Context()
    eps_d = torch.from_numpy(eps).cuda()
    ctx.honeycomb(w, l, eps_d, edge=p["edge"], t=p["t"])
    lo, hi = ctx.gershgorin()
    ctx.set_bounds(lo, hi)
    x = np.tile(np.arange(l), w).astype(np.float64)
    x0 = l // 2
    runs, finals = [], []
    for dt, paper_s, paper_M in zip(p["dts"], (378.0, 97.0, 45.0), (104, 264, 1210)):
        M = ctx.plan(dt)
        K = int(round(p["t_end"] / dt))
        psi = torch.from_numpy(psi0).cuda()
        ctx.propagate(psi, 2, None, None, P.NO_CHECK | P.GRAPH)  # warm-up (captures the graph)
        psi = torch.from_numpy(psi0).cuda()
        t = timed(torch, lambda: ctx.propagate(psi, K, None, None, P.NO_CHECK | P.GRAPH))
        f = psi.cpu().numpy()
        finals.append(f)
        rho = np.abs(f) ** 2
        runs.append(dict(dt=dt, M=M, steps=K, seconds=t, passes=ctx.plan_passes(), paper_seconds=paper_s,
                         paper_M=paper_M, norm_deviation=abs(float(rho.sum()) - 1.0),
                         rms_distance_columns=float(np.sqrt((rho * (x - x0) ** 2).sum() / rho.sum())),
                         participation_fraction=float(rho.sum() ** 2 / (rho ** 2).sum() / rho.size)))
    ref = finals[0]
    for r, f in zip(runs[1:], finals[1:]):
        r["rel_l2_vs_dt1"] = float(np.linalg.norm(f - ref) / np.linalg.norm(ref))
    ctx.close()
    return dict(workload=W.TABLE2.name, W=p["W"], seed=p["seed"], runs=runs)


def bench_shard(torch, P, gpus=(1, 2, 4, 8), shapes=((128, 8192), (1024, 65536)), D=5):
    """One GPU's share of a ribbon cut into N slabs along its length (the
    sharding the design describes; the library runs on one GPU): the dominant
    pass timed on a slab of L/N columns plus D halo columns on each side that
    the pass recomputes (D = its orders, 5 for these M = 20 ribbons), and the
    halo a pass would exchange per side: D columns of v_{k-1} and v_k,
    2 D W 16 bytes.  No exchange is run or timed here."""
    out = []
    for (w, l) in shapes:
        for n in gpus:
            halo = D if n > 1 else 0
            cols = l // n + 2 * halo
            eps_d = torch.from_numpy(W.anderson_disorder(w, cols, 0.5, 11)).cuda()
            ctx = P.Context()
            ctx.honeycomb(w, cols, eps_d)
            lo, hi = ctx.gershgorin()
            ctx.set_bounds(lo, hi)
            M = ctx.plan(1.0)
            passes = ctx.plan_passes()
            assert max(passes) == D, passes
            ms, name, orders = ctx.time_recursion_kernel(100 if w * cols <= (1 << 22) else 20)
            ctx.close()
            del eps_d
            out.append(dict(ribbon=f"{w}x{l}", gpus=n, slab=f"{w}x{cols}", M=M, passes=passes, kernel=name,
                            us_per_pass=ms * 1e3, step_us_compute=ms * 1e3 * len(passes),
                            halo_bytes_per_pass_per_side=2 * halo * w * 16))
        torch.cuda.empty_cache()
    return out


def bench_triad(torch, total_bytes, reps):
    """A STREAM-style triad a = b + s c in float64 (torch's elementwise kernel)
    over three arrays of total_bytes together: 2 reads and 1 write per
    element.  Returns GB/s from HIP events around `reps` launches."""
    n = max(1, int(total_bytes) // 24)
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    c = torch.full_like(b, 0.5)
    a = torch.empty_like(b)
    for _ in range(3):
        torch.add(b, c, alpha=2.0, out=a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.add(b, c, alpha=2.0, out=a)
    e1.record()
    e1.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    return 24 * n / sec / 1e9


def bench_copy(torch, nbytes=1 << 30, reps=5):
    """A plain device copy of known size: the reference that scales the
    hardware byte counters (FETCH_SIZE, WRITE_SIZE) of the other kernels."""
    n = nbytes // 16
    src = torch.zeros(n, dtype=torch.complex128, device="cuda")
    dst = torch.empty_like(src)
    t = timed(torch, lambda: dst.copy_(src), reps)
    return dict(bytes_each_way=n * 16, reps=reps, GBs=2 * n * 16 * reps / t / 1e9)


def cpu_baseline(target_seconds=12.0):
    """The serial oracle on the first steps of the headline workload."""
    import oracle as O
    p = W.GRAPHENE.params
    eps, psi0 = W.ribbon_inputs(p["width"], p["length"], p["W"], p["seed"], 20.0, 1.0)
    H = O.honeycomb(p["width"], p["length"], eps, edge=p["edge"])
    lo, hi = H.gershgorin()
    plan = O.Plan(lo, hi, p["dt"])
    t0 = time.perf_counter()
    O.propagate(H, plan, psi0, 1)
    t1 = time.perf_counter() - t0
    steps = max(1, int(target_seconds / max(t1, 1e-3)))
    t0 = time.perf_counter()
    O.propagate(H, plan, psi0, steps)
    t = time.perf_counter() - t0
    cpu = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=steps * plan.M / t, unit="H·v/s", cores=1, kind="oracle",
                sample=f"{steps} time steps (M={plan.M}) of the 128x8192 zigzag ribbon, "
                       f"serial C oracle, {t:.1f} s; host CPU: {cpu}")


def _oracle_batch_system(args):
    """One batched ribbon through the serial oracle for `steps` steps (a
    worker of cpu_other_workloads' process pool): (site-orders, seconds)."""
    width, length, Wd, seed, dt, steps = args
    import oracle as O
    eps, psi0 = W.ribbon_inputs(width, length, Wd, seed)
    H = O.honeycomb(width, length, eps)
    plan = O.Plan(float(eps.min()) - 3.0, float(eps.max()) + 3.0, dt)
    t0 = time.perf_counter()
    O.propagate(H, plan, psi0, steps)
    return width * length * plan.M * steps, time.perf_counter() - t0


def cpu_other_workloads(gpu_extra):
    """The serial oracle on bounded samples of the other workloads, beside the
    GPU's rate for the same work: the double well and the Holstein ring on one
    core, and one step of all 256 batched ribbons over a pool of host cores."""
    import multiprocessing as mp

    import oracle as O
    out = {}
    # double well (config 1): a few steps of M = 7256
    p = W.DOUBLE_WELL.params
    x, dx, V, psi0 = W.double_well_inputs(p["n"], p["xmin"], p["xmax"], p["a"], p["b"], p["x0"],
                                          p["sigma"], p["k0"])
    H = O.chain1d(V, dx)
    lo, hi = H.gershgorin()
    plan = O.Plan(lo, hi, p["dt"])
    t0 = time.perf_counter()
    O.propagate(H, plan, psi0, 4)
    t = time.perf_counter() - t0
    row = dict(cores=1, sample=f"4 steps, M = {plan.M}", oracle_orders_per_s=4 * plan.M / t)
    if "double_well" in gpu_extra:
        row["gpu_orders_per_s"] = gpu_extra["double_well"]["orders_per_s"]
    out["double_well"] = row
    # Holstein ring (config 3), g^2 = 2
    p = W.HOLSTEIN.params
    H = O.holstein(p["L"], p["nph"], p["t"], p["w0"], np.sqrt(2.0), 0.0, p["periodic"])
    lo, hi = H.gershgorin()
    plan = O.Plan(lo, hi, p["dt"])
    psi0 = W.holstein_vacuum_site(p["L"], 0, O.holstein_nconf(p["L"], p["nph"]))
    t0 = time.perf_counter()
    O.propagate(H, plan, psi0, 2)
    t = time.perf_counter() - t0
    row = dict(cores=1, sample=f"2 steps, M = {plan.M}, D = {H.n}", oracle_hv_per_s=2 * plan.M / t)
    if "holstein" in gpu_extra:
        row["gpu_hv_per_s"] = gpu_extra["holstein"]["g2=2.0"]["hv_per_s"]
    out["holstein_ring"] = row
    # batched (config 4): one step of every ribbon, the systems spread over
    # a pool of host processes
    pb = W.BATCHED.params
    descs = W.batched_ribbons(pb["nsys"], pb["seed_base"])
    cores = max(1, min(16, os.cpu_count() or 1))
    jobs = [(d.width, d.length, d.W, d.seed, pb["dt"], 1) for d in descs]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_batch_system, jobs, chunksize=4)
    t = time.perf_counter() - t0
    row = dict(cores=cores, sample=f"1 step of all {len(descs)} ribbons, {cores} processes (pool start included)",
               oracle_site_orders_per_s=sum(r[0] for r in res) / t,
               oracle_site_orders_per_s_per_core=sum(r[0] for r in res) / sum(r[1] for r in res))
    if "batched" in gpu_extra:
        row["gpu_site_orders_per_s"] = gpu_extra["batched"]["site_orders_per_s"]
    out["batched"] = row
    return out


# ---------------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--sections",
                    default="main,double_well,table1,table2,holstein,batched,adjoint,polaron,sweep,shard,cpu")
    ap.add_argument("--mode", default="auto", choices=["auto", "direct", "graph"])
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(see the design notes for how the propagation would shard)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_0907_3022_amd as P
    P.load_library()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    sections = set(args.sections.split(","))

    if args.mode == "auto":
        mode_name, mode_flags = bench_mode_choice(torch, P)
    else:
        mode_name, mode_flags = args.mode, (P.GRAPH if args.mode == "graph" else 0)

    log(f"[bench] main: zigzag ribbon 128x8192, {args.steps} steps, warmup {args.warmup}, mode {mode_name}")
    r = bench_main(torch, P, args.steps, args.warmup, mode_flags)
    hv = args.steps * r["M"]
    value = hv / r["seconds"] if r["seconds"] > 0 else 0.0
    unit_bytes = PAIR_BYTES if r["orders"] >= 2 else STENCIL_BYTES
    achieved = unit_bytes * r["n"] / (r["ms_iter"] * 1e-3) / 1e9
    traffic = traffic_record(r["kernel"])
    line = {
        "metric": "H·v Chebyshev steps/s + achieved HBM GB/s; batched & adjoint vs plain",
        "value": value,
        "unit": "H·v/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["seconds"] / max(args.steps, 1) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "zigzag_ribbon_128x8192", "sites": r["n"], "disorder_W": 0.5,
                   "dt": 1.0, "chebyshev_order": r["M"], "time_steps": args.steps,
                   "launch_mode": mode_name, "orders_per_pass": r["passes"], "complex128": True},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": r["kernel"], "kernel_ms_per_launch": r["ms_iter"],
                     "orders_per_launch": r["orders"],
                     "algorithmic_bytes_per_launch": unit_bytes * r["n"]},
        "single_order": {"kernel": r["kernel_single"], "kernel_ms_per_launch": r["ms_single"],
                         "GBs": STENCIL_BYTES * r["n"] / (r["ms_single"] * 1e-3) / 1e9,
                         "hv_per_s": hv / r["seconds_single"]},
        "time_steps_per_s": args.steps / r["seconds"] if r["seconds"] > 0 else 0.0,
        "step_equivalent_GBs": STENCIL_BYTES * r["n"] * hv / r["seconds"] / 1e9 if r["seconds"] > 0 else 0.0,
        "norm_drift": r["norm_drift"],
    }
    r["ctx"].close()
    # measured ceilings: a plain streaming kernel over 3 GiB (HBM) and over the
    # footprint of one pass of the dominant kernel (resident in the 256 MB MALL
    # like the pass itself)
    footprint = unit_bytes * r["n"]
    tri_hbm = bench_triad(torch, 3 << 30, 20)
    tri_fp = bench_triad(torch, footprint, 400)
    line["roofline"]["measured_ceiling"] = {
        "kernel": "triad a = b + s*c, float64, torch elementwise",
        "GBs_3GiB": tri_hbm, "GBs_same_footprint": tri_fp, "footprint_bytes": footprint,
        "frac_of_same_footprint": achieved / tri_fp if tri_fp > 0 else None}
    extra = {}
    if "double_well" in sections:
        log("[bench] double well N=4096, 200 steps")
        extra["double_well"] = bench_double_well(torch, P, W.DOUBLE_WELL.params["K"])
    if "table1" in sections:
        log("[bench] double well to t = 40: Chebyshev vs Crank-Nicolson")
        extra["table1"] = bench_table1(torch, P)
    if "table2" in sections:
        log("[bench] armchair ribbon 10x1000 to t = 1e4 at dt = 1, 10, 100 (Table 2 shape)")
        extra["table2"] = bench_table2(torch, P)
    if "holstein" in sections:
        log("[bench] Holstein ring L=10, N_ph<=10, 500 steps")
        extra["holstein"] = bench_holstein(torch, P, W.HOLSTEIN.params["K"])
    if "batched" in sections:
        log("[bench] batched 256 ribbons, 200 steps")
        extra["batched"] = bench_batched(torch, P, W.BATCHED.params["K"])
    if "adjoint" in sections:
        log("[bench] adjoint, 100 steps, order ~64")
        extra["adjoint"] = bench_adjoint(torch, P, W.ADJOINT.params["K"])
    if "polaron" in sections:
        log("[bench] polaron at the paper's size (D = 622,751,220)")
        extra["polaron_paper"] = bench_polaron_paper(torch, P)
    if "sweep" in sections:
        log("[bench] ribbon size sweep")
        extra["sweep"] = bench_sweep(torch, P, [(128, 8192), (256, 16384), (512, 32768), (1024, 65536)])
        # the same pass where its working set streams HBM (the headline's fits
        # the last-level cache): the sweep's points from 16M sites
        hbm = [r for r in extra["sweep"] if r["sites"] >= (16 << 20)]
        line["roofline"]["hbm_regime"] = [
            {"shape": r["shape"], "kernel": r["kernel"], "kernel_ms_per_launch": r["kernel_ms"],
             "achieved": r["GBs"], "frac": r["GBs"] / HBM_PEAK_GBS,
             "frac_of_measured_ceiling": r["GBs"] / tri_hbm if tri_hbm > 0 else None} for r in hbm]
    if "shard" in sections:
        log("[bench] one GPU's share of a ribbon cut into 2, 4, 8 slabs")
        extra["shard"] = bench_shard(torch, P)
    if "copy" in sections:
        log("[bench] reference copy")
        extra["copy"] = bench_copy(torch)
    if "cpu" in sections:
        log("[bench] CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline()
        log("[bench] CPU oracle on the other workloads")
        extra["cpu_other_workloads"] = cpu_other_workloads(extra)
    else:
        line["cpu_baseline"] = None
    line["extra"] = extra
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
