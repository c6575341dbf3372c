// Adjoint (reverse-mode) kernels for dL/dV of the on-site potential.
//
// The forward step of Sect. 2.2 (arXiv:0907.3022) is a polynomial
// p(H~) psi built by v_{k+1} = 2 H~ v_k - v_{k-1}.  Its reverse sweep runs
// the same three-term recursion backwards on the adjoint vectors:
//   u_M = conj(g_M) gbar,
//   u_k = conj(g_k) gbar + 2 H~ u_{k+1} - u_{k+2}   (1 <= k < M),
//   u_0 = conj(g_0) gbar + H~ u_1 - u_2,
// and every level adds its share of dL/dV_i = (1/a) Re[conj(u_1) v_0 +
// 2 sum_{k>=1} conj(u_{k+1}) v_k].  H~ is real symmetric for the stencils,
// so it is its own adjoint and the forward operators are reused unchanged.
#include <hip/hip_runtime.h>

#include "device_ops.h"
#include "internal.h"
#include "deep_walk.h"
#include "pair.h"
#include "pair_walk.h"

namespace chebtd {

// out = H~ vk (first) or 2 H~ vk - vkm1
__global__ __launch_bounds__(kBlock) void k_recompute_chain(OpChain op, const double2 *__restrict__ vk,
                                                            const double2 *__restrict__ vkm1,
                                                            double2 *__restrict__ out, int first)
{
    const int64_t i = ChainRow::row(op);
    if (i < 0) return;
    const double2 h2 = ChainRow::apply2(op, i, vk, vk[i]);
    out[i] = first ? cscale(0.5, h2) : csub(h2, vkm1[i]);
}

template <int EDGE>
__global__ __launch_bounds__(kBlock) void k_recompute_honey(OpHoney op, const double2 *__restrict__ vk,
                                                            const double2 *__restrict__ vkm1,
                                                            double2 *__restrict__ out, int first)
{
    int32_t x, y;
    const int64_t i = HoneyRow<EDGE>::row_xy(op, x, y);
    if (i < 0) return;
    const double2 h2 = HoneyRow<EDGE>::apply2(op, i, x, y, vk, vk[i]);
    out[i] = first ? cscale(0.5, h2) : csub(h2, vkm1[i]);
}

// u = g * gbar
__global__ __launch_bounds__(kBlock) void k_adj_init(const double2 *__restrict__ gbar, double2 g,
                                                     double2 *__restrict__ u, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) u[i] = cfma(g, gbar[i], make_double2(0.0, 0.0));
}

// One reverse level:
//   out_i = gk gbar_i + f H~ u1 |_i - u2_i        (f = 2, or 1 when half)
//   grad_i += (f/a) Re[conj(u1_i) vk_i]
// out may alias gbar (level 0 writes u_0 over gbar); u2 may be null.
__device__ __forceinline__ void level_body(int64_t i, double2 h2, double2 u1i, const double2 *u2,
                                           double2 *out, const double2 *gbar, const double2 *vk,
                                           double2 gk, int half, double gfac, double *grad)
{
    double2 hv = half ? cscale(0.5, h2) : h2;
    if (u2) hv = csub(hv, u2[i]);
    const double2 gb = gbar[i];
    const double2 v = vk[i];
    grad[i] += gfac * (u1i.x * v.x + u1i.y * v.y);
    out[i] = cfma(gk, gb, hv);
}

__global__ __launch_bounds__(kBlock) void k_adj_level_chain(OpChain op, const double2 *__restrict__ u1,
                                                            const double2 *u2, double2 *out,
                                                            const double2 *gbar, const double2 *__restrict__ vk,
                                                            double2 gk, int half, double gfac,
                                                            double *__restrict__ grad)
{
    const int64_t i = ChainRow::row(op);
    if (i < 0) return;
    const double2 ui = u1[i];
    level_body(i, ChainRow::apply2(op, i, u1, ui), ui, u2, out, gbar, vk, gk, half, gfac, grad);
}

template <int EDGE>
__global__ __launch_bounds__(kBlock) void k_adj_level_honey(OpHoney op, const double2 *__restrict__ u1,
                                                            const double2 *u2, double2 *out,
                                                            const double2 *gbar, const double2 *__restrict__ vk,
                                                            double2 gk, int half, double gfac,
                                                            double *__restrict__ grad)
{
    int32_t x, y;
    const int64_t i = HoneyRow<EDGE>::row_xy(op, x, y);
    if (i < 0) return;
    const double2 ui = u1[i];
    level_body(i, HoneyRow<EDGE>::apply2(op, i, x, y, u1, ui), ui, u2, out, gbar, vk, gk, half, gfac,
               grad);
}

// ---------------------------------------------------------------------------
// Two levels per pass (brick-wall lattices: ribbons, and the chain as a
// ribbon of one row), walked like the forward pair kernel (pair_walk.h).
// ---------------------------------------------------------------------------

// Forward vectors without accumulation: head v_1 = H~ psi, v_2 = 2 H~ v_1 -
// psi; else v_{k+1}, v_{k+2} from (v_{k-1}, v_k).
template <int EDGE, bool HEAD>
__global__ __launch_bounds__(256) void k_recompute_pair(OpPair op, const double2 *__restrict__ vkm1,
                                                        const double2 *__restrict__ vk, double2 *__restrict__ out1,
                                                        double2 *__restrict__ out2)
{
    const int32_t gw = __builtin_amdgcn_readfirstlane(logical_block(op.xcd_remap) * 4 + (int32_t)(threadIdx.x >> 6));
    const int32_t strip = gw % op.nstrips, chunk = gw / op.nstrips;
    const double2 zero = make_double2(0.0, 0.0);
    double nrm = 0.0, en = 0.0;
    if (chunk < op.nchunks)
        pair_walk<EDGE, HEAD, false>(op, strip, chunk, vkm1, vk, out1, out2, nullptr, zero, zero, zero, nullptr,
                                     nrm, en);
}

namespace {
// operands of one row loaded one iteration ahead (see pair_walk.h)
struct AdjPrefetch {
    double2 a, km1, ext, gb, vk, vkm1;
    double e, grad;
};
}  // namespace

// Reverse levels k and k-1 (k-1 >= 1) of the wavefront's strip and chunk:
//   u_k     = cg1 gbar + 2 H~ u_{k+1} - u_{k+2}  (rows ys-1 .. ye; halo rows
//             are recomputed, not stored)
//   u_{k-1} = cg2 gbar + 2 H~ u_k - u_{k+1}      (own rows)
//   grad   += gf (Re[conj(u_{k+1}) v_k] + Re[conj(u_k) v_{k-1}])
// with cg1 = conj(g_k), cg2 = conj(g_{k-1}), gf = 2/a; without HAS_U2,
// u_{k+2} = 0 (k = M-1).  Outputs go to buffers distinct from the inputs.
template <int EDGE, bool HAS_U2>
__device__ __forceinline__ void adj_pair_walk(const OpPair &op, int32_t strip, int32_t chunk,
                                              const double2 *__restrict__ uk2, const double2 *__restrict__ uk1,
                                              double2 *__restrict__ out1, double2 *__restrict__ out2,
                                              const double2 *__restrict__ gbar, const double2 *__restrict__ vk,
                                              const double2 *__restrict__ vkm1, double2 cg1, double2 cg2,
                                              double gf, double *__restrict__ grad)
{
    using namespace pairdev;
    const int lane = threadIdx.x & 63;
    const int32_t W = op.W, L = op.L;
    const int32_t x = strip * kPairStrip + lane - 1;
    const bool colok = x >= 0 && x < L;
    const bool own = colok && lane >= 1 && lane <= kPairStrip;
    const double2 zero = make_double2(0.0, 0.0);
    const int32_t ys = chunk * op.rows;
    const int32_t ye = min(ys + op.rows, W);
    auto okr = [&](int32_t r) -> bool { return colok && r >= 0 && r < W; };
    auto ld = [&](const double2 *v, int32_t r) -> double2 { return ldg(v, okr(r) ? (int64_t)r * L + x : 0); };
    auto ld_on = [&](int32_t r) -> double { return ldg(op.onsite, okr(r) ? (int64_t)r * L + x : 0); };
    const int32_t xe = lane == 0 ? x - 1 : x + 1;
    const bool ext_lane = (lane == 0 || lane == 63) && xe >= 0 && xe < L;
    auto ok_ext = [&](int32_t r) -> bool { return ext_lane && r >= 0 && r < W; };
    auto ld_ext = [&](int32_t r) -> double2 { return ldg(uk1, ok_ext(r) ? (int64_t)r * L + xe : 0); };
    double2 a_m1 = csel(okr(ys - 2), ld(uk1, ys - 2), zero);  // u_{k+1} rows r-1, r
    double2 a_0 = csel(okr(ys - 1), ld(uk1, ys - 1), zero);
    AdjPrefetch p0, p1;
    p0.a = ld(uk1, ys);
    p0.km1 = HAS_U2 ? ld(uk2, ys - 1) : zero;
    p0.gb = ld(gbar, ys - 1);
    p0.e = ld_on(ys - 1);
    p0.ext = ld_ext(ys - 1);
    p0.vk = p0.vkm1 = zero;
    p0.grad = 0.0;
    double2 b_m2 = zero, b_m1 = zero;  // u_k rows r-2, r-1
    double e_m1 = 0.0;                 // on-site term, row r-1
    double2 gb_m1 = zero;              // gbar, row r-1
    auto row_step = [&](int32_t r, const AdjPrefetch &cur, AdjPrefetch &nx) {
        nx.a = ld(uk1, r + 2);
        nx.km1 = HAS_U2 ? ld(uk2, r + 1) : zero;
        nx.gb = ld(gbar, r + 1);
        nx.e = ld_on(r + 1);
        nx.ext = ld_ext(r + 1);
        {
            const bool ok = own && r >= ys && r < ye;
            const int64_t io = ok ? (int64_t)r * L + x : 0;
            nx.vk = ldg(vk, io);
            nx.vkm1 = ldg(vkm1, io);
            nx.grad = ldg(grad, io);
        }
        const double2 a_p1 = csel(okr(r + 1), cur.a, zero);
        const double2 ext = csel(ok_ext(r), cur.ext, zero);
        const bool rowok = r >= 0 && r < W;
        const int64_t ir = (int64_t)r * L + x;
        // ---- level k at row r ----
        const double2 left = from_left(a_0, ext), right = from_right(a_0, ext);
        const bool even_r = ((x + r) & 1) == 0;
        double2 s;
        if (EDGE == CHEBTD_ZIGZAG)
            s = cadd(cadd(left, right), csel(even_r, a_p1, a_m1));
        else
            s = cadd(cadd(a_m1, a_p1), csel(even_r, right, left));
        const double d0 = op.s2 * (cur.e + op.dshift);
        const double2 h = make_double2(fma(d0, a_0.x, op.off2 * s.x), fma(d0, a_0.y, op.off2 * s.y));
        double2 b_0 = cfma(cg1, cur.gb, HAS_U2 ? csub(h, cur.km1) : h);
        b_0 = csel(colok && rowok, b_0, zero);
        if (own && r >= ys && r < ye) stg(out1, ir, b_0);
        // ---- level k-1 at row q = r-1 ----
        if (r - 1 >= ys) {
            const int32_t q = r - 1;
            const int64_t iq = (int64_t)q * L + x;
            const double2 l2 = from_left0(b_m1), r2 = from_right0(b_m1);
            const bool even_q = ((x + q) & 1) == 0;
            double2 s2;
            if (EDGE == CHEBTD_ZIGZAG)
                s2 = cadd(cadd(l2, r2), csel(even_q, b_0, b_m2));
            else
                s2 = cadd(cadd(b_m2, b_0), csel(even_q, r2, l2));
            const double d1 = op.s2 * (e_m1 + op.dshift);
            const double2 h2 = make_double2(fma(d1, b_m1.x, op.off2 * s2.x), fma(d1, b_m1.y, op.off2 * s2.y));
            const double2 c = cfma(cg2, gb_m1, csub(h2, a_m1));
            if (own) {
                stg(out2, iq, c);
                // own-row operands of row q were loaded with the previous row
                const double t1 = a_m1.x * cur.vk.x + a_m1.y * cur.vk.y;
                const double t2 = b_m1.x * cur.vkm1.x + b_m1.y * cur.vkm1.y;
                // grouped as two single-level updates, level k first, so
                // every pairing of the levels gives the same bits
                const double gk = cur.grad + gf * t1;
                stg(grad, iq, gk + gf * t2);
            }
        }
        a_m1 = a_0;
        a_0 = a_p1;
        b_m2 = b_m1;
        b_m1 = b_0;
        e_m1 = cur.e;
        gb_m1 = cur.gb;
    };
    int32_t r = ys - 1;
    for (; r + 1 <= ye; r += 2) {
        row_step(r, p0, p1);
        row_step(r + 1, p1, p0);
    }
    if (r <= ye) row_step(r, p0, p1);
}

template <int EDGE, bool HAS_U2>
__global__ __launch_bounds__(256) void k_adj_pair(OpPair op, const double2 *__restrict__ uk2,
                                                  const double2 *__restrict__ uk1, double2 *__restrict__ out1,
                                                  double2 *__restrict__ out2, const double2 *__restrict__ gbar,
                                                  const double2 *__restrict__ vk, const double2 *__restrict__ vkm1,
                                                  double2 cg1, double2 cg2, double gf, double *__restrict__ grad)
{
    const int32_t gw = __builtin_amdgcn_readfirstlane(logical_block(op.xcd_remap) * 4 + (int32_t)(threadIdx.x >> 6));
    const int32_t strip = gw % op.nstrips, chunk = gw / op.nstrips;
    if (chunk < op.nchunks)
        adj_pair_walk<EDGE, HAS_U2>(op, strip, chunk, uk2, uk1, out1, out2, gbar, vk, vkm1, cg1, cg2, gf, grad);
}

hipError_t launch_recompute_pair(const Ctx &c, hipStream_t s, bool head, const double2 *vkm1, const double2 *vk,
                                 double2 *out1, double2 *out2)
{
    const OpPair op = make_pair_op(c, c.pair_rows);
    const int64_t nb = pair_grid_blocks(c, c.pair_rows);
    if (nb <= 0 || nb > INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid((unsigned)nb), block(256);
    const bool zig = c.kind == HKind::Chain || c.edge == CHEBTD_ZIGZAG;
    if (head && zig)
        hipLaunchKernelGGL((k_recompute_pair<CHEBTD_ZIGZAG, true>), grid, block, 0, s, op, vkm1, vk, out1, out2);
    else if (head)
        hipLaunchKernelGGL((k_recompute_pair<CHEBTD_ARMCHAIR, true>), grid, block, 0, s, op, vkm1, vk, out1, out2);
    else if (zig)
        hipLaunchKernelGGL((k_recompute_pair<CHEBTD_ZIGZAG, false>), grid, block, 0, s, op, vkm1, vk, out1, out2);
    else
        hipLaunchKernelGGL((k_recompute_pair<CHEBTD_ARMCHAIR, false>), grid, block, 0, s, op, vkm1, vk, out1,
                           out2);
    return hipGetLastError();
}

hipError_t launch_adj_pair(const Ctx &c, hipStream_t s, bool has_u2, const double2 *uk2, const double2 *uk1,
                           double2 *out1, double2 *out2, const double2 *gbar, const double2 *vk,
                           const double2 *vkm1, double2 cg1, double2 cg2, double *grad)
{
    const OpPair op = make_pair_op(c, c.pair_rows);
    const int64_t nb = pair_grid_blocks(c, c.pair_rows);
    if (nb <= 0 || nb > INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid((unsigned)nb), block(256);
    const bool zig = c.kind == HKind::Chain || c.edge == CHEBTD_ZIGZAG;
    const double gf = 2.0 / c.a;
    if (zig && has_u2)
        hipLaunchKernelGGL((k_adj_pair<CHEBTD_ZIGZAG, true>), grid, block, 0, s, op, uk2, uk1, out1, out2, gbar, vk,
                           vkm1, cg1, cg2, gf, grad);
    else if (zig)
        hipLaunchKernelGGL((k_adj_pair<CHEBTD_ZIGZAG, false>), grid, block, 0, s, op, uk2, uk1, out1, out2, gbar,
                           vk, vkm1, cg1, cg2, gf, grad);
    else if (has_u2)
        hipLaunchKernelGGL((k_adj_pair<CHEBTD_ARMCHAIR, true>), grid, block, 0, s, op, uk2, uk1, out1, out2, gbar,
                           vk, vkm1, cg1, cg2, gf, grad);
    else
        hipLaunchKernelGGL((k_adj_pair<CHEBTD_ARMCHAIR, false>), grid, block, 0, s, op, uk2, uk1, out1, out2, gbar,
                           vk, vkm1, cg1, cg2, gf, grad);
    return hipGetLastError();
}

hipError_t launch_recompute(const Ctx &c, hipStream_t s, const double2 *vk, const double2 *vkm1,
                            double2 *vkp1, int first)
{
    const dim3 grid((unsigned)grid_blocks(c)), block(kBlock);
    if (c.kind == HKind::Chain)
        hipLaunchKernelGGL(k_recompute_chain, grid, block, 0, s, make_chain(c), vk, vkm1, vkp1, first);
    else if (c.kind == HKind::Honeycomb && c.edge == CHEBTD_ZIGZAG)
        hipLaunchKernelGGL(k_recompute_honey<CHEBTD_ZIGZAG>, grid, block, 0, s, make_honey(c), vk, vkm1,
                           vkp1, first);
    else if (c.kind == HKind::Honeycomb)
        hipLaunchKernelGGL(k_recompute_honey<CHEBTD_ARMCHAIR>, grid, block, 0, s, make_honey(c), vk, vkm1,
                           vkp1, first);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_adj_init(hipStream_t s, const double2 *gbar, double2 g, double2 *u, int64_t n)
{
    const int64_t nb = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_adj_init, dim3((unsigned)nb), dim3(kBlock), 0, s, gbar, g, u, n);
    return hipGetLastError();
}

// gscale: 2 for levels k >= 1 (2 H~), 1 for level 0 (H~)
hipError_t launch_adj_level(const Ctx &c, hipStream_t s, const double2 *u1, double2 *u2_in,
                            const double2 *gbar_in, double2 *out, const double2 *vk, double2 gk,
                            double gscale, int has_u2, double *grad)
{
    const dim3 grid((unsigned)grid_blocks(c)), block(kBlock);
    const int half = gscale == 1.0;
    const double gfac = gscale / c.a;
    const double2 *u2 = has_u2 ? u2_in : nullptr;
    if (c.kind == HKind::Chain)
        hipLaunchKernelGGL(k_adj_level_chain, grid, block, 0, s, make_chain(c), u1, u2, out, gbar_in, vk, gk,
                           half, gfac, grad);
    else if (c.kind == HKind::Honeycomb && c.edge == CHEBTD_ZIGZAG)
        hipLaunchKernelGGL(k_adj_level_honey<CHEBTD_ZIGZAG>, grid, block, 0, s, make_honey(c), u1, u2, out,
                           gbar_in, vk, gk, half, gfac, grad);
    else if (c.kind == HKind::Honeycomb)
        hipLaunchKernelGGL(k_adj_level_honey<CHEBTD_ARMCHAIR>, grid, block, 0, s, make_honey(c), u1, u2,
                           out, gbar_in, vk, gk, half, gfac, grad);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// D levels (orders) per pass: the deep walk of deep_walk.h in its
// recomputation and adjoint modes.
// ---------------------------------------------------------------------------

// Forward vectors, each level stored: head v_1 .. v_D from psi; else
// v_{k+1} .. v_{k+D} from (v_{k-1}, v_k).
template <int EDGE, int D, bool HEAD>
__global__ __launch_bounds__(256) void k_recompute_deep(OpPair op, DeepArgs<D> args)
{
    double nrm = 0.0, en = 0.0;
    deep_dispatch<EDGE, D, HEAD, kDeepAll>(op, args, nrm, en);
}

// Reverse levels k .. k-D+1 (all >= 1) from (u_{k+2}, u_{k+1}), writing
// u_{k-D+2}, u_{k-D+1} and adding the levels' shares to dL/dV.
template <int EDGE, int D>
__global__ __launch_bounds__(256) void k_adj_deep(OpPair op, DeepArgs<D> args)
{
    double nrm = 0.0, en = 0.0;
    deep_dispatch<EDGE, D, false, kDeepAdj>(op, args, nrm, en);
}

// Reverse levels k .. k-D+1 (>= 0) from (u_{k+2}, u_{k+1}) with the forward
// vectors run downwards beside them from (v_{k+1}, v_k): writes u_{k-D+2},
// u_{k-D+1}, v_{k-D+1}, v_{k-D} and adds the levels' shares to dL/dV.
template <int EDGE, int D>
__global__ __launch_bounds__(256) void k_rev_deep(OpPair op, DeepArgs<D> args)
{
    double nrm = 0.0, en = 0.0;
    deep_dispatch<EDGE, D, false, kDeepRev>(op, args, nrm, en);
}

namespace {

template <int D>
hipError_t launch_recompute_deep_d(const Ctx &c, hipStream_t s, int rows, bool head, const double2 *vkm1,
                                   const double2 *vk, double2 *const *all)
{
    const OpPair op = make_deep_op(c, rows, D);
    const int64_t nb = deep_grid_blocks(c, rows, D);
    if (nb <= 0 || nb > INT32_MAX || !deep_offsets_fit(op.W, op.L)) return hipErrorInvalidValue;
    DeepArgs<D> A{};
    A.vkm1 = vkm1;
    A.vk = vk;
    for (int j = 0; j < D; ++j) A.all[j] = all[j];
    const dim3 grid((unsigned)nb), block(256);
    const bool zig = c.kind == HKind::Chain || c.edge == CHEBTD_ZIGZAG;
    if (head && zig)
        hipLaunchKernelGGL((k_recompute_deep<CHEBTD_ZIGZAG, D, true>), grid, block, 0, s, op, A);
    else if (head)
        hipLaunchKernelGGL((k_recompute_deep<CHEBTD_ARMCHAIR, D, true>), grid, block, 0, s, op, A);
    else if (zig)
        hipLaunchKernelGGL((k_recompute_deep<CHEBTD_ZIGZAG, D, false>), grid, block, 0, s, op, A);
    else
        hipLaunchKernelGGL((k_recompute_deep<CHEBTD_ARMCHAIR, D, false>), grid, block, 0, s, op, A);
    return hipGetLastError();
}

template <int D>
hipError_t launch_adj_deep_d(const Ctx &c, hipStream_t s, int rows, const double2 *uk2, const double2 *uk1,
                             double2 *out1, double2 *out2, const double2 *gbar, double *grad,
                             const double2 *fwd, const double2 *cw)
{
    const OpPair op = make_deep_op(c, rows, D);
    const int64_t nb = deep_grid_blocks(c, rows, D);
    if (nb <= 0 || nb > INT32_MAX || !adj_deep_fits(c, D)) return hipErrorInvalidValue;
    DeepArgs<D> A{};
    A.vkm1 = uk2;
    A.vk = uk1;
    A.out1 = out1;
    A.out2 = out2;
    A.gbar = gbar;
    A.grad = grad;
    A.gf = 2.0 / c.a;
    A.fwd = fwd;
    for (int j = 0; j < D; ++j) A.w.g[j + 1] = cw[j];
    const dim3 grid((unsigned)nb), block(256);
    const bool zig = c.kind == HKind::Chain || c.edge == CHEBTD_ZIGZAG;
    if (zig)
        hipLaunchKernelGGL((k_adj_deep<CHEBTD_ZIGZAG, D>), grid, block, 0, s, op, A);
    else
        hipLaunchKernelGGL((k_adj_deep<CHEBTD_ARMCHAIR, D>), grid, block, 0, s, op, A);
    return hipGetLastError();
}

template <int D>
hipError_t launch_rev_deep_d(const Ctx &c, hipStream_t s, int rows, const RevPass &p)
{
    const OpPair op = make_deep_op(c, rows, D);
    const int64_t nb = deep_grid_blocks(c, rows, D);
    if (nb <= 0 || nb > INT32_MAX || !deep_offsets_fit(op.W, op.L)) return hipErrorInvalidValue;
    DeepArgs<D> A{};
    A.vkm1 = p.uk2;
    A.vk = p.uk1;
    A.out1 = p.out1;
    A.out2 = p.out2;
    A.gbar = p.gbar;
    A.grad = p.grad;
    A.gf = 2.0 / c.a;
    A.gfD = p.last0 ? 1.0 / c.a : 2.0 / c.a;
    A.hD = p.last0 ? 0.5 : 1.0;
    A.rv1 = p.v1;
    A.rv0 = p.v0;
    A.rout1 = p.vout1;
    A.rout2 = p.vout2;
    for (int j = 0; j < D; ++j) A.w.g[j + 1] = p.cw[j];
    const dim3 grid((unsigned)nb), block(256);
    const bool zig = c.kind == HKind::Chain || c.edge == CHEBTD_ZIGZAG;
    if (zig)
        hipLaunchKernelGGL((k_rev_deep<CHEBTD_ZIGZAG, D>), grid, block, 0, s, op, A);
    else
        hipLaunchKernelGGL((k_rev_deep<CHEBTD_ARMCHAIR, D>), grid, block, 0, s, op, A);
    return hipGetLastError();
}

}  // namespace

bool rev_deep_fits(const Ctx &c)
{
    if (!pair_supported(c)) return false;
    const OpPair op = make_pair_op(c, 1);
    return deep_offsets_fit(op.W, op.L);
}

hipError_t launch_rev_deep(const Ctx &c, hipStream_t s, int D, int rows, const RevPass &p)
{
    switch (D) {
        case 2: return launch_rev_deep_d<2>(c, s, rows, p);
        case 3: return launch_rev_deep_d<3>(c, s, rows, p);
        case 4: return launch_rev_deep_d<4>(c, s, rows, p);
        case 5: return launch_rev_deep_d<5>(c, s, rows, p);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_recompute_deep(const Ctx &c, hipStream_t s, int D, int rows, bool head, const double2 *vkm1,
                                 const double2 *vk, double2 *const *all)
{
    switch (D) {
        case 3: return launch_recompute_deep_d<3>(c, s, rows, head, vkm1, vk, all);
        case 4: return launch_recompute_deep_d<4>(c, s, rows, head, vkm1, vk, all);
        case 5: return launch_recompute_deep_d<5>(c, s, rows, head, vkm1, vk, all);
        case 6: return launch_recompute_deep_d<6>(c, s, rows, head, vkm1, vk, all);
        default: return hipErrorInvalidValue;
    }
}

bool adj_deep_fits(const Ctx &c, int D)
{
    const OpPair op = make_pair_op(c, 1);
    return deep_offsets_fit(op.W, op.L) && (int64_t)D * op.W * op.L * 16 <= (int64_t(1) << 30);
}

hipError_t launch_adj_deep(const Ctx &c, hipStream_t s, int D, int rows, const double2 *uk2, const double2 *uk1,
                           double2 *out1, double2 *out2, const double2 *gbar, double *grad,
                           const double2 *fwd, const double2 *cw)
{
    switch (D) {
        case 3: return launch_adj_deep_d<3>(c, s, rows, uk2, uk1, out1, out2, gbar, grad, fwd, cw);
        case 4: return launch_adj_deep_d<4>(c, s, rows, uk2, uk1, out1, out2, gbar, grad, fwd, cw);
        case 5: return launch_adj_deep_d<5>(c, s, rows, uk2, uk1, out1, out2, gbar, grad, fwd, cw);
        case 6: return launch_adj_deep_d<6>(c, s, rows, uk2, uk1, out1, out2, gbar, grad, fwd, cw);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace chebtd
