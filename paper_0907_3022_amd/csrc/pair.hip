// Two Chebyshev orders per pass over HBM for brick-wall lattices: the
// honeycomb ribbons of eq. (model) and, as a ribbon of width 1, the 1D
// finite-difference chain of Sect. 3.1 (arXiv:0907.3022, Sect. 2.2 recursion).
//
// One pass reads v_{k-1}, v_k, the on-site term and acc once and writes
// v_{k+1}, v_{k+2} and acc (104 B per site for two orders instead of
// 2 x 88 B).  Each wavefront owns a strip of 62 columns and a chunk of rows
// (pair_walk.h); wavefronts are numbered strip-fastest, so consecutive ones
// read adjacent memory.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "device_ops.h"
#include "internal.h"
#include "pair.h"
#include "pair_walk.h"
#include "deep_walk.h"

namespace chebtd {

template <int EDGE, bool HEAD>
__global__ __launch_bounds__(256) void k_pair(OpPair op, const double2 *__restrict__ vkm1,
                                              const double2 *__restrict__ vk, double2 *__restrict__ out1,
                                              double2 *__restrict__ out2, double2 *__restrict__ acc,
                                              double2 g0, double2 g1, double2 g2, double2 *__restrict__ ckpt,
                                              double *partials, NeFinal fin)
{
    __shared__ double red[2 * 4];
    if (!HEAD && fin.partials && blockIdx.x == 0) finalize_ne_block(fin, nullptr, red);
    const int32_t gw = __builtin_amdgcn_readfirstlane(logical_block(op.xcd_remap) * 4 + (int32_t)(threadIdx.x >> 6));
    const int32_t strip = gw % op.nstrips;
    const int32_t chunk = gw / op.nstrips;
    double nrm = 0.0, en = 0.0;
    if (chunk < op.nchunks)  // uniform per wavefront
        pair_walk<EDGE, HEAD>(op, strip, chunk, vkm1, vk, out1, out2, acc, g0, g1, g2, ckpt, nrm, en);
    if (HEAD) {
        block_sum2(nrm, en, red);
        if (threadIdx.x == 0) {
            partials[2 * blockIdx.x] = nrm;
            partials[2 * blockIdx.x + 1] = en;
        }
    }
}

template <int EDGE, int D, bool HEAD, bool NT>
__global__ __launch_bounds__(256) void k_deep(OpPair op, DeepArgs<D> args, double *partials, NeFinal fin)
{
    __shared__ double red[2 * 4];
    if (!HEAD && fin.partials && blockIdx.x == 0) finalize_ne_block(fin, nullptr, red);
    double nrm = 0.0, en = 0.0;
    deep_dispatch<EDGE, D, HEAD, kDeepProp, NT>(op, args, nrm, en);
    if (HEAD) {
        block_sum2(nrm, en, red);
        if (threadIdx.x == 0) {
            partials[2 * blockIdx.x] = nrm;
            partials[2 * blockIdx.x + 1] = en;
        }
    }
}

OpPair make_pair_op(const Ctx &c, int rows)
{
    OpPair op{};
    op.s2 = 2.0 / c.a;
    if (c.kind == HKind::Chain) {
        op.onsite = c.V;
        op.dshift = 1.0 / (c.dx * c.dx) - c.b;
        op.off2 = 2.0 * (-0.5 / (c.dx * c.dx)) / c.a;
        op.W = 1;
        op.L = (int32_t)c.n;
    } else {
        op.onsite = c.eps;
        op.dshift = -c.b;
        op.off2 = -2.0 * c.t_hop / c.a;
        op.W = (int32_t)c.W;
        op.L = (int32_t)c.L;
    }
    op.rows = rows < 1 ? 1 : rows;
    op.nstrips = (op.L + kPairStrip - 1) / kPairStrip;
    op.nchunks = (op.W + op.rows - 1) / op.rows;
    op.xcd_remap = 1;
    return op;
}

int64_t pair_grid_blocks(const Ctx &c, int rows)
{
    const OpPair op = make_pair_op(c, rows);
    const int64_t waves = (int64_t)op.nstrips * op.nchunks;
    return (waves + 3) / 4;
}

bool pair_supported(const Ctx &c)
{
    if (c.kind == HKind::Honeycomb) return c.L < (1 << 30) && c.W < (1 << 30);
    return c.kind == HKind::Chain && c.n < ((int64_t)1 << 31);
}

hipError_t launch_pair(const Ctx &c, hipStream_t s, int rows, bool head, const double2 *vkm1, const double2 *vk,
                       double2 *out1, double2 *out2, double2 *acc, double2 g0, double2 g1, double2 g2,
                       double2 *ckpt, double *partials, const NeFinal *fin_in)
{
    NeFinal fin{};
    if (fin_in && !head) fin = *fin_in;
    const OpPair op = make_pair_op(c, rows);
    const int64_t nb = pair_grid_blocks(c, rows);
    if (nb <= 0 || nb > INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid((unsigned)nb), block(256);
    const bool zig = c.kind == HKind::Chain || c.edge == CHEBTD_ZIGZAG;
    if (head) {
        if (zig)
            hipLaunchKernelGGL((k_pair<CHEBTD_ZIGZAG, true>), grid, block, 0, s, op, vkm1, vk, out1, out2, acc, g0,
                               g1, g2, ckpt, partials, fin);
        else
            hipLaunchKernelGGL((k_pair<CHEBTD_ARMCHAIR, true>), grid, block, 0, s, op, vkm1, vk, out1, out2, acc,
                               g0, g1, g2, ckpt, partials, fin);
    } else {
        if (zig)
            hipLaunchKernelGGL((k_pair<CHEBTD_ZIGZAG, false>), grid, block, 0, s, op, vkm1, vk, out1, out2, acc,
                               g0, g1, g2, ckpt, partials, fin);
        else
            hipLaunchKernelGGL((k_pair<CHEBTD_ARMCHAIR, false>), grid, block, 0, s, op, vkm1, vk, out1, out2, acc,
                               g0, g1, g2, ckpt, partials, fin);
    }
    return hipGetLastError();
}

}  // namespace chebtd

namespace chebtd {

OpPair make_deep_op(const Ctx &c, int rows, int D)
{
    OpPair op = make_pair_op(c, rows);
    op.nstrips = (op.L + deep_strip(D) - 1) / deep_strip(D);
    return op;
}

int64_t deep_grid_blocks(const Ctx &c, int rows, int D)
{
    const OpPair op = make_deep_op(c, rows, D);
    const int64_t waves = (int64_t)op.nstrips * op.nchunks;
    return (waves + 3) / 4;
}

namespace {

template <int D>
hipError_t launch_deep_d(const Ctx &c, hipStream_t s, int rows, bool head, const double2 *vkm1, const double2 *vk,
                         double2 *out1, double2 *out2, double2 *acc, const double2 *g, double2 *ckpt,
                         double *partials, const NeFinal *fin_in)
{
    const OpPair op = make_deep_op(c, rows, D);
    const int64_t nb = deep_grid_blocks(c, rows, D);
    if (nb <= 0 || nb > INT32_MAX || !deep_offsets_fit(op.W, op.L)) return hipErrorInvalidValue;
    DeepArgs<D> A{};
    A.vkm1 = vkm1;
    A.vk = vk;
    A.out1 = out1;
    A.out2 = out2;
    A.acc = acc;
    A.ckpt = ckpt;
    for (int j = 0; j <= D; ++j) A.w.g[j] = g[j];
    NeFinal fin{};
    if (fin_in && !head) fin = *fin_in;
    const dim3 grid((unsigned)nb), block(256);
    const bool zig = c.kind == HKind::Chain || c.edge == CHEBTD_ZIGZAG;
    const bool nt = deep_stream_stores(c);
    if (nt) {
        if (head && zig)
            hipLaunchKernelGGL((k_deep<CHEBTD_ZIGZAG, D, true, true>), grid, block, 0, s, op, A, partials, fin);
        else if (head)
            hipLaunchKernelGGL((k_deep<CHEBTD_ARMCHAIR, D, true, true>), grid, block, 0, s, op, A, partials, fin);
        else if (zig)
            hipLaunchKernelGGL((k_deep<CHEBTD_ZIGZAG, D, false, true>), grid, block, 0, s, op, A, partials, fin);
        else
            hipLaunchKernelGGL((k_deep<CHEBTD_ARMCHAIR, D, false, true>), grid, block, 0, s, op, A, partials, fin);
    } else if (head && zig) {
        hipLaunchKernelGGL((k_deep<CHEBTD_ZIGZAG, D, true, false>), grid, block, 0, s, op, A, partials, fin);
    } else if (head) {
        hipLaunchKernelGGL((k_deep<CHEBTD_ARMCHAIR, D, true, false>), grid, block, 0, s, op, A, partials, fin);
    } else if (zig) {
        hipLaunchKernelGGL((k_deep<CHEBTD_ZIGZAG, D, false, false>), grid, block, 0, s, op, A, partials, fin);
    } else {
        hipLaunchKernelGGL((k_deep<CHEBTD_ARMCHAIR, D, false, false>), grid, block, 0, s, op, A, partials, fin);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_deep(const Ctx &c, hipStream_t s, int D, int rows, bool head, const double2 *vkm1,
                       const double2 *vk, double2 *out1, double2 *out2, double2 *acc, const double2 *g,
                       double2 *ckpt, double *partials, const NeFinal *fin)
{
    switch (D) {
        case 3: return launch_deep_d<3>(c, s, rows, head, vkm1, vk, out1, out2, acc, g, ckpt, partials, fin);
        case 4: return launch_deep_d<4>(c, s, rows, head, vkm1, vk, out1, out2, acc, g, ckpt, partials, fin);
        case 5: return launch_deep_d<5>(c, s, rows, head, vkm1, vk, out1, out2, acc, g, ckpt, partials, fin);
        case 6: return launch_deep_d<6>(c, s, rows, head, vkm1, vk, out1, out2, acc, g, ckpt, partials, fin);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace chebtd
