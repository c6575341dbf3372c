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

}  // namespace chebtd
