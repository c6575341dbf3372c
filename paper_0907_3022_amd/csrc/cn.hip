// Crank-Nicolson, eq. (CN) of arXiv:0907.3022 (the comparison method of
// Sect. 2.2 and Table 1), for the tridiagonal 1D chain of Sect. 3.1:
//   (1 + i dt H/2) psi_{s+1} = (1 - i dt H/2) psi_s = 2 psi_s - A psi_s,
// with A = 1 + i dt H/2.  A does not change between steps, so its Thomas
// factors are computed once on the host: A = L U with unit lower bidiagonal L
// (multipliers m_j) and upper bidiagonal U (pivots d_j, super-diagonal o).
// Each step then solves two first-order linear recurrences,
//   y_j = r_j - m_j y_{j-1}                 (forward),
//   x_j = y_j / d_j - (o / d_j) x_{j+1}     (backward),
// which one wavefront evaluates as parallel scans of affine maps: each lane
// owns a contiguous chunk of the chain, folds it sequentially, and the
// lanes' chunk maps are combined by a Kogge-Stone scan across lanes whose
// map products are step-independent and precomputed.  The vectors live in
// LDS; all S steps run in one launch.
#include <hip/hip_runtime.h>

#include "cn.h"
#include "device_ops.h"

namespace chebtd {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ double2 shfl_c(double2 v, int src)
{
    return make_double2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

}  // namespace

// psi: complex[n] in/out; t: the step-independent tables of this chain.
__global__ __launch_bounds__(64) void k_cn_chain(CnDev t, double2 *psi, int64_t S)
{
    extern __shared__ double2 lds[];
    double2 *x = lds;          // current state
    double2 *y = lds + t.n;    // forward-sweep values
    const int lane = threadIdx.x;
    const int j0 = lane * t.chunk, j1 = min(j0 + t.chunk, t.n);
    for (int j = j0; j < j1; ++j) x[j] = psi[j];
    __syncthreads();
    const double2 zero = make_double2(0.0, 0.0);
    for (int64_t s = 0; s < S; ++s) {
        // right-hand side r = 2 x - A x, then the lane's forward fold with y_in = 0
        double2 b = zero;
        for (int j = j0; j < j1; ++j) {
            double2 ax = cmul(t.a[j], x[j]);
            double2 nb = zero;
            if (j > 0) nb = cadd(nb, x[j - 1]);
            if (j + 1 < t.n) nb = cadd(nb, x[j + 1]);
            ax = cadd(ax, cmul(t.o, nb));
            const double2 r = csub(cscale(2.0, x[j]), ax);
            b = cadd(cmul(t.fa[j], b), r);  // fa_j = -m_j
            y[j] = b;
        }
        // inclusive scan of the lanes' chunk maps (P, B): B += Pstage * B_left
        for (int d = 0; d < 6; ++d) {
            const double2 bl = shfl_c(b, lane - (1 << d) >= 0 ? lane - (1 << d) : lane);
            if (lane >= (1 << d)) b = cadd(b, cmul(t.fstage[d * 64 + lane], bl));
        }
        double2 yin = shfl_c(b, lane > 0 ? lane - 1 : 0);
        if (lane == 0) yin = zero;
        for (int j = j0; j < j1; ++j) y[j] = cadd(y[j], cmul(t.fpre[j], yin));
        __syncthreads();
        // backward sweep, lane chunks folded from their high end
        b = zero;
        for (int j = j1 - 1; j >= j0; --j) {
            b = cadd(cmul(t.ba[j], b), cmul(t.invd[j], y[j]));  // ba_j = -o/d_j
            x[j] = b;
        }
        for (int d = 0; d < 6; ++d) {
            const double2 br = shfl_c(b, lane + (1 << d) < 64 ? lane + (1 << d) : lane);
            if (lane + (1 << d) < 64) b = cadd(b, cmul(t.bstage[d * 64 + lane], br));
        }
        double2 xin = shfl_c(b, lane < 63 ? lane + 1 : 63);
        if (lane == 63) xin = zero;
        for (int j = j0; j < j1; ++j) x[j] = cadd(x[j], cmul(t.bpre[j], xin));
        __syncthreads();
    }
    for (int j = j0; j < j1; ++j) psi[j] = x[j];
}

hipError_t launch_cn_chain(hipStream_t s, const CnDev &t, double2 *psi, int64_t S)
{
    const size_t lds = 2 * (size_t)t.n * sizeof(double2);
    if (lds > 65536) {
        // above the default dynamic LDS limit: raise it for this kernel
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_cn_chain),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_cn_chain, dim3(1), dim3(64), lds, s, t, psi, S);
    return hipGetLastError();
}

}  // namespace chebtd
