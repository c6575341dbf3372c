// Crank-Nicolson, eq. (CN) of arXiv:0907.3022 (the comparison method of
// Sect. 2.2 and Table 1), for the tridiagonal 1D chain of Sect. 3.1:
//   (1 + i dt H/2) psi_{s+1} = (1 - i dt H/2) psi_s = 2 psi_s - A psi_s,
// with A = 1 + i dt H/2.  A does not change between steps, so its Thomas
// factors are computed once on the host: A = L U with unit lower bidiagonal L
// (multipliers m_j) and upper bidiagonal U (pivots d_j, super-diagonal o).
// Each step then solves two first-order linear recurrences,
//   y_j = r_j - m_j y_{j-1}                 (forward),
//   x_j = (y_j - o x_{j+1}) / d_j           (backward),
// with r = 2x - A x.  Each is a composition of affine maps z -> p z + q.
//
// One workgroup of 256 threads (one wavefront per SIMD) runs all S steps:
// thread t holds sites t*C .. t*C+C-1 of the state and their factors in
// registers, folds its chunk, and the chunk maps are combined by an inclusive
// scan inside each wavefront (DPP row shifts, then row broadcasts, or lane
// shuffles for the backward direction) and a 4-entry carry across wavefronts
// through LDS.  The map products of the scan do not depend on the step and
// come precomputed from the host; only the offsets move.  Three barriers per
// step; the chain never leaves the CU.
#include <hip/hip_runtime.h>

#include "cn.h"

namespace chebtd {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

// a + p * b
__device__ __forceinline__ double2 cfma(double2 p, double2 b, double2 a)
{
    return make_double2(fma(p.x, b.x, fma(-p.y, b.y, a.x)), fma(p.x, b.y, fma(p.y, b.x, a.y)));
}

// r - i*oim*b
__device__ __forceinline__ double2 sub_io(double2 r, double oim, double2 b)
{
    return make_double2(fma(oim, b.y, r.x), fma(-oim, b.x, r.y));
}

// DPP move of a double; lanes without a valid source (or outside the row mask) get 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ double2 dpp_c(double2 v)
{
    return make_double2(dpp_d<CTRL, ROWS>(v.x), dpp_d<CTRL, ROWS>(v.y));
}

__device__ __forceinline__ double2 shfl_c(double2 v, int src)
{
    return make_double2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

constexpr int kRowShr = 0x110, kRowShl = 0x100, kRowBcast15 = 0x142, kRowBcast31 = 0x143;

}  // namespace

template <int C>
__global__ __launch_bounds__(kCnThreads) void k_cn_chain(CnDev t, double2 *psi, int64_t S)
{
    __shared__ double2 fwd_tot[4], bwd_tot[4], edge_first[4], edge_last[4];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, row = lane >> 4;
    const double2 zero = make_double2(0.0, 0.0);
    const double oim = t.oim;
    double2 st[C], fa[C], invd[C];
    double aim[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = tid * C + c;
        st[c] = j < t.n ? psi[j] : zero;
        fa[c] = t.fa[c * kCnThreads + tid];
        invd[c] = t.invd[c * kCnThreads + tid];
        aim[c] = t.aim[c * kCnThreads + tid];
    }
    double2 fs[6], bs[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        fs[k] = t.fstage[k * kCnThreads + tid];
        bs[k] = t.bstage[k * kCnThreads + tid];
    }
    const double2 pex = t.pex[tid], qex = t.qex[tid];
    double2 ptot[4], qtot[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        ptot[w] = t.ptot[w];
        qtot[w] = t.qtot[w];
    }
    if (lane == 0) edge_first[wave] = st[0];
    if (lane == 63) edge_last[wave] = st[C - 1];
    __syncthreads();

    for (int64_t s = 0; s < S; ++s) {
        // right-hand side r = 2x - A x = x - i (aim x + oim (x_left + x_right)), in place
        double2 xl = shfl_c(st[C - 1], lane > 0 ? lane - 1 : 0);
        double2 xr = shfl_c(st[0], lane < 63 ? lane + 1 : 63);
        if (lane == 0) xl = wave > 0 ? edge_last[wave - 1] : zero;
        if (lane == 63) xr = wave < 3 ? edge_first[wave + 1] : zero;
        double2 prev = xl;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const double2 x = st[c];
            const double2 nx = (c + 1 < C) ? st[c + 1] : xr;
            const double sr = fma(aim[c], x.x, oim * (prev.x + nx.x));
            const double si = fma(aim[c], x.y, oim * (prev.y + nx.y));
            st[c] = make_double2(x.x + si, x.y - sr);
            prev = x;
        }
        // forward: fold the chunk from y_in = 0, scan the lanes' maps
        double2 b = zero;
#pragma unroll
        for (int c = 0; c < C; ++c) b = cfma(fa[c], b, st[c]);
        b = cfma(fs[0], dpp_c<kRowShr | 1, 0xF>(b), b);
        b = cfma(fs[1], dpp_c<kRowShr | 2, 0xF>(b), b);
        b = cfma(fs[2], dpp_c<kRowShr | 4, 0xF>(b), b);
        b = cfma(fs[3], dpp_c<kRowShr | 8, 0xF>(b), b);
        b = cfma(fs[4], dpp_c<kRowBcast15, 0xA>(b), b);
        b = cfma(fs[5], dpp_c<kRowBcast31, 0xC>(b), b);
        if (lane == 63) fwd_tot[wave] = b;
        __syncthreads();
        double2 carry = zero;
#pragma unroll
        for (int w = 0; w < 3; ++w)
            if (w < wave) carry = cfma(ptot[w], carry, fwd_tot[w]);
        double2 y = shfl_c(b, lane > 0 ? lane - 1 : 0);
        if (lane == 0) y = zero;
        y = cfma(pex, carry, y);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            y = cfma(fa[c], y, st[c]);
            st[c] = y;
        }
        // backward: fold the chunk from its high end with x_in = 0, scan downwards
        b = zero;
#pragma unroll
        for (int c = C - 1; c >= 0; --c) b = cmul(invd[c], sub_io(st[c], oim, b));
        b = cfma(bs[0], dpp_c<kRowShl | 1, 0xF>(b), b);
        b = cfma(bs[1], dpp_c<kRowShl | 2, 0xF>(b), b);
        b = cfma(bs[2], dpp_c<kRowShl | 4, 0xF>(b), b);
        b = cfma(bs[3], dpp_c<kRowShl | 8, 0xF>(b), b);
        {
            const double2 o4 = shfl_c(b, (row == 0 || row == 2) ? 16 * (row + 1) : lane);
            if (row == 0 || row == 2) b = cfma(bs[4], o4, b);
            const double2 o5 = shfl_c(b, row < 2 ? 32 : lane);
            if (row < 2) b = cfma(bs[5], o5, b);
        }
        if (lane == 0) bwd_tot[wave] = b;
        __syncthreads();
        carry = zero;
#pragma unroll
        for (int w = 3; w > 0; --w)
            if (w > wave) carry = cfma(qtot[w], carry, bwd_tot[w]);
        double2 x = shfl_c(b, lane < 63 ? lane + 1 : 63);
        if (lane == 63) x = zero;
        x = cfma(qex, carry, x);
#pragma unroll
        for (int c = C - 1; c >= 0; --c) {
            x = cmul(invd[c], sub_io(st[c], oim, x));
            st[c] = x;
        }
        if (lane == 0) edge_first[wave] = st[0];
        if (lane == 63) edge_last[wave] = st[C - 1];
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = tid * C + c;
        if (j < t.n) psi[j] = st[c];
    }
}

hipError_t launch_cn_chain(hipStream_t s, const CnDev &t, double2 *psi, int64_t S)
{
    const dim3 grid(1), block(kCnThreads);
    switch (t.chunk) {
        case 1: hipLaunchKernelGGL(k_cn_chain<1>, grid, block, 0, s, t, psi, S); break;
        case 2: hipLaunchKernelGGL(k_cn_chain<2>, grid, block, 0, s, t, psi, S); break;
        case 4: hipLaunchKernelGGL(k_cn_chain<4>, grid, block, 0, s, t, psi, S); break;
        case 8: hipLaunchKernelGGL(k_cn_chain<8>, grid, block, 0, s, t, psi, S); break;
        case 16: hipLaunchKernelGGL(k_cn_chain<16>, grid, block, 0, s, t, psi, S); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace chebtd
