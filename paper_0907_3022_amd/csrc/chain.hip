// Whole runs of a short 1D chain (Sect. 3.1 of arXiv:0907.3022, the double
// well on N <= 4096 grid points) in one workgroup: every step of the
// Chebyshev propagator (Sect. 2.2) with all vectors in registers.
//
// T = 256 or 512 threads (one or two wavefronts per SIMD); thread t owns
// sites t*R .. t*R+R-1.
// One recursion order is
//   X <- 2 H~ Y - X        (v_{k+1} written over v_{k-1} in place)
//   acc += g_{k+1} X
// so two orders per loop iteration swap the roles of the two register
// arrays without copies.  Neighbours across lanes move by DPP wave shifts;
// the first and last site of each wavefront go through LDS (double
// buffered), one barrier per order, and the interior sites are computed
// while those LDS reads are in flight.  Sites past the end of the chain have
// zero coefficients, so they stay zero and act as the Dirichlet boundary.
// The step weights are read from LDS when they fit there.
#include <hip/hip_runtime.h>

#include "device_ops.h"
#include "internal.h"
#include "pair_walk.h"

namespace chebtd {

namespace {


template <int R>
struct ChainRegs {
    double d[R];  // 2 (H_ii - b) / a
    double o[R];  // 2 H_{i,i+-1} / a (0 past the end)
};

}  // namespace

// G_LDS: the step weights gamma_0..gamma_M are copied to LDS first, so that
// reading them never waits behind a scalar-cache miss (scalar loads share a
// wait counter with LDS, and the per-order edge exchange waits on it).
template <int R, int T, bool G_LDS>
__global__ __launch_bounds__(T) void k_chain_small(OpChain op, const double2 *psi_in,
                                                               double2 *psi_out,
                                                               const double2 *__restrict__ gamma, int M,
                                                               int64_t K, double a, double b,
                                                               double *norm_out, double *energy_out,
                                                               double2 *ckpt)
{
    using namespace pairdev;
    constexpr int NW = T / 64;
    __shared__ double2 edge_lo[2][NW], edge_hi[2][NW];  // first / last site of each wavefront
    __shared__ double red[2 * NW];
    extern __shared__ double2 g_lds[];  // gamma_0..gamma_M when G_LDS
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int64_t row0 = (int64_t)tid * R;
    const double2 zero = make_double2(0.0, 0.0);
    ChainRegs<R> c;
    double2 A[R], B[R], acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = row0 + r;
        const bool ok = i < op.n;
        c.d[r] = ok ? op.s2 * (op.V[i] + op.dsh) : 0.0;
        c.o[r] = ok ? op.off2 : 0.0;
        B[r] = ok ? psi_in[i] : zero;
        A[r] = zero;
    }
    const double2 *gam = gamma;
    if (G_LDS) {
        for (int k = tid; k <= M; k += T) g_lds[k] = gamma[k];
        gam = g_lds;  // the barrier in the first publish() orders these writes
    }
    int buf = 0;
    auto publish = [&](const double2 (&X)[R]) {
        if (lane == 0) edge_lo[buf][wave] = X[0];
        if (lane == 63) edge_hi[buf][wave] = X[R - 1];
        __syncthreads();
    };
    // X <- 2 H~ Y - X (REC) or X <- H~ Y (head), from Y's edges in edge_*[buf]
    auto apply = [&](double2 (&X)[R], const double2 (&Y)[R], bool head) {
        // every lane reads the neighbouring wavefronts' edges (one broadcast
        // address each); lanes 0 and 63 use them
        const double2 el = edge_hi[buf][wave > 0 ? wave - 1 : 0];
        const double2 er = edge_lo[buf][wave < NW - 1 ? wave + 1 : NW - 1];
        const double2 l0 = from_left0(Y[R - 1]);  // lane l-1's last site
        const double2 rR = from_right0(Y[0]);     // lane l+1's first site
        auto row = [&](int r, double2 l, double2 rr) {
            const double sx = l.x + rr.x, sy = l.y + rr.y;
            if (head)
                X[r] = make_double2(0.5 * fma(c.d[r], Y[r].x, c.o[r] * sx), 0.5 * fma(c.d[r], Y[r].y, c.o[r] * sy));
            else
                X[r] = make_double2(fma(c.d[r], Y[r].x, fma(c.o[r], sx, -X[r].x)),
                                    fma(c.d[r], Y[r].y, fma(c.o[r], sy, -X[r].y)));
        };
#pragma unroll
        for (int r = 1; r + 1 < R; ++r) row(r, Y[r - 1], Y[r + 1]);
        const double2 left = csel(lane == 0, wave > 0 ? el : zero, l0);
        const double2 right = csel(lane == 63, wave < NW - 1 ? er : zero, rR);
        if (R == 1) {
            row(0, left, right);
        } else {
            row(0, left, Y[1]);
            row(R - 1, Y[R - 2], right);
        }
    };
    // orders of one step read gamma one iteration ahead (uniform loads)
    auto g_at = [&](int k) -> double2 { return gam[k < M ? k : M]; };

    publish(B);
    for (int64_t s = 0; s < K; ++s) {
        // head: A = v_1 = H~ psi, acc = g_0 psi + g_1 v_1, norm and energy
        apply(A, B, true);
        buf ^= 1;
        double nrm = 0.0, e = 0.0;
        const double2 g0 = gam[0];
        const double2 g1 = M >= 1 ? gam[1] : zero;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (ckpt && row0 + r < op.n) ckpt[(size_t)s * op.n + row0 + r] = B[r];
            nrm += B[r].x * B[r].x + B[r].y * B[r].y;
            e += B[r].x * A[r].x + B[r].y * A[r].y;
            acc[r] = cfma(g1, A[r], cfma(g0, B[r], zero));
        }
        block_sum2(nrm, e, red);
        if (tid == 0) {
            if (norm_out) norm_out[s] = nrm;
            if (energy_out) energy_out[s] = a * e + b * nrm;
        }
        publish(A);
        // orders 2 .. M: B holds v_{k-1}, A holds v_k, alternately
        int k = 1;
        double2 ga = g_at(2), gb = g_at(3);
        for (; k + 2 <= M; k += 2) {
            const double2 g2 = ga, g3 = gb;
            ga = g_at(k + 3);
            gb = g_at(k + 4);
            apply(B, A, false);  // v_{k+1} over v_{k-1}
            buf ^= 1;
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = cfma(g2, B[r], acc[r]);
            publish(B);
            apply(A, B, false);  // v_{k+2} over v_k
            buf ^= 1;
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = cfma(g3, A[r], acc[r]);
            publish(A);
        }
        if (k + 1 <= M) {  // one order left: v_M over v_{M-2}
            apply(B, A, false);
            buf ^= 1;
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = cfma(ga, B[r], acc[r]);
        }
        // psi_{s+1} = acc
#pragma unroll
        for (int r = 0; r < R; ++r) {
            B[r] = acc[r];
            A[r] = zero;
        }
        publish(B);
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (row0 + r < op.n) psi_out[row0 + r] = B[r];
}

bool chain_small_fits(int64_t n) { return n >= 1 && n <= 4096; }

namespace {

template <int R, int T>
hipError_t launch_chain_rt(const Ctx &c, hipStream_t s, const OpChain &op, double2 *psi, double2 *out,
                           const double2 *gamma_dev, int64_t K, double *norm_out, double *energy_out,
                           double2 *ckpt, bool g_lds, size_t dyn)
{
    if (g_lds) {
        if (dyn > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_chain_small<R, T, true>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL((k_chain_small<R, T, true>), dim3(1), dim3(T), dyn, s, op, psi, out, gamma_dev, c.M, K,
                           c.a, c.b, norm_out, energy_out, ckpt);
    } else {
        hipLaunchKernelGGL((k_chain_small<R, T, false>), dim3(1), dim3(T), 0, s, op, psi, out, gamma_dev, c.M, K,
                           c.a, c.b, norm_out, energy_out, ckpt);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_chain_small(const Ctx &c, hipStream_t s, double2 *psi, double2 *out,
                              const double2 *gamma_dev, int64_t K, double *norm_out,
                              double *energy_out, double2 *ckpt)
{
    const OpChain op = make_chain(c);
    // weights in LDS when they fit beside the kernel's own few hundred bytes
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c.device) != hipSuccess)
        max_lds = 65536;
    const size_t gbytes = (size_t)(c.M + 1) * sizeof(double2);
    const bool g_lds = gbytes + 1024 <= (size_t)max_lds;
    const size_t dyn = g_lds ? gbytes : 0;
    // two wavefronts per SIMD for the longer chains (one issues while the
    // other waits on the edge exchange; measured 15% faster at n = 4096),
    // one for the shorter ones
    const int64_t n = c.n;
    if (n > 1024) {
        if (n <= 512) return launch_chain_rt<1, 512>(c, s, op, psi, out, gamma_dev, K, norm_out, energy_out, ckpt, g_lds, dyn);
        if (n <= 1024) return launch_chain_rt<2, 512>(c, s, op, psi, out, gamma_dev, K, norm_out, energy_out, ckpt, g_lds, dyn);
        if (n <= 2048) return launch_chain_rt<4, 512>(c, s, op, psi, out, gamma_dev, K, norm_out, energy_out, ckpt, g_lds, dyn);
        if (n <= 4096) return launch_chain_rt<8, 512>(c, s, op, psi, out, gamma_dev, K, norm_out, energy_out, ckpt, g_lds, dyn);
        return hipErrorInvalidValue;
    }
    if (n <= 256) return launch_chain_rt<1, 256>(c, s, op, psi, out, gamma_dev, K, norm_out, energy_out, ckpt, g_lds, dyn);
    if (n <= 512) return launch_chain_rt<2, 256>(c, s, op, psi, out, gamma_dev, K, norm_out, energy_out, ckpt, g_lds, dyn);
    if (n <= 1024) return launch_chain_rt<4, 256>(c, s, op, psi, out, gamma_dev, K, norm_out, energy_out, ckpt, g_lds, dyn);
    if (n <= 2048) return launch_chain_rt<8, 256>(c, s, op, psi, out, gamma_dev, K, norm_out, energy_out, ckpt, g_lds, dyn);
    if (n <= 4096) return launch_chain_rt<16, 256>(c, s, op, psi, out, gamma_dev, K, norm_out, energy_out, ckpt, g_lds, dyn);
    return hipErrorInvalidValue;
}

}  // namespace chebtd
