// Whole runs of a short 1D chain (Sect. 3.1 of arXiv:0907.3022, the double
// well on N <= 4096 grid points) in one launch: every step of the Chebyshev
// propagator (Sect. 2.2) with all vectors in registers, in one workgroup
// (k_chain_small) or, past 128 sites, spread over workgroups of one
// wavefront that exchange halo strips every few dozen orders (k_chain_multi).
//
// k_chain_small:
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

#include <algorithm>
#include <cstdio>
#include <cstdlib>

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

// The same run spread over P workgroups for chains longer than one
// workgroup's share.  Workgroup w owns the S sites [w S, w S + S) and keeps
// H more on each side (local site j is chain site w S - H + j), all in
// registers as above.  A site's value after an order depends on its
// neighbours' values before it, so the sites a workgroup holds correctly
// shrink by one per order from each end: after at most H orders exactly its
// own S sites are right.  Then it writes its first and last H own sites of
// both vectors to `xbuf`, raises its epoch flag (release at agent scope),
// waits for its two neighbours' flags (acquire) and reads their strips into
// its halo.  Every site's arithmetic is that of the one-workgroup kernel.
//
// xbuf holds two epochs (even, odd): a workgroup writes epoch e + 2's strips
// only after its neighbours raised epoch e + 1, which they do after reading
// its epoch e strips.  Neighbours are at most one epoch apart, so any two
// workgroups at most P - 1, and a step takes at least one epoch; the
// per-step norm and energy partials therefore sit in a ring of kChainRing
// >= P + 1 steps, summed in workgroup order by the last workgroup to arrive.
// psi may be read and written in place: each workgroup reads its sites and
// halo at the start and counts itself in; none writes psi_out before all
// have.  Every wait is bounded in wall-clock time: past the limit the
// workgroup records a timeout, stops, and writes NaN to its sites.
struct ChainXDev {
    double2 *xbuf;     // [2 epochs][P][2 strips][2 vectors][H]
    int32_t *flags;    // [P] epochs published
    int32_t *sync;     // [kChainRing] step arrivals, then setup arrivals, then the timeout flag
    double *part;      // [kChainRing][P][2] norm and energy partials
    int32_t H, S, P;
    int64_t spin_limit;  // wall-clock ticks a wait may take
};

__global__ void k_chain_multi_clear(int32_t *flags, int32_t *sync, int P)
{
    for (int i = threadIdx.x; i < P; i += blockDim.x) flags[i] = 0;
    for (int i = threadIdx.x; i < kChainRing + 2; i += blockDim.x) sync[i] = 0;
}

template <int R, int T, bool G_LDS>
__global__ __launch_bounds__(T) void k_chain_multi(OpChain op, const double2 *psi_in, double2 *psi_out,
                                                   const double2 *__restrict__ gamma, int M, int64_t K,
                                                   double a, double b, double *norm_out, double *energy_out,
                                                   double2 *ckpt, ChainXDev x)
{
    using namespace pairdev;
    constexpr int NW = T / 64;
    __shared__ double2 edge_lo[2][NW], edge_hi[2][NW];
    __shared__ double red[2 * NW];
    __shared__ int32_t s_bad;
    extern __shared__ double2 g_lds[];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int32_t w = blockIdx.x, P = x.P, H = x.H, S = x.S;
    const int64_t base = (int64_t)w * S - H;  // chain site of local site 0
    const int32_t j0 = tid * R;
    const double2 zero = make_double2(0.0, 0.0);
    int32_t *const arrive = x.sync + kChainRing, *const timeout = x.sync + kChainRing + 1;
    double d[R], o[R];
    double2 A[R], B[R], acc[R];
    bool own[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t g = base + j0 + r;
        const bool in = g >= 0 && g < op.n;
        d[r] = in ? op.s2 * (op.V[g] + op.dsh) : 0.0;
        o[r] = in ? op.off2 : 0.0;
        B[r] = in ? psi_in[g] : zero;
        A[r] = zero;
        acc[r] = zero;
        own[r] = in && j0 + r >= H && j0 + r < H + S;
    }
    const double2 *gam = gamma;
    if (G_LDS) {
        for (int k = tid; k <= M; k += T) g_lds[k] = gamma[k];
        gam = g_lds;
    }
    if (tid == 0) s_bad = 0;
    // psi_in has been read by every thread before the workgroup counts itself in
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) __hip_atomic_fetch_add(arrive, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);

    int buf = 0;
    // a one-wavefront workgroup needs no edge exchange (and no barrier) per order
    auto publish = [&](const double2 (&X)[R]) {
        if constexpr (NW > 1) {
            if (lane == 0) edge_lo[buf][wave] = X[0];
            if (lane == 63) edge_hi[buf][wave] = X[R - 1];
            __syncthreads();
        }
    };
    auto apply = [&](double2 (&X)[R], const double2 (&Y)[R], bool head) {
        double2 el = zero, er = zero;
        if constexpr (NW > 1) {
            el = edge_hi[buf][wave > 0 ? wave - 1 : 0];
            er = edge_lo[buf][wave < NW - 1 ? wave + 1 : NW - 1];
        }
        const double2 l0 = from_left0(Y[R - 1]);
        const double2 rR = from_right0(Y[0]);
        auto row = [&](int r, double2 l, double2 rr) {
            const double sx = l.x + rr.x, sy = l.y + rr.y;
            if (head)
                X[r] = make_double2(0.5 * fma(d[r], Y[r].x, o[r] * sx), 0.5 * fma(d[r], Y[r].y, o[r] * sy));
            else
                X[r] = make_double2(fma(d[r], Y[r].x, fma(o[r], sx, -X[r].x)),
                                    fma(d[r], Y[r].y, fma(o[r], sy, -X[r].y)));
        };
#pragma unroll
        for (int r = 1; r + 1 < R; ++r) row(r, Y[r - 1], Y[r + 1]);
        // one wavefront: lanes 0 and 63 already read 0 from the shifts
        const double2 left = NW > 1 ? csel(lane == 0, wave > 0 ? el : zero, l0) : l0;
        const double2 right = NW > 1 ? csel(lane == 63, wave < NW - 1 ? er : zero, rR) : rR;
        if (R == 1) {
            row(0, left, right);
        } else {
            row(0, left, Y[1]);
            row(R - 1, Y[R - 2], right);
        }
    };
    // bounded wait until *flag >= need (thread 0); false past the limit or
    // once another workgroup has timed out
    auto wait_at_least = [&](int32_t *flag, int32_t need, int64_t t0) -> bool {
        int64_t spins = 0;
        // a limit of 0 gives up at once (set from the host to test the time-out path)
        while (x.spin_limit <= 0 || __hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
            if (x.spin_limit <= 0 || wall_clock64() - t0 > x.spin_limit ||
                ((++spins & 255) == 0 && __hip_atomic_load(timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                __hip_atomic_store(timeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        return true;
    };
    auto strip = [&](int e, int32_t wg, int side, int vec) -> double2 * {
        return x.xbuf + ((((size_t)(e & 1) * P + wg) * 2 + side) * 2 + vec) * (size_t)H;
    };
    // publish this workgroup's strips of (B, A), wait for the neighbours',
    // read them into the halo; false (uniformly) after a timeout
    int32_t ep = 0;
    auto exchange = [&]() -> bool {
        double2 *f0 = strip(ep, w, 0, 0), *f1 = strip(ep, w, 0, 1);
        double2 *l0 = strip(ep, w, 1, 0), *l1 = strip(ep, w, 1, 1);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int32_t j = j0 + r;
            if (j >= H && j < 2 * H) {
                f0[j - H] = B[r];
                f1[j - H] = A[r];
            }
            if (j >= S && j < S + H) {
                l0[j - S] = B[r];
                l1[j - S] = A[r];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        const int e = ep++;
        if (tid == 0) {
            __hip_atomic_store(&x.flags[w], ep, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const int64_t t0 = wall_clock64();
            bool ok = true;
            if (w > 0) ok = wait_at_least(&x.flags[w - 1], ep, t0);
            if (ok && w + 1 < P) ok = wait_at_least(&x.flags[w + 1], ep, t0);
            s_bad = ok ? 0 : 1;
        }
        __syncthreads();
        if (__builtin_amdgcn_readfirstlane(s_bad)) return false;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int32_t wl = w > 0 ? w - 1 : w, wr = w + 1 < P ? w + 1 : w;  // read only if they exist
        const double2 *lb0 = strip(e, wl, 1, 0), *lb1 = strip(e, wl, 1, 1);
        const double2 *rb0 = strip(e, wr, 0, 0), *rb1 = strip(e, wr, 0, 1);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int32_t j = j0 + r;
            if (j < H && w > 0) {
                B[r] = lb0[j];
                A[r] = lb1[j];
            }
            if (j >= H + S && w + 1 < P) {
                B[r] = rb0[j - H - S];
                A[r] = rb1[j - H - S];
            }
        }
        return true;
    };

    bool ok = true;
    publish(B);
    for (int64_t s = 0; s < K && ok; ++s) {
        if (ckpt) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (own[r]) ckpt[(size_t)s * op.n + base + j0 + r] = B[r];
        }
        // head: A = v_1 = H~ psi, acc = g_0 psi + g_1 v_1, own sites' norm and energy
        apply(A, B, true);
        buf ^= 1;
        double nrm = 0.0, en = 0.0;
        const double2 g0 = gam[0];
        const double2 g1 = M >= 1 ? gam[1] : zero;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            nrm += own[r] ? B[r].x * B[r].x + B[r].y * B[r].y : 0.0;
            en += own[r] ? B[r].x * A[r].x + B[r].y * A[r].y : 0.0;
            acc[r] = cfma(g1, A[r], cfma(g0, B[r], zero));
        }
        block_sum2(nrm, en, red);
        if (tid == 0 && (norm_out || energy_out)) {
            const int slot = (int)(s % kChainRing);
            double *pw = x.part + ((size_t)slot * P + w) * 2;
            pw[0] = nrm;
            pw[1] = en;
            if (__hip_atomic_fetch_add(&x.sync[slot], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == P - 1) {
                double sn = 0.0, se = 0.0;
                for (int i = 0; i < P; ++i) {
                    sn += x.part[((size_t)slot * P + i) * 2];
                    se += x.part[((size_t)slot * P + i) * 2 + 1];
                }
                if (norm_out) norm_out[s] = sn;
                if (energy_out) energy_out[s] = a * se + b * sn;
                __hip_atomic_store(&x.sync[slot], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        publish(A);
        // orders 2 .. M in pairs, at most H orders between exchanges (the head
        // counts as one); B holds v_{k-1}, A holds v_k at every exchange
        int left = H - 1;
        int k = 1;
        for (; k + 2 <= M; k += 2) {
            if (left < 2) {
                if (!(ok = exchange())) break;
                publish(A);
                left = H;
            }
            const double2 g2 = gam[k + 1], g3 = gam[k + 2];
            apply(B, A, false);
            buf ^= 1;
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = cfma(g2, B[r], acc[r]);
            publish(B);
            apply(A, B, false);
            buf ^= 1;
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = cfma(g3, A[r], acc[r]);
            publish(A);
            left -= 2;
        }
        if (!ok) break;
        if (k + 1 <= M) {  // one order left: v_M over v_{M-2}
            if (left < 1) {
                if (!(ok = exchange())) break;
                publish(A);
            }
            const double2 gm = gam[M];
            apply(B, A, false);
            buf ^= 1;
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = cfma(gm, B[r], acc[r]);
        }
        // psi_{s+1} = acc, right on the own sites; the halo comes from the neighbours
#pragma unroll
        for (int r = 0; r < R; ++r) {
            B[r] = acc[r];
            A[r] = zero;
        }
        if (s + 1 < K && !(ok = exchange())) break;
        publish(B);
    }
    // every workgroup has read psi_in before any writes psi_out
    if (ok) {
        if (tid == 0) s_bad = wait_at_least(arrive, P, wall_clock64()) ? 0 : 1;
        __syncthreads();
        ok = __builtin_amdgcn_readfirstlane(s_bad) == 0;
    }
    const double nan = __builtin_nan("");
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (own[r]) psi_out[base + j0 + r] = ok ? B[r] : make_double2(nan, nan);
}

bool chain_small_fits(int64_t n) { return n >= 1 && n <= 4096; }

// Workgroups of one wavefront: an order then needs no barrier, only lane
// shifts, and the run pays an exchange every H orders instead.  Measured on
// MI355X (quartic well on [-20, 20], dt = 0.5), orders per second: 6.6M at
// n = 400 and 5.6M at 1024 with two sites per lane and H = 40 (H = 32: 6.3M,
// 5.2M); 5.6M at 1500, 5.4M at 2048 and 5.3M at 4096 with four sites per lane
// and H = 80 (H = 64: 5.4M, 5.3M, 5.1M); the one-workgroup kernel runs 4.0M,
// 3.8M, 3.0M, 3.0M and 2.1M there.  CHEBTD_CHAIN_MULTI = "R,T,H" overrides,
// "0" keeps one workgroup.
ChainMultiCfg chain_multi_config(int64_t n)
{
    ChainMultiCfg cfg;
    int R = n <= 1024 ? 2 : 4, T = 64, H = n <= 1024 ? 40 : 80;
    if (const char *env = std::getenv("CHEBTD_CHAIN_MULTI"))
        if (std::sscanf(env, "%d,%d,%d", &R, &T, &H) != 3) R = 0;
    const bool shape = (R == 1 && T == 512) || (R == 2 && T == 256) || (R == 2 && T == 512) || (R == 4 && T == 256) ||
                       (R == 2 && T == 64) || (R == 4 && T == 64) || (R == 8 && T == 64) || (R == 4 && T == 128);
    // from 129 sites (below that one workgroup holds the chain with one site per lane)
    if (!shape || H < 2 || (H & 1) || R * T < 3 * H || n <= 128 || !chain_small_fits(n)) return cfg;
    const int64_t S = (int64_t)R * T - 2 * H, P = (n + S - 1) / S;
    if (P < 2 || P > kChainMaxWG) return cfg;
    cfg.R = R;
    cfg.T = T;
    cfg.H = H;
    cfg.S = S;
    cfg.P = P;
    return cfg;
}

namespace {
constexpr size_t kChainIntBytes = 1024;  // flags [kChainMaxWG], then sync [kChainRing + 2]
static_assert((kChainMaxWG + kChainRing + 2) * sizeof(int32_t) <= kChainIntBytes, "int area");

size_t chain_part_bytes(const ChainMultiCfg &cfg) { return (size_t)kChainRing * cfg.P * 2 * sizeof(double); }

ChainXDev chain_x_layout(const Ctx &c, const ChainMultiCfg &cfg, int64_t spin_limit)
{
    char *p = static_cast<char *>(c.chainx.p);
    ChainXDev x{};
    x.flags = reinterpret_cast<int32_t *>(p);
    x.sync = x.flags + kChainMaxWG;
    x.part = reinterpret_cast<double *>(p + kChainIntBytes);
    x.xbuf = reinterpret_cast<double2 *>(p + kChainIntBytes + chain_part_bytes(cfg));
    x.H = cfg.H;
    x.S = (int32_t)cfg.S;
    x.P = (int32_t)cfg.P;
    x.spin_limit = spin_limit;
    return x;
}
}  // namespace

size_t chain_multi_scratch_bytes(const ChainMultiCfg &cfg)
{
    if (cfg.R == 0) return 0;
    return kChainIntBytes + chain_part_bytes(cfg) + (size_t)2 * cfg.P * 4 * cfg.H * sizeof(double2);
}

// the several-workgroup run's timeout flag when it runs for this context
int32_t *chain_multi_timeout(const Ctx &c)
{
    const ChainMultiCfg cfg = chain_multi_config(c.n);
    if (cfg.R == 0 || !c.chainx.p || c.chainx.bytes < chain_multi_scratch_bytes(cfg)) return nullptr;
    return chain_x_layout(c, cfg, 0).sync + kChainRing + 1;
}

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

template <int R, int T>
hipError_t launch_chain_multi_rt(const Ctx &c, hipStream_t s, const OpChain &op, const ChainMultiCfg &cfg,
                                 double2 *psi, double2 *out, const double2 *gamma_dev, int64_t K,
                                 double *norm_out, double *energy_out, double2 *ckpt, bool g_lds, size_t dyn)
{
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c.device) != hipSuccess || khz <= 0)
        khz = 100000;
    // two seconds per wait; CHEBTD_CHAIN_SPIN (wall-clock ticks) shortens it
    // (0: every wait gives up at once)
    int64_t limit = (int64_t)khz * 1000 * 2;
    if (const char *env = std::getenv("CHEBTD_CHAIN_SPIN")) limit = std::max<int64_t>(0, std::atoll(env));
    const ChainXDev x = chain_x_layout(c, cfg, limit);
    hipLaunchKernelGGL(k_chain_multi_clear, dim3(1), dim3(128), 0, s, x.flags, x.sync, x.P);
    const dim3 grid((unsigned)cfg.P), block(T);
    if (g_lds) {
        if (dyn > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_chain_multi<R, T, true>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL((k_chain_multi<R, T, true>), grid, block, dyn, s, op, psi, out, gamma_dev, c.M, K, c.a,
                           c.b, norm_out, energy_out, ckpt, x);
    } else {
        hipLaunchKernelGGL((k_chain_multi<R, T, false>), grid, block, 0, s, op, psi, out, gamma_dev, c.M, K, c.a,
                           c.b, norm_out, energy_out, ckpt, x);
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
    const ChainMultiCfg cfg = chain_multi_config(c.n);
    if (cfg.R > 0 && c.chainx.p && c.chainx.bytes >= chain_multi_scratch_bytes(cfg)) {
        if (cfg.T == 64 && cfg.R == 2)
            return launch_chain_multi_rt<2, 64>(c, s, op, cfg, psi, out, gamma_dev, K, norm_out, energy_out, ckpt,
                                                g_lds, dyn);
        if (cfg.T == 64 && cfg.R == 4)
            return launch_chain_multi_rt<4, 64>(c, s, op, cfg, psi, out, gamma_dev, K, norm_out, energy_out, ckpt,
                                                g_lds, dyn);
        if (cfg.T == 64)
            return launch_chain_multi_rt<8, 64>(c, s, op, cfg, psi, out, gamma_dev, K, norm_out, energy_out, ckpt,
                                                g_lds, dyn);
        if (cfg.T == 128)
            return launch_chain_multi_rt<4, 128>(c, s, op, cfg, psi, out, gamma_dev, K, norm_out, energy_out, ckpt,
                                                 g_lds, dyn);
        if (cfg.R == 1)
            return launch_chain_multi_rt<1, 512>(c, s, op, cfg, psi, out, gamma_dev, K, norm_out, energy_out, ckpt,
                                                 g_lds, dyn);
        if (cfg.R == 2 && cfg.T == 256)
            return launch_chain_multi_rt<2, 256>(c, s, op, cfg, psi, out, gamma_dev, K, norm_out, energy_out, ckpt,
                                                 g_lds, dyn);
        if (cfg.R == 2)
            return launch_chain_multi_rt<2, 512>(c, s, op, cfg, psi, out, gamma_dev, K, norm_out, energy_out, ckpt,
                                                 g_lds, dyn);
        return launch_chain_multi_rt<4, 256>(c, s, op, cfg, psi, out, gamma_dev, K, norm_out, energy_out, ckpt,
                                             g_lds, dyn);
    }
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
