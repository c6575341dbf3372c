// Batched propagation of many independent honeycomb ribbons of uneven size
// (the disorder-ensemble use of Sect. 3.2 of arXiv:0907.3022): every system
// has its own grid, on-site energies, spectral scale (a, b), order M and
// Bessel weights, and each system's sites are cut into tiles of `tile`
// consecutive site indices.
//
// Three schedules:
//  * levels:     one launch per recursion level; block b takes tile b of the
//                systems still active at that level (systems are sorted by
//                M, descending, so the active ones form a prefix).
//  * pairs:      one launch per two recursion orders; every system's
//                wavefronts walk its strips and row chunks as the
//                single-system two-orders-per-pass kernel does (pair_walk.h),
//                and systems with odd M finish with a one-order tail launch.
//  * persistent: one launch per time step; resident workgroups pull
//                (level, system, tile) items from a queue ordered level by
//                level.  Before a tile of level k runs, every tile of level
//                k-1 of the same system must be done; per-system completion
//                counters (release/acquire at agent scope) carry that
//                dependency.  The wait is bounded in wall-clock time: past
//                the limit the kernel records a timeout, finishes the queue
//                without computing and exits, so every wave terminates.
//                Items are dequeued in level order and a dequeued item's
//                dependencies were dequeued earlier by running workgroups,
//                so the earliest unfinished item can always proceed.
#include <hip/hip_runtime.h>

#include "batch_internal.h"
#include "device_ops.h"
#include "deep_walk.h"
#include "pair_walk.h"

namespace chebtd {

// site index -> (x, y) walker over one tile
struct TileWalk {
    int64_t i, end;
    int32_t x, y, L;
    __device__ __forceinline__ void start(int64_t t0, int64_t n, int32_t tile, int32_t Lx)
    {
        L = Lx;
        i = t0 + threadIdx.x;
        end = t0 + tile < n ? t0 + tile : n;
        y = (int32_t)(i / L);
        x = (int32_t)(i - (int64_t)y * L);
    }
    __device__ __forceinline__ bool ok() const { return i < end; }
    __device__ __forceinline__ void next()
    {
        i += blockDim.x;
        x += blockDim.x;
        while (x >= L) {
            x -= L;
            ++y;
        }
    }
};

__device__ __forceinline__ double2 honey_apply2(const SysDev &sd, int64_t i, int32_t x, int32_t y,
                                                const double2 *v, double2 vi)
{
    OpHoney op;
    op.eps = sd.eps;
    op.b = sd.b;
    op.s2 = sd.s2;
    op.off2 = sd.off2;
    op.W = sd.W;
    op.L = sd.L;
    if (sd.edge == CHEBTD_ZIGZAG) return HoneyRow<CHEBTD_ZIGZAG>::apply2(op, i, x, y, v, vi);
    return HoneyRow<CHEBTD_ARMCHAIR>::apply2(op, i, x, y, v, vi);
}

// Level k of one tile of system sd in step parity `par`
//   k = 0: v1 = H~ psi -> A, acc = g0 psi + g1 v1 -> nxt
//   k > 0: v_{k+1} = 2 H~ v_k - v_{k-1} over v_{k-1}; acc += g_{k+1} v_{k+1}
__device__ __forceinline__ void tile_level(const SysDev &sd, const double2 *gamma, int k, int tile_idx,
                                           int32_t tile, int par)
{
    double2 *cur = par ? sd.B : sd.psi;
    double2 *nxt = par ? sd.psi : sd.B;
    double2 *A = sd.A;
    const int64_t n = (int64_t)sd.W * sd.L;
    TileWalk w;
    w.start((int64_t)tile_idx * tile, n, tile, sd.L);
    const double2 *g = gamma + sd.gamma_off;
    if (k == 0) {
        const double2 g0 = ldg(g, 0);
        const double2 g1 = sd.M >= 1 ? ldg(g, 1) : make_double2(0.0, 0.0);
        for (; w.ok(); w.next()) {
            const double2 vi = ldg(cur, w.i);
            const double2 h = cscale(0.5, honey_apply2(sd, w.i, w.x, w.y, cur, vi));
            stg(A, w.i, h);
            stg(nxt, w.i, cfma(g1, h, cfma(g0, vi, make_double2(0.0, 0.0))));
        }
    } else {
        const double2 gk = ldg(g, k + 1);
        const double2 *vk = (k & 1) ? A : cur;
        double2 *vprev = (k & 1) ? cur : A;
        for (; w.ok(); w.next()) {
            const double2 vi = ldg(vk, w.i);
            const double2 nv = csub(honey_apply2(sd, w.i, w.x, w.y, vk, vi), ldg(vprev, w.i));
            stg(vprev, w.i, nv);
            stg(nxt, w.i, cfma(gk, nv, ldg(nxt, w.i)));
        }
    }
}

// ---------------------------------------------------------------------------
// levels schedule
// ---------------------------------------------------------------------------
__global__ void k_batch_level(const SysDev *__restrict__ sys, const double2 *__restrict__ gamma,
                              const int32_t *__restrict__ blk_sys, const int32_t *__restrict__ blk_tile,
                              int k, int32_t tile, int par)
{
    const int32_t s = blk_sys[blockIdx.x];
    const SysDev sd = sys[s];
    if (k > 0 && k > sd.M - 1) return;
    tile_level(sd, gamma, k, blk_tile[blockIdx.x], tile, par);
}

// ---------------------------------------------------------------------------
// pairs schedule
// ---------------------------------------------------------------------------
// Buffers of one step (cur = state entering the step, nxt = accumulator):
// pass 0 reads cur and writes its last two orders to (A, C); odd passes read
// (A, C) and write (D, cur); even passes >= 2 read (D, cur) and write (A, C).
// cur is free once the head has read it.  The deep schedule's passes follow
// the same rotation.
template <bool HEAD>
__global__ __launch_bounds__(256) void k_batch_pair(const SysDev *__restrict__ sys,
                                                    const double2 *__restrict__ gamma,
                                                    const int32_t *__restrict__ blk_sys,
                                                    const int32_t *__restrict__ blk_wave0, int q, int deep_D,
                                                    int par)
{
    const int32_t lb = logical_block(1);
    const SysDev sd = sys[blk_sys[lb]];
    const int pass = (deep_D > 0 ? sd.ndeep : 0) + q;
    const int k = (deep_D > 0 ? sd.kdeep : 0) + 2 * q;
    const int32_t gw = __builtin_amdgcn_readfirstlane(blk_wave0[lb] + (int32_t)(threadIdx.x >> 6));
    const int32_t strip = gw % sd.nstrips;
    const int32_t chunk = gw / sd.nstrips;
    if (chunk >= sd.nchunks) return;  // uniform per wavefront; the kernel has no barrier
    OpPair op{};
    op.onsite = sd.eps;
    op.dshift = -sd.b;
    op.s2 = sd.s2;
    op.off2 = sd.off2;
    op.W = sd.W;
    op.L = sd.L;
    op.rows = sd.rows;
    op.nstrips = sd.nstrips;
    op.nchunks = sd.nchunks;
    double2 *cur = par ? sd.B : sd.psi;
    double2 *nxt = par ? sd.psi : sd.B;
    const double2 *g = gamma + sd.gamma_off;
    const double2 zero = make_double2(0.0, 0.0);
    double nrm = 0.0, en = 0.0;
    const double2 *in1, *in2;
    double2 *o1, *o2;
    double2 g0 = zero, g1, g2;
    if (HEAD) {
        in1 = nullptr;
        in2 = cur;
        o1 = sd.A;
        o2 = sd.C;
        g0 = ldg(g, 0);
        g1 = ldg(g, 1);
        g2 = ldg(g, 2);
    } else {
        const bool odd = pass & 1;
        in1 = odd ? sd.A : sd.D;
        in2 = odd ? sd.C : cur;
        o1 = odd ? sd.D : sd.A;
        o2 = odd ? cur : sd.C;
        g1 = ldg(g, k + 1);
        g2 = ldg(g, k + 2);
    }
    if (sd.edge == CHEBTD_ZIGZAG)
        pair_walk<CHEBTD_ZIGZAG, HEAD>(op, strip, chunk, in1, in2, o1, o2, nxt, g0, g1, g2, nullptr, nrm, en);
    else
        pair_walk<CHEBTD_ARMCHAIR, HEAD>(op, strip, chunk, in1, in2, o1, o2, nxt, g0, g1, g2, nullptr, nrm, en);
}

// D orders per pass over the batch (the deep walk of deep_walk.h, each
// system with its own operator, grid and weights), buffers as k_batch_pair.
// D is the batch's depth `base` or base + 1 (a system's first ndeep_ext
// passes); the system's grid and first order follow from it.
template <bool HEAD, int D>
__global__ __launch_bounds__(256) void k_batch_deep(const SysDev *__restrict__ sys,
                                                    const double2 *__restrict__ gamma,
                                                    const int32_t *__restrict__ blk_sys,
                                                    const int32_t *__restrict__ blk_wave0, int pass, int base,
                                                    int par)
{
    const int32_t lb = logical_block(1);
    const SysDev sd = sys[blk_sys[lb]];
    const bool ext = D != base;
    const int32_t nstrips = ext ? sd.dnstrips_ext : sd.dnstrips, nchunks = ext ? sd.dnchunks_ext : sd.dnchunks;
    const int32_t gw = __builtin_amdgcn_readfirstlane(blk_wave0[lb] + (int32_t)(threadIdx.x >> 6));
    const int32_t strip = gw % nstrips;
    const int32_t chunk = gw / nstrips;
    if (chunk >= nchunks) return;  // uniform per wavefront; the kernel has no barrier
    const int k = (base + 1) * min(pass, sd.ndeep_ext) + base * max(0, pass - sd.ndeep_ext);
    OpPair op{};
    op.onsite = sd.eps;
    op.dshift = -sd.b;
    op.s2 = sd.s2;
    op.off2 = sd.off2;
    op.W = sd.W;
    op.L = sd.L;
    op.rows = ext ? sd.drows_ext : sd.drows;
    op.nstrips = nstrips;
    op.nchunks = nchunks;
    double2 *cur = par ? sd.B : sd.psi;
    double2 *nxt = par ? sd.psi : sd.B;
    const double2 *g = gamma + sd.gamma_off;
    DeepArgs<D> A{};
    if (HEAD) {
        A.vkm1 = nullptr;
        A.vk = cur;
        A.out1 = sd.A;
        A.out2 = sd.C;
    } else {
        const bool odd = pass & 1;
        A.vkm1 = odd ? sd.A : sd.D;
        A.vk = odd ? sd.C : cur;
        A.out1 = odd ? sd.D : sd.A;
        A.out2 = odd ? cur : sd.C;
    }
    A.acc = nxt;
    // the system's final pass (no pairs or tail after it): nothing reads its
    // two orders, so only acc is written
    if (pass == sd.ndeep - 1 && sd.M == sd.kdeep) A.out1 = A.out2 = nullptr;
#pragma unroll
    for (int j = 0; j <= D; ++j) A.w.g[j] = (HEAD || j > 0) ? ldg(g, k + j) : make_double2(0.0, 0.0);
    double nrm = 0.0, en = 0.0;
    if (sd.edge == CHEBTD_ZIGZAG)
        deep_wave<CHEBTD_ZIGZAG, D, HEAD, kDeepProp>(op, strip, chunk, A, nrm, en);
    else
        deep_wave<CHEBTD_ARMCHAIR, D, HEAD, kDeepProp>(op, strip, chunk, A, nrm, en);
}

// The last order M of a system its passes left one short: v_M = 2 H~ v_{M-1}
// - v_{M-2} over v_{M-2}, acc += g_M v_M.  The system's last pass (index
// npass-1 of the schedule) left (v_{M-2}, v_{M-1}) in (A, C) when that index
// is even, in (D, cur) when odd.
__global__ void k_batch_tail(const SysDev *__restrict__ sys, const double2 *__restrict__ gamma,
                             const int32_t *__restrict__ blk_sys, const int32_t *__restrict__ blk_tile,
                             int32_t tile, int par, int deep)
{
    const SysDev sd = sys[blk_sys[blockIdx.x]];
    double2 *cur = par ? sd.B : sd.psi;
    double2 *nxt = par ? sd.psi : sd.B;
    const bool even = (((deep ? sd.npass_deep : sd.npass_pairs) - 1) & 1) == 0;
    double2 *vprev = even ? sd.A : sd.D;
    const double2 *vk = even ? sd.C : cur;
    const double2 gM = ldg(gamma + sd.gamma_off, sd.M);
    const int64_t n = (int64_t)sd.W * sd.L;
    TileWalk w;
    w.start((int64_t)blk_tile[blockIdx.x] * tile, n, tile, sd.L);
    for (; w.ok(); w.next()) {
        const double2 vi = ldg(vk, w.i);
        const double2 nv = csub(honey_apply2(sd, w.i, w.x, w.y, vk, vi), ldg(vprev, w.i));
        stg(vprev, w.i, nv);
        stg(nxt, w.i, cfma(gM, nv, ldg(nxt, w.i)));
    }
}

// ---------------------------------------------------------------------------
// persistent schedule
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t upper_index(const int64_t *a, int32_t cnt, int64_t v)
{
    // largest j in [0, cnt) with a[j] <= v (a ascending, a[0] = 0)
    int32_t lo = 0, hi = cnt - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (a[mid] <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Loop shape matters here: every thread-0-only action (publishing the
// previous tile, fetching and decoding the next item, waiting for its
// dependencies) sits in one block at the top of the loop, followed by a
// barrier, and the exit test reads the item through readfirstlane so that
// the compiler sees a uniform loop exit.  A thread-0-only tail before the
// back edge together with an exit the compiler cannot prove uniform lets it
// rotate the loop so that lanes 1..63 of wave 0 re-enter the barrier with a
// stale item while lane 0 waits outside the inner loop: a hang.
__global__ void k_batch_persistent(const SysDev *__restrict__ sys, const double2 *__restrict__ gamma,
                                   const QueueDev q, int32_t tile, int par, int64_t *queue_head,
                                   int32_t *done, int32_t *timeout_flag, int64_t spin_limit)
{
    __shared__ int32_t s_info[6];  // item (lo, hi), k, system, tile, skip
    int32_t pending = -1;          // system whose tile this block finished last (thread 0)
    for (;;) {
        if (threadIdx.x == 0) {
            if (pending >= 0)
                __hip_atomic_fetch_add(&done[pending], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const int64_t item = __hip_atomic_fetch_add(queue_head, (int64_t)1, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
            int32_t k = 0, s = 0, t = 0, skip = 0;
            const int32_t valid = item < q.total;
            if (valid) {
                // level k: items [q.level_off[k], q.level_off[k+1])
                k = upper_index(q.level_off, q.nlevels, item);
                const int64_t r = item - q.level_off[k];
                // active systems at level k are a prefix of the M-sorted order
                const int32_t j = upper_index(q.tile_prefix, q.level_active[k], r);
                s = q.order[j];
                t = (int32_t)(r - q.tile_prefix[j]);
                if (k > 0) {
                    // every tile of level k-1 of system s must be done; the wait
                    // is bounded in wall-clock ticks
                    const int32_t need = k * sys[s].ntiles;
                    const int64_t t_start = wall_clock64();
                    int64_t spins = 0;
                    while (__hip_atomic_load(&done[s], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
                        if (wall_clock64() - t_start > spin_limit ||
                            ((++spins & 255) == 0 &&
                             __hip_atomic_load(timeout_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                            __hip_atomic_store(timeout_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            skip = 1;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(8);
                    }
                }
            }
            s_info[0] = valid;
            s_info[2] = k;
            s_info[3] = s;
            s_info[4] = t;
            s_info[5] = skip;
            pending = valid ? s : -1;
        }
        __syncthreads();
        const int32_t valid = __builtin_amdgcn_readfirstlane(s_info[0]);
        if (!valid) break;
        const int32_t k = __builtin_amdgcn_readfirstlane(s_info[2]);
        const int32_t s = __builtin_amdgcn_readfirstlane(s_info[3]);
        const int32_t t = __builtin_amdgcn_readfirstlane(s_info[4]);
        const int32_t skip = __builtin_amdgcn_readfirstlane(s_info[5]);
        // the other tiles' results become visible to every thread of the block
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (!skip) tile_level(sys[s], gamma, k, t, tile, par);
        // this block's stores complete before thread 0 publishes the tile
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
    }
}

// the timeout flag cleared by a kernel (no memset node when a caller
// captures the call into a graph)
__global__ void k_batch_clear_flag(int32_t *flag) { flag[0] = 0; }

__global__ void k_batch_reset(int64_t *queue_head, int32_t *done, int32_t nsys)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) queue_head[0] = 0;
    if (i < nsys) done[i] = 0;
}

__global__ void k_batch_copy_back(const SysDev *__restrict__ sys, const int32_t *__restrict__ blk_sys,
                                  const int32_t *__restrict__ blk_tile, int32_t tile)
{
    const SysDev sd = sys[blk_sys[blockIdx.x]];
    const int64_t n = (int64_t)sd.W * sd.L;
    const int64_t t0 = (int64_t)blk_tile[blockIdx.x] * tile;
    const int64_t end = t0 + tile < n ? t0 + tile : n;
    for (int64_t i = t0 + threadIdx.x; i < end; i += blockDim.x) stg(sd.psi, i, ldg(sd.B, i));
}

hipError_t launch_batch_level(hipStream_t s, const SysDev *sys, const double2 *gamma, const int32_t *blk_sys,
                              const int32_t *blk_tile, int64_t nblocks, int k, int32_t tile, int par,
                              int block)
{
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_level, dim3((unsigned)nblocks), dim3(block), 0, s, sys, gamma, blk_sys,
                       blk_tile, k, tile, par);
    return hipGetLastError();
}

hipError_t launch_batch_persistent(hipStream_t s, const SysDev *sys, const double2 *gamma, const QueueDev &q,
                                   int32_t tile, int par, int64_t *queue_head, int32_t *done,
                                   int32_t *timeout_flag, int nsys, int grid, int block, int64_t spin_limit)
{
    hipLaunchKernelGGL(k_batch_reset, dim3((nsys + 255) / 256), dim3(256), 0, s, queue_head, done, nsys);
    hipLaunchKernelGGL(k_batch_persistent, dim3(grid), dim3(block), 0, s, sys, gamma, q, tile, par,
                       queue_head, done, timeout_flag, spin_limit);
    return hipGetLastError();
}

hipError_t launch_batch_pair(hipStream_t s, const SysDev *sys, const double2 *gamma, const int32_t *blk_sys,
                             const int32_t *blk_wave0, int64_t nblocks, int q, int deep_D, int par)
{
    if (nblocks <= 0) return hipSuccess;
    // a head pass only where no deep pass came first (pairs schedule, q = 0)
    if (q == 0 && deep_D == 0)
        hipLaunchKernelGGL(k_batch_pair<true>, dim3((unsigned)nblocks), dim3(256), 0, s, sys, gamma, blk_sys,
                           blk_wave0, q, deep_D, par);
    else
        hipLaunchKernelGGL(k_batch_pair<false>, dim3((unsigned)nblocks), dim3(256), 0, s, sys, gamma, blk_sys,
                           blk_wave0, q, deep_D, par);
    return hipGetLastError();
}

namespace {
template <int D>
hipError_t launch_batch_deep_d(hipStream_t s, const SysDev *sys, const double2 *gamma, const int32_t *blk_sys,
                               const int32_t *blk_wave0, int64_t nblocks, int pass, int base, int par)
{
    if (pass == 0)
        hipLaunchKernelGGL((k_batch_deep<true, D>), dim3((unsigned)nblocks), dim3(256), 0, s, sys, gamma, blk_sys,
                           blk_wave0, pass, base, par);
    else
        hipLaunchKernelGGL((k_batch_deep<false, D>), dim3((unsigned)nblocks), dim3(256), 0, s, sys, gamma,
                           blk_sys, blk_wave0, pass, base, par);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_batch_deep(hipStream_t s, int D, const SysDev *sys, const double2 *gamma,
                             const int32_t *blk_sys, const int32_t *blk_wave0, int64_t nblocks, int pass, int base,
                             int par)
{
    if (nblocks <= 0) return hipSuccess;
    switch (D) {
        case 4: return launch_batch_deep_d<4>(s, sys, gamma, blk_sys, blk_wave0, nblocks, pass, base, par);
        case 5: return launch_batch_deep_d<5>(s, sys, gamma, blk_sys, blk_wave0, nblocks, pass, base, par);
        case 6: return launch_batch_deep_d<6>(s, sys, gamma, blk_sys, blk_wave0, nblocks, pass, base, par);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_clear_flag(hipStream_t s, int32_t *flag)
{
    hipLaunchKernelGGL(k_batch_clear_flag, dim3(1), dim3(1), 0, s, flag);
    return hipGetLastError();
}

hipError_t launch_batch_tail(hipStream_t s, const SysDev *sys, const double2 *gamma, const int32_t *blk_sys,
                             const int32_t *blk_tile, int64_t nblocks, int32_t tile, int par, int block, int deep)
{
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_tail, dim3((unsigned)nblocks), dim3(block), 0, s, sys, gamma, blk_sys, blk_tile,
                       tile, par, deep);
    return hipGetLastError();
}

hipError_t launch_batch_copy_back(hipStream_t s, const SysDev *sys, const int32_t *blk_sys,
                                  const int32_t *blk_tile, int64_t nblocks, int32_t tile, int block)
{
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_copy_back, dim3((unsigned)nblocks), dim3(block), 0, s, sys, blk_sys, blk_tile,
                       tile);
    return hipGetLastError();
}

}  // namespace chebtd
