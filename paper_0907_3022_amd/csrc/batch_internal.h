// Device-side descriptors of the batched ribbon path (batch.hip/batch.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace chebtd {

// One ribbon of a batch, as the kernels see it.
struct SysDev {
    const double *eps;  // on-site energies
    double2 *psi;       // caller's state (in/out)
    double2 *A, *B;     // work vectors: v_1, v_3, ... and the accumulator/state
    int32_t W, L, edge, M;
    double b, s2, off2;  // shift, 2/a, -2t/a
    int64_t gamma_off;   // first weight in the concatenated table
    int32_t ntiles;
    int32_t pad;
    // two-orders-per-pass schedule: two more work vectors and the wavefront grid
    double2 *C, *D;
    int32_t rows, nstrips, nchunks, pad2;
    // deep schedule: the wavefront grid of the walk at the batch's depth D,
    // and the passes each schedule gives the system (the odd-order tail reads
    // the vectors its last pass left)
    int32_t drows, dnstrips, dnchunks;
    int32_t npass_pairs, npass_deep;
    int32_t ndeep;      // deep passes of the system (then pairs, then the tail)
    int32_t ndeep_ext;  // the first ndeep_ext of them take D + 1 orders
    int32_t kdeep;      // orders the deep passes cover
    int32_t drows_ext, dnstrips_ext, dnchunks_ext;  // the walk's grid at D + 1
};

// Work queue of the persistent schedule (item = level, system, tile).
struct QueueDev {
    const int64_t *level_off;    // [nlevels + 1]
    const int32_t *level_active; // [nlevels]: systems active at a level (prefix of order)
    const int64_t *tile_prefix;  // [nsys + 1]: tiles before the j-th system of order
    const int32_t *order;        // [nsys]: systems sorted by M, descending
    int32_t nlevels;
    int32_t pad;
    int64_t total;
};

hipError_t launch_batch_level(hipStream_t s, const SysDev *sys, const double2 *gamma, const int32_t *blk_sys,
                              const int32_t *blk_tile, int64_t nblocks, int k, int32_t tile, int par,
                              int block);
hipError_t launch_batch_persistent(hipStream_t s, const SysDev *sys, const double2 *gamma, const QueueDev &q,
                                   int32_t tile, int par, int64_t *queue_head, int32_t *done,
                                   int32_t *timeout_flag, int nsys, int grid, int block, int64_t spin_limit);
// pairs schedule: level 0 is the step head (orders 1, 2), level p >= 1 runs
// orders 2p+1 and 2p+2; blk_sys / blk_wave0 give each block's system and its
// first wavefront in that system's strip-major wavefront numbering.
// Two orders per pass: the q-th two-order pass of each listed system, after
// its deep passes when `deep_D` > 0 (sd.ndeep passes covering sd.kdeep
// orders), so pass index sd.ndeep + q (0: the head) and orders k+1, k+2 with
// k = sd.kdeep + 2q; the pass index picks the buffers (batch.hip).
hipError_t launch_batch_pair(hipStream_t s, const SysDev *sys, const double2 *gamma, const int32_t *blk_sys,
                             const int32_t *blk_wave0, int64_t nblocks, int q, int deep_D, int par);
// Deep pass `pass` of each listed system, D = base or base + 1 orders (D = 4,
// 5, 6): a system's first ndeep_ext passes take base + 1 orders, the others
// base, so pass p starts after k = (base + 1) min(p, ndeep_ext) + base
// max(0, p - ndeep_ext) orders; all listed systems take D orders in this pass.
hipError_t launch_batch_deep(hipStream_t s, int D, const SysDev *sys, const double2 *gamma,
                             const int32_t *blk_sys, const int32_t *blk_wave0, int64_t nblocks, int pass, int base,
                             int par);
// the last order M of systems left with one order, one tile per block; the
// vectors are those the system's last pass of the schedule (deep or not) left
hipError_t launch_batch_tail(hipStream_t s, const SysDev *sys, const double2 *gamma, const int32_t *blk_sys,
                             const int32_t *blk_tile, int64_t nblocks, int32_t tile, int par, int block,
                             int deep);
hipError_t launch_batch_clear_flag(hipStream_t s, int32_t *flag);
// the deep schedule's passes for M orders at depth D (batch.cpp)
void batch_deep_split(int M, int D, int *npass, int *next);
hipError_t launch_batch_copy_back(hipStream_t s, const SysDev *sys, const int32_t *blk_sys,
                                  const int32_t *blk_tile, int64_t nblocks, int32_t tile, int block);

}  // namespace chebtd
