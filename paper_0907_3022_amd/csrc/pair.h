// Two-orders-per-pass recursion kernel for brick-wall lattices (pair.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_ops.h"
#include "internal.h"

namespace chebtd {

struct OpPair {
    const double *onsite;  // eps (ribbon) or V (chain)
    double dshift;         // -b (ribbon) or 1/dx^2 - b (chain)
    double s2;             // 2/a
    double off2;           // -2t/a (ribbon) or -1/(dx^2 a) (chain)
    int32_t W, L;          // rows, columns (a chain is one row of n columns)
    int32_t rows;          // rows per chunk
    int32_t nstrips, nchunks;
    int32_t xcd_remap;
};

constexpr int kPairStripCols = 62;  // columns a wavefront owns
// columns a wavefront of the D-orders walk owns (each level past the first
// loses one lane per side)
constexpr int deep_strip_cols(int D) { return 66 - 2 * D; }

OpPair make_pair_op(const Ctx &c, int rows);
int64_t pair_grid_blocks(const Ctx &c, int rows);
// rows per wavefront chunk for a ribbon of W rows (api.cpp)
int pair_rows_for_width(int64_t W);
bool pair_supported(const Ctx &c);
// head: v1 = H~ vk, v2 = 2 H~ v1 - vk, acc = g0 vk + g1 v1 + g2 v2 (+ partials, ckpt)
// else: v_{k+1} = 2 H~ vk - vkm1, v_{k+2} = 2 H~ v_{k+1} - vk, acc += g1 v_{k+1} + g2 v_{k+2}
// D = 3 .. 6 orders per pass (deep_walk.h): the same buffers and roles as
// launch_pair, with the weights g_k .. g_{k+D} in g (g[0] used by the head)
OpPair make_deep_op(const Ctx &c, int rows, int D);
int64_t deep_grid_blocks(const Ctx &c, int rows, int D);
// whether the propagation's deep passes stream their stores past the caches:
// from 16M sites, where the working set is far past the last-level cache
inline bool deep_stream_stores(const Ctx &c) { return c.n >= (int64_t(16) << 20); }

// The deep kernel's 32-bit buffer offsets stay unambiguous for a W x L
// lattice: rows from -(D+1) to W+D+1 at 16 B per site, plus the 2^31 bias of
// lanes outside the lattice, never wrap into the buffer (D <= 6).
inline bool deep_offsets_fit(int64_t W, int64_t L)
{
    return (W + 2 * 6 + 2) * L * 16 <= (int64_t(1) << 31);
}
hipError_t launch_deep(const Ctx &c, hipStream_t s, int D, int rows, bool head, const double2 *vkm1,
                       const double2 *vk, double2 *out1, double2 *out2, double2 *acc, const double2 *g,
                       double2 *ckpt, double *partials, const NeFinal *fin);

// fin (non-head passes, may be null): block 0 also finishes the step's norm
// and energy from the head's partials
hipError_t launch_pair(const Ctx &c, hipStream_t s, int rows, bool head, const double2 *vkm1, const double2 *vk,
                       double2 *out1, double2 *out2, double2 *acc, double2 g0, double2 g1, double2 g2,
                       double2 *ckpt, double *partials, const NeFinal *fin = nullptr);

}  // namespace chebtd
