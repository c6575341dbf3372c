// Crank-Nicolson comparison method for the 1D chain (cn.hip, cn.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace chebtd {

constexpr int kCnThreads = 256;  // one workgroup: one wavefront per SIMD of a CU
constexpr int kCnMaxChunk = 16;  // sites per thread, so n <= 4096

// Step-independent tables of A = 1 + i dt H/2 = L U, laid out per thread t
// of the workgroup; site j = t * chunk + c, padded to 256 * chunk sites.
// Complex numbers are (re, im) pairs.
struct CnDev {
    const double *aim;      // Im a_j = dt/2 (1/dx^2 + V_j)        [chunk][256]
    const double2 *fa;      // -m_j (forward factor; 1 on padding)  [chunk][256]
    const double2 *invd;    // 1/d_j (0 on padding)                 [chunk][256]
    const double2 *fstage;  // forward scan multipliers             [6][256]
    const double2 *bstage;  // backward scan multipliers            [6][256]
    const double2 *pex;     // forward exclusive lane products      [256]
    const double2 *qex;     // backward exclusive lane products     [256]
    const double2 *ptot;    // forward map product of each wave     [4]
    const double2 *qtot;    // backward map product of each wave    [4]
    double oim;             // Im of the off-diagonal o = -i dt/(4 dx^2)
    int32_t n, chunk;
};

hipError_t launch_cn_chain(hipStream_t s, const CnDev &t, double2 *psi, int64_t S);

}  // namespace chebtd
