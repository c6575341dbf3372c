// Crank-Nicolson comparison method for the 1D chain (cn.hip, cn.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace chebtd {

// Step-independent tables of A = 1 + i dt H/2 = L U (device pointers).
struct CnDev {
    const double2 *a;       // diagonal of A                         [n]
    const double2 *fa;      // forward map factor  -m_j (0 at j = 0)  [n]
    const double2 *fpre;    // prod of fa over the lane chunk up to j [n]
    const double2 *ba;      // backward map factor -o/d_j (0 at n-1)  [n]
    const double2 *invd;    // 1/d_j                                  [n]
    const double2 *bpre;    // prod of ba from j to the chunk end     [n]
    const double2 *fstage;  // forward scan multipliers  [6][64]
    const double2 *bstage;  // backward scan multipliers [6][64]
    double2 o;              // off-diagonal of A
    int32_t n, chunk;
};

hipError_t launch_cn_chain(hipStream_t s, const CnDev &t, double2 *psi, int64_t S);

}  // namespace chebtd
