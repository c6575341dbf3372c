// Host side of the Crank-Nicolson comparison method, eq. (CN): factor the
// step-independent tridiagonal A = 1 + i dt H/2 of the 1D chain once and
// tabulate the affine-map products the one-workgroup scan kernel needs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "cn.h"
#include "internal.h"

namespace chebtd {
int fail(Ctx *c, int code, const std::string &msg);
int hip_fail(Ctx *c, hipError_t e, const char *what);
int ensure(Ctx *c, DevBuf &b, size_t bytes, const char *what);
void release(DevBuf &b);
}  // namespace chebtd

using namespace chebtd;
struct chebtd_ctx : public Ctx {};
using cd = std::complex<double>;

extern "C" int chebtd_crank_nicolson(chebtd_ctx *ctx, double *psi_dev, double dt, int64_t S)
{
    if (!ctx) return fail(nullptr, CHEBTD_E_ARG, "null context");
    Ctx *c = static_cast<Ctx *>(ctx);
    if (c->kind != HKind::Chain) return fail(c, CHEBTD_E_STATE, "chebtd_crank_nicolson: needs a 1D chain");
    if (!psi_dev || S < 0 || !(dt > 0.0) || !std::isfinite(dt))
        return fail(c, CHEBTD_E_ARG, "chebtd_crank_nicolson: need psi, S >= 0 and dt > 0");
    const int n = (int)c->n;
    if (n > kCnThreads * kCnMaxChunk)
        return fail(c, CHEBTD_E_ARG,
                    "chebtd_crank_nicolson: the chain must fit one workgroup's registers (n <= " +
                        std::to_string(kCnThreads * kCnMaxChunk) + ")");
    if (S == 0) return CHEBTD_OK;
    std::vector<double> V((size_t)n);
    hipError_t e = hipMemcpy(V.data(), c->V, (size_t)n * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "chebtd_crank_nicolson: reading V");
    const double inv2 = 1.0 / (c->dx * c->dx);
    const double oim = 0.5 * dt * (-0.5 * inv2);  // o = i*oim
    const cd o(0.0, oim);
    int C = 1;
    while (C * kCnThreads < n) C *= 2;
    const int T = kCnThreads, N = C * T;
    // Thomas factors of A, padded: beyond the chain fa = 1, 1/d = 0, so the
    // forward values there are never used and the backward values are 0
    std::vector<double> aim((size_t)N, 0.0);
    std::vector<cd> fa((size_t)N, 1.0), invd((size_t)N, 0.0);
    cd d_prev = 0.0;
    for (int j = 0; j < n; ++j) {
        aim[j] = 0.5 * dt * (inv2 + V[j]);
        const cd a(1.0, aim[j]);
        if (j == 0) {
            fa[j] = 0.0;
            d_prev = a;
        } else {
            const cd m = o / d_prev;
            fa[j] = -m;
            d_prev = a - m * o;
        }
        invd[j] = 1.0 / d_prev;
    }
    // chunk map products: forward p_j = fa_j, backward p_j = -o/d_j
    std::vector<cd> Pf(T, 1.0), Qb(T, 1.0);
    for (int t = 0; t < T; ++t)
        for (int q = 0; q < C; ++q) {
            Pf[t] *= fa[(size_t)t * C + q];
            Qb[t] *= -o * invd[(size_t)t * C + q];
        }
    // the products each lane holds before every scan stage, replaying the
    // kernel's stages: row shifts by 1, 2, 4, 8 inside 16-lane rows, then
    // rows 1 and 3 (forward) / 0 and 2 (backward) from the neighbouring row's
    // edge lane, then the upper (lower) half from lane 31 (32)
    std::vector<cd> fst((size_t)6 * T), bst((size_t)6 * T), pex(T), qex(T), ptot(4), qtot(4);
    for (int w = 0; w < 4; ++w) {
        std::vector<cd> acc(Pf.begin() + 64 * w, Pf.begin() + 64 * w + 64), nxt;
        for (int k = 0; k < 6; ++k) {
            nxt = acc;
            for (int l = 0; l < 64; ++l) {
                fst[(size_t)k * T + 64 * w + l] = acc[l];
                const int row = l / 16;
                int src = -1;
                if (k < 4 && l % 16 >= (1 << k)) src = l - (1 << k);
                if (k == 4 && (row == 1 || row == 3)) src = 16 * row - 1;
                if (k == 5 && row >= 2) src = 31;
                if (src >= 0) nxt[l] = acc[l] * acc[src];
            }
            acc = nxt;
        }
        for (int l = 0; l < 64; ++l) pex[64 * w + l] = l > 0 ? acc[l - 1] : cd(1.0);
        ptot[w] = acc[63];
        acc.assign(Qb.begin() + 64 * w, Qb.begin() + 64 * w + 64);
        for (int k = 0; k < 6; ++k) {
            nxt = acc;
            for (int l = 0; l < 64; ++l) {
                bst[(size_t)k * T + 64 * w + l] = acc[l];
                const int row = l / 16;
                int src = -1;
                if (k < 4 && l % 16 + (1 << k) < 16) src = l + (1 << k);
                if (k == 4 && (row == 0 || row == 2)) src = 16 * (row + 1);
                if (k == 5 && row < 2) src = 32;
                if (src >= 0) nxt[l] = acc[l] * acc[src];
            }
            acc = nxt;
        }
        for (int l = 0; l < 64; ++l) qex[64 * w + l] = l < 63 ? acc[l + 1] : cd(1.0);
        qtot[w] = acc[0];
    }
    // upload, per-thread layouts [c][t]
    std::vector<cd> blob;
    blob.reserve((size_t)3 * N + 12 * T + 2 * T + 8);
    for (int q = 0; q < C; ++q)
        for (int t = 0; t < T; ++t) blob.push_back(fa[(size_t)t * C + q]);
    for (int q = 0; q < C; ++q)
        for (int t = 0; t < T; ++t) blob.push_back(invd[(size_t)t * C + q]);
    blob.insert(blob.end(), fst.begin(), fst.end());
    blob.insert(blob.end(), bst.begin(), bst.end());
    blob.insert(blob.end(), pex.begin(), pex.end());
    blob.insert(blob.end(), qex.begin(), qex.end());
    blob.insert(blob.end(), ptot.begin(), ptot.end());
    blob.insert(blob.end(), qtot.begin(), qtot.end());
    const size_t cplx_bytes = blob.size() * sizeof(cd);
    std::vector<double> aim_t((size_t)N);
    for (int q = 0; q < C; ++q)
        for (int t = 0; t < T; ++t) aim_t[(size_t)q * T + t] = aim[(size_t)t * C + q];
    DevBuf tab;
    int rc = ensure(c, tab, cplx_bytes + aim_t.size() * sizeof(double), "Crank-Nicolson tables");
    if (rc) return rc;
    e = hipMemcpy(tab.p, blob.data(), cplx_bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(static_cast<char *>(tab.p) + cplx_bytes, aim_t.data(), aim_t.size() * sizeof(double),
                      hipMemcpyHostToDevice);
    const double2 *base = static_cast<const double2 *>(tab.p);
    CnDev t;
    t.fa = base;
    t.invd = base + N;
    t.fstage = base + 2 * N;
    t.bstage = base + 2 * N + 6 * T;
    t.pex = base + 2 * N + 12 * T;
    t.qex = base + 2 * N + 13 * T;
    t.ptot = base + 2 * N + 14 * T;
    t.qtot = base + 2 * N + 14 * T + 4;
    t.aim = reinterpret_cast<const double *>(static_cast<char *>(tab.p) + cplx_bytes);
    t.oim = oim;
    t.n = n;
    t.chunk = C;
    if (e == hipSuccess) e = launch_cn_chain(c->stream, t, reinterpret_cast<double2 *>(psi_dev), S);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    release(tab);
    if (e != hipSuccess) return hip_fail(c, e, "chebtd_crank_nicolson");
    return CHEBTD_OK;
}
