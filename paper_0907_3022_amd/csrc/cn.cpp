// Host side of the Crank-Nicolson comparison method, eq. (CN): factor the
// step-independent tridiagonal A = 1 + i dt H/2 of the 1D chain once and
// tabulate the affine-map products the one-wavefront scan kernel needs.
#include <hip/hip_runtime.h>

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
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess)
        max_lds = 65536;
    if ((size_t)2 * n * sizeof(double2) > (size_t)max_lds)
        return fail(c, CHEBTD_E_ARG,
                    "chebtd_crank_nicolson: the chain must fit twice in one workgroup's LDS (n <= " +
                        std::to_string(max_lds / 32) + ")");
    if (S == 0) return CHEBTD_OK;
    std::vector<double> V((size_t)n);
    hipError_t e = hipMemcpy(V.data(), c->V, (size_t)n * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "chebtd_crank_nicolson: reading V");
    const cd h(0.0, 0.5 * dt);  // i dt / 2
    const double inv2 = 1.0 / (c->dx * c->dx);
    const cd o = h * (-0.5 * inv2);
    const int chunk = (n + 63) / 64;
    // Thomas factors of A
    std::vector<cd> a(n), d(n), fa(n), ba(n), invd(n), fpre(n), bpre(n);
    for (int j = 0; j < n; ++j) a[j] = 1.0 + h * (inv2 + V[j]);
    d[0] = a[0];
    fa[0] = 0.0;
    for (int j = 1; j < n; ++j) {
        const cd m = o / d[j - 1];
        d[j] = a[j] - m * o;
        fa[j] = -m;
    }
    for (int j = 0; j < n; ++j) {
        invd[j] = 1.0 / d[j];
        ba[j] = (j + 1 < n) ? -o / d[j] : cd(0.0);
    }
    // chunk products and in-chunk prefix / suffix products
    std::vector<cd> Pf(64, 1.0), Pb(64, 1.0);
    for (int l = 0; l < 64; ++l) {
        const int j0 = l * chunk, j1 = std::min(j0 + chunk, n);
        cd p = 1.0;
        for (int j = j0; j < j1; ++j) {
            p *= fa[j];
            fpre[j] = p;
        }
        Pf[l] = p;
        p = 1.0;
        for (int j = j1 - 1; j >= j0; --j) {
            p *= ba[j];
            bpre[j] = p;
        }
        Pb[l] = p;
    }
    // Kogge-Stone: the map product each lane holds at the start of stage d
    std::vector<cd> fst(6 * 64, 0.0), bst(6 * 64, 0.0);
    std::vector<cd> accf = Pf, accb = Pb;
    for (int dd = 0; dd < 6; ++dd) {
        const int off = 1 << dd;
        std::vector<cd> nf = accf, nb = accb;
        for (int l = 0; l < 64; ++l) {
            fst[dd * 64 + l] = accf[l];
            bst[dd * 64 + l] = accb[l];
            if (l >= off) nf[l] = accf[l] * accf[l - off];
            if (l + off < 64) nb[l] = accb[l] * accb[l + off];
        }
        accf = nf;
        accb = nb;
    }
    // upload: six per-site tables, then the two stage tables
    std::vector<cd> blob;
    blob.reserve((size_t)6 * n + 2 * 6 * 64);
    for (auto *v : {&a, &fa, &fpre, &ba, &invd, &bpre}) blob.insert(blob.end(), v->begin(), v->end());
    blob.insert(blob.end(), fst.begin(), fst.end());
    blob.insert(blob.end(), bst.begin(), bst.end());
    DevBuf tab;
    int rc = ensure(c, tab, blob.size() * sizeof(cd), "Crank-Nicolson tables");
    if (rc) return rc;
    e = hipMemcpy(tab.p, blob.data(), blob.size() * sizeof(cd), hipMemcpyHostToDevice);
    CnDev t;
    const double2 *base = static_cast<const double2 *>(tab.p);
    t.a = base;
    t.fa = base + n;
    t.fpre = base + 2 * n;
    t.ba = base + 3 * n;
    t.invd = base + 4 * n;
    t.bpre = base + 5 * n;
    t.fstage = base + 6 * n;
    t.bstage = base + 6 * n + 6 * 64;
    t.o = make_double2(o.real(), o.imag());
    t.n = n;
    t.chunk = chunk;
    if (e == hipSuccess) e = launch_cn_chain(c->stream, t, reinterpret_cast<double2 *>(psi_dev), S);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    release(tab);
    if (e != hipSuccess) return hip_fail(c, e, "chebtd_crank_nicolson");
    return CHEBTD_OK;
}
