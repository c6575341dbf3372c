// Internal declarations of the chebtd library (host runtime + HIP kernels).
// Not part of the public ABI; see include/chebtd.h for the contract.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "chebtd.h"

namespace chebtd {

constexpr int kMaxDepth = 6;  // most Chebyshev orders one deep-walk pass carries

// ---------------------------------------------------------------------------
// Operators: each applies 2 H~ = (2/a)(H - b) to row i of a complex vector.
// The step head needs H~ itself and takes exactly half (a power-of-two
// scaling, so no rounding is added).
// ---------------------------------------------------------------------------
struct OpChain {
    const double *V;  // on-site potential, float64[n]
    double dsh;       // 1/dx^2 - b  (diagonal without V)
    double s2;        // 2/a
    double off2;      // 2 * (-1/(2 dx^2)) / a
    int64_t n;
};

struct OpHoney {
    const double *eps;  // on-site energies, float64[W*L]
    double b;           // shift
    double s2;          // 2/a
    double off2;        // -2 t / a
    int32_t W, L;       // grid (rows, columns)
    int32_t xblocks;    // ceil(L / block)
    int32_t xcd_remap;  // 1: map blocks XCD-contiguously
};

// Matrix-free Holstein operator, eq. (ghm): per state (r, i) the raised and
// lowered phonon configurations of site i and its occupation, per
// configuration the total phonon number.
// state index i = site * nconf + r (rank r of the phonon configuration)
struct OpHol {
    const int32_t *up;     // rank of n + e_i, or -1     [state]
    const int32_t *dn;     // rank of n - e_i, or -1     [state]
    const uint8_t *occ;    // n_i                        [state]
    const uint8_t *tot;    // sum_j n_j                  [configuration]
    const double *Delta;   // Delta_i                    [site]
    const double *gw0;     // g_i w0                     [site]
    const double *sq;      // sqrt(0 .. nph+1)
    double w0, t, b, s2;
    int32_t L, periodic;
    int64_t n;
    uint32_t nconf;
};

struct OpCsr {
    const int64_t *rowptr;
    const int32_t *col;
    const double2 *val;
    double b;
    double s2;  // 2/a
    int64_t n;
};

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
enum class HKind { None = 0, Chain, Honeycomb, Csr, Holstein };

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct BatchState;  // batched ribbons (batch.cpp)
struct AdjState;    // adjoint storage (adjoint.cpp)

struct Ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    int num_cus = 256;
    std::string err;

    // Hamiltonian
    HKind kind = HKind::None;
    int64_t n = 0;
    // chain
    double dx = 0.0;
    const double *V = nullptr;
    // honeycomb
    int64_t W = 0, L = 0;
    int edge = 0;
    double t_hop = 1.0;
    const double *eps = nullptr;
    // csr
    int64_t nnz = 0;
    const int64_t *rowptr = nullptr;
    const int32_t *col = nullptr;
    const double *val = nullptr;
    // Holstein (owned device copies)
    bool holstein = false;
    int hol_L = 0, hol_nph = 0;
    int64_t hol_nconf = 0;
    // matrix-free tables (per state: up, dn, occ; per configuration: tot) and
    // per-site constants (Delta, g w0, then the sqrt table)
    DevBuf hol_occ, hol_up, hol_dn, hol_tot, hol_site;
    int hol_periodic = 0;
    double hol_t = 0.0, hol_w0 = 0.0;
    const double *hol_delta = nullptr;  // per-step Delta_i during a time-dependent run
    int hol_spt = 0;    // electron sites per thread of the walk; 0: all L
    int hol_remap = 0;  // 1: XCD-contiguous configuration ranges in the walk
    // binomial table C(a, m), a <= nph + L + 1, m <= L (row-major, L + 1 per
    // row) from which the walk ranks the phonon partners itself; empty when
    // it would not fit the walk's LDS budget (the walk then reads the tables)
    DevBuf hol_binom;
    int hol_brows = 0;

    // bounds and plan
    bool has_bounds = false;
    double emin = 0.0, emax = 0.0, alpha = 0.01, a = 1.0, b = 0.0;
    bool has_plan = false;
    double dt = 0.0;
    int M = 0;
    std::vector<double> gamma;  // interleaved complex, M+1 entries
    DevBuf gamma_dev;           // device copy of gamma

    // work vectors: two complex vectors of length n, two more for the
    // two-orders-per-pass kernel
    DevBuf vA, vB, vC, vD;
    bool use_pairs = false;  // brick-wall H with M >= 2 and pair buffers present
    int pair_rows = 16;      // rows per wavefront chunk of the pair kernel
    // orders per pass of one step on the multi-order path, the head's first
    // and a single-order pass (if any) last: 2 runs the pair kernel, 3 ..
    // kMaxDepth the deep kernel
    std::vector<int> passes;
    int deep_rows[kMaxDepth + 1] = {};  // rows per wavefront chunk of the deep kernel, by depth
    // reduction scratch: partial sums, step counter, results
    DevBuf partials;   // double[2 * max_blocks]
    DevBuf results;    // double[16]
    DevBuf counter;    // int64[4]
    DevBuf chainx;     // exchange strips, flags and partials of the several-workgroup chain run
    double *pinned = nullptr;  // host pinned double[16]
    double check_tol = 1e-6;
    int64_t plan_version = 0;  // bumped by every plan
    int64_t run_seq = 0;       // numbers the checkpointing propagation runs

    // graph cache for CHEBTD_GRAPH
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
    const void *graph_key[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t ev_a = nullptr, ev_b = nullptr;

    BatchState *batch = nullptr;
    AdjState *adj = nullptr;
};

// ---------------------------------------------------------------------------
// Host helpers (plan.cpp, holstein.cpp)
// ---------------------------------------------------------------------------
int bessel_miller(double z, int kmax, std::vector<double> &J);
int truncation_order(double z, double tol);
void step_weights(double a, double b, double dt, int M, std::vector<double> &gamma);
void shift_scale(double emin, double emax, double alpha, double *a, double *b);

struct HolsteinCsr {
    int64_t n = 0, nnz = 0, nconf = 0;
    std::vector<int64_t> rowptr;
    std::vector<int32_t> col;
    std::vector<double> val;  // complex interleaved
};
struct HolsteinTables {
    int L = 0, nph = 0;
    int64_t nconf = 0, n = 0;
    std::vector<int32_t> up, dn;  // per state
    std::vector<uint8_t> occ;     // per state
    std::vector<uint8_t> tot;     // per configuration
};
int holstein_tables(int L, int nph, int periodic, HolsteinTables &out, std::string &err);
int holstein_count(int L, int nph, int64_t *count);
int holstein_build(int L, int nph, double t, double w0, const double *g, const double *Delta,
                   int periodic, HolsteinCsr &out, std::string &err);

// ---------------------------------------------------------------------------
// Kernel launchers (kernels.hip).  All enqueue on `s` and return hipError_t.
// ---------------------------------------------------------------------------
constexpr int kBlock = 256;
// LDS the Holstein walk may give its binomial table (beyond it, the walk
// reads the per-state partner tables instead)
constexpr int kHolBinomBytes = 16384;
int64_t grid_blocks(const Ctx &c);
// blocks of the norm and region sums (grid-stride: one partial pair per
// block, at most kReduceBlocks of them whatever n is)
constexpr int64_t kReduceBlocks = 2048;
inline int64_t reduce_blocks(int64_t n)
{
    const int64_t nb = (n + kBlock - 1) / kBlock;
    return nb < kReduceBlocks ? (nb > 0 ? nb : 1) : kReduceBlocks;
}
// blocks (one partial pair each) of the single-order step head
int64_t head_blocks(const Ctx &c);

hipError_t launch_head(const Ctx &c, hipStream_t s, const double2 *v0, double2 *v1, double2 *acc,
                       double2 g0, double2 g1, double2 *ckpt, double *partials);
hipError_t launch_iter(const Ctx &c, hipStream_t s, const double2 *vk, double2 *vprev,
                       double2 *acc, double2 g);
// Holstein or CSR order with the accumulator brought up to date for the
// last nacc (0 .. 3) orders: acc += ga v_{k-1} + gb v_k + gc v_{k+1}, leading
// terms dropped; nacc = 0 leaves acc untouched (kernels.hip)
hipError_t launch_iter_lazy(const Ctx &c, hipStream_t s, const double2 *vk, double2 *vprev, double2 *acc, int nacc,
                            double2 ga, double2 gb, double2 gc);
hipError_t launch_finalize_ne(hipStream_t s, const double *partials, int nparts, double a, double b,
                              double *norm_out, double *energy_out, int64_t *step_counter,
                              double *dst2);
hipError_t launch_reset_counter(hipStream_t s, int64_t *counter);
hipError_t launch_norm(const Ctx &c, hipStream_t s, const double2 *psi, double *partials);
hipError_t launch_sum_partials(hipStream_t s, const double *partials, int nparts, int stride,
                               double *out);
hipError_t launch_copy(hipStream_t s, const double2 *src, double2 *dst, int64_t n);
hipError_t launch_scale_copy(hipStream_t s, const double2 *src, double2 *dst, double2 g, int64_t n);
hipError_t launch_density(hipStream_t s, const double2 *psi, double *rho, int64_t n);
hipError_t launch_region(hipStream_t s, const double2 *psi, const uint8_t *mask, int64_t n,
                         double *partials, double *out);
hipError_t launch_gershgorin(const Ctx &c, hipStream_t s, double *partials, double *out2);
hipError_t launch_holstein_obs(hipStream_t s, const double2 *psi, const uint8_t *occ,
                               const int32_t *up, int64_t nconf, int L, double *partials,
                               double *n_out, double *nph_out, double *chi_out);
int holstein_obs_blocks(int64_t nconf);
// one-workgroup persistent chain kernel: whole K-step run in one launch
bool chain_small_fits(int64_t n);
// The same run over several workgroups (chain.hip): R sites per thread, T
// threads, H halo sites per side (orders between exchanges), S own sites per
// workgroup (R T = S + 2 H), P workgroups; R = 0 when one workgroup runs it.
constexpr int kChainRing = 128;  // steps of norm/energy partials in flight (>= P + 1)
constexpr int kChainMaxWG = 64;  // most workgroups of one run
struct ChainMultiCfg {
    int R = 0, T = 0, H = 0;
    int64_t S = 0, P = 0;
};
ChainMultiCfg chain_multi_config(int64_t n);
size_t chain_multi_scratch_bytes(const ChainMultiCfg &cfg);
// device address of that run's timeout flag (int32) when it runs for c, else null
int32_t *chain_multi_timeout(const Ctx &c);
hipError_t launch_chain_small(const Ctx &c, hipStream_t s, double2 *psi, double2 *out,
                              const double2 *gamma_dev, int64_t K, double *norm_out,
                              double *energy_out, double2 *ckpt);
hipError_t launch_fill_zero(hipStream_t s, double *p, int64_t count);
hipError_t launch_csr_check(hipStream_t s, const int64_t *rowptr, const int32_t *col, int64_t n,
                            int64_t nnz, int64_t *flag);

// adjoint kernels (adjoint.hip)
hipError_t launch_recompute(const Ctx &c, hipStream_t s, const double2 *vk, const double2 *vkm1,
                            double2 *vkp1, int first);
// two orders per pass for chains and ribbons (adjoint.hip): the forward
// vectors without accumulation, and reverse levels k, k-1 together
hipError_t launch_recompute_pair(const Ctx &c, hipStream_t s, bool head, const double2 *vkm1, const double2 *vk,
                                 double2 *out1, double2 *out2);
hipError_t launch_adj_pair(const Ctx &c, hipStream_t s, bool has_u2, const double2 *uk2, const double2 *uk1,
                           double2 *out1, double2 *out2, const double2 *gbar, const double2 *vk,
                           const double2 *vkm1, double2 cg1, double2 cg2, double *grad);
hipError_t launch_adj_init(hipStream_t s, const double2 *gbar, double2 g, double2 *u, int64_t n);
// D = 3 .. 6 levels per pass (deep walk): recomputation storing v_{k+1} ..
// v_{k+D} to all[0 .. D-1] (head: v_1 .. v_D from psi = vk); adjoint levels
// k .. k-D+1 >= 1 from (u_{k+2} = uk2, may be null; u_{k+1} = uk1) into
// out1 = u_{k-D+2}, out2 = u_{k-D+1}, with the forward vectors v_{k-D+1} ..
// v_k stored n apart from fwd = v_{k-D+1} and cw[j-1] = conj(g_{k-j+1});
// adj_deep_fits tells whether the lattice allows D adjoint levels per pass.
hipError_t launch_recompute_deep(const Ctx &c, hipStream_t s, int D, int rows, bool head, const double2 *vkm1,
                                 const double2 *vk, double2 *const *all);
bool adj_deep_fits(const Ctx &c, int D);
hipError_t launch_adj_deep(const Ctx &c, hipStream_t s, int D, int rows, const double2 *uk2, const double2 *uk1,
                           double2 *out1, double2 *out2, const double2 *gbar, double *grad, const double2 *fwd,
                           const double2 *cw);
// D = 2 .. kMaxRevDepth adjoint levels k .. k-D+1 >= 0 per pass with the
// forward vectors regenerated downwards (v_{k-j} = 2 H~ v_{k-j+1} - v_{k-j+2})
// beside them: no stored forward vectors are read.  last0: level k-D+1 is
// level 0 (out2 = u_0; out1 and the forward outputs may then be null).
constexpr int kMaxRevDepth = 5;
struct RevPass {
    const double2 *uk2, *uk1;  // u_{k+2} (null: zero), u_{k+1}
    double2 *out1, *out2;      // u_{k-D+2}, u_{k-D+1}
    const double2 *gbar;
    double *grad;
    const double2 *v1, *v0;    // v_{k+1}, v_k
    double2 *vout1, *vout2;    // v_{k-D+1}, v_{k-D}
    double2 cw[kMaxRevDepth];  // conj(g_{k-j+1}), j = 1 .. D
    bool last0;
};
bool rev_deep_fits(const Ctx &c);
hipError_t launch_rev_deep(const Ctx &c, hipStream_t s, int D, int rows, const RevPass &p);
hipError_t launch_adj_level(const Ctx &c, hipStream_t s, const double2 *u1, double2 *u2_in,
                            const double2 *gbar_in, double2 *out, const double2 *vk, double2 gk,
                            double gscale, int has_u2, double *grad);

// small helpers
const char *hip_err_name(hipError_t e);

}  // namespace chebtd
