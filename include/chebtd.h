/*
 * chebtd -- Chebyshev time propagation of quantum states on one AMD MI355X
 * (gfx950) GPU.  C ABI.
 *
 * Method: Fehske, Schleede, Schubert, Wellein, Filinov, Bishop, "Numerical
 * approaches to time evolution of complex quantum systems", arXiv:0907.3022,
 * Sect. 2.2.  One time step applies
 *     U(dt) = e^{-i b dt} [ c_0 + 2 sum_{k=1}^{M} c_k T_k(H~) ],  eq. (U_1)
 * with H~ = (H - b)/a, c_k = (-i)^k J_k(a dt), computed through the
 * recursion v_{k+1} = 2 H~ v_k - v_{k-1}, v_1 = H~ v_0, v_0 = psi, and
 * truncated at the order M beyond which every |J_k(a dt)| < tol
 * (eq. (dec_Bessel)).  hbar = 1.
 *
 * Conventions shared by every entry point
 *  - Complex vectors are complex128, interleaved (re, im), contiguous, passed
 *    as double* pointing at the first real part.  Real vectors are float64.
 *  - Pointers named *_dev are device pointers (hipMalloc'd or torch CUDA
 *    tensors on the context's device); *_host are host pointers.
 *  - The caller owns every array it passes.  Builders borrow device arrays
 *    (potentials, CSR): they must stay alive and unchanged until the next
 *    builder call on the context or chebtd_destroy.
 *  - All GPU work is enqueued on the context's stream (chebtd_create) and is
 *    asynchronous unless a function says it synchronises.
 *  - Every function returns a status (0 = CHEBTD_OK, negative = error) and
 *    never throws; chebtd_last_error() describes the last failure.  A
 *    failing call leaves the context usable unless it returns CHEBTD_E_HIP.
 *  - One context must not be used from two host threads at once.
 */
#ifndef CHEBTD_H
#define CHEBTD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define CHEBTD_OK 0
#define CHEBTD_E_ARG (-1)      /* bad argument: null pointer, size, range  */
#define CHEBTD_E_HIP (-2)      /* a HIP runtime call failed                 */
#define CHEBTD_E_DIVERGED (-3) /* norm changed or became non-finite: the   */
                               /* spectral bounds do not enclose H          */
#define CHEBTD_E_OOM (-4)      /* device or host allocation failed          */
#define CHEBTD_E_STATE (-5)    /* call out of order (no H, no plan, ...)    */
#define CHEBTD_E_TIMEOUT (-6)  /* a persistent kernel's bounded wait ran   */
                               /* out; its results are invalid              */

/* ---- honeycomb ribbon edges ------------------------------------------- */
#define CHEBTD_ZIGZAG 0
#define CHEBTD_ARMCHAIR 1

/* ---- chebtd_propagate flags ------------------------------------------- */
#define CHEBTD_KEEP_CHECKPOINTS 1u /* store psi at every step for adjoint  */
#define CHEBTD_NO_CHECK 2u         /* skip the end-of-call norm check (no  */
                                   /* host synchronisation)                 */
#define CHEBTD_GRAPH 4u            /* replay each pair of steps from a     */
                                   /* captured hipGraph                     */
#define CHEBTD_NO_PERSISTENT 8u    /* chains of n <= 4096: passes launched  */
                                   /* per step instead of the whole run in  */
                                   /* one launch                            */
#define CHEBTD_SINGLE_ORDER 16u    /* chains and ribbons: one recursion     */
                                   /* order per pass instead of two         */

typedef struct chebtd_ctx chebtd_ctx;

/* ======================================================================= */
/* Context                                                                  */
/* ======================================================================= */

/* Create a context bound to the current HIP device and `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the handle. */
int chebtd_create(chebtd_ctx **out, void *hip_stream);

/* Release every device buffer the context owns.  NULL is a no-op. */
int chebtd_destroy(chebtd_ctx *ctx);

/* Re-bind the context to another stream of the same device. */
int chebtd_set_stream(chebtd_ctx *ctx, void *hip_stream);

/* Text of the last error on `ctx` (or of the last failed chebtd_create when
 * ctx is NULL).  Valid until the next call on the same context. */
const char *chebtd_last_error(const chebtd_ctx *ctx);

/* Library version as 10000*major + 100*minor + patch. */
int chebtd_version(void);

/* ======================================================================= */
/* Hamiltonians (Sect. 3).  Each call replaces the context's Hamiltonian    */
/* and invalidates its bounds and plan.                                     */
/* ======================================================================= */

/* 1D finite-difference Hamiltonian of Sect. 3.1: H = -(1/2) d^2/dx^2 + V(x)
 * on n points with spacing dx (m = hbar = 1), three-point Laplacian,
 * Dirichlet ends: H_jj = 1/dx^2 + V_j, H_{j,j+-1} = -1/(2 dx^2).
 * V_dev: float64[n] device array (borrowed).  n >= 1, dx > 0. */
int chebtd_h_chain1d(chebtd_ctx *ctx, int64_t n, double dx, const double *V_dev);

/* Honeycomb ribbon, eq. (model): H = -t sum_<ij> (c_i^+ c_j + h.c.)
 * + sum_j eps_j n_j, drawn as a brick wall on a width x length grid, site
 * index y*length + x.  CHEBTD_ZIGZAG: sites bond to (x+-1, y) and to
 * (x, y+1) if x+y is even, (x, y-1) if odd (zigzag edges at y = 0 and
 * y = width-1).  CHEBTD_ARMCHAIR: sites bond to (x, y+-1) and to (x+1, y)
 * if x+y is even, (x-1, y) if odd (armchair edges along x).  Open
 * boundaries.  eps_dev: float64[width*length] device array (borrowed). */
int chebtd_h_honeycomb(chebtd_ctx *ctx, int64_t width, int64_t length, int edge,
                       double t_hop, const double *eps_dev);

/* General Hermitian sparse H in CSR form (rows sorted or not, each entry
 * once): rowptr_dev int64[n+1], col_dev int32[nnz], val_dev complex128[nnz]
 * (interleaved), all device arrays (borrowed).  The structure is checked on
 * the device (synchronises): CHEBTD_E_ARG if rowptr does not run from 0 to
 * nnz without decreasing or a column lies outside [0, n).  The values must
 * describe a Hermitian matrix; that is not checked. */
int chebtd_h_csr(chebtd_ctx *ctx, int64_t n, int64_t nnz, const int64_t *rowptr_dev,
                 const int32_t *col_dev, const double *val_dev);

/* Generalised Holstein Hamiltonian, eq. (ghm), one spinless electron on L
 * sites (ring if periodic != 0, which needs L >= 3; open chain otherwise)
 * times phonon states with total phonon number <= nph (Sect. 3.3):
 *   H = sum_i Delta_i n_i - t sum_i (c_i^+ c_{i+1} + h.c.)
 *       - sum_i g_i w0 (b_i^+ + b_i) n_i + w0 sum_i b_i^+ b_i.
 * Basis: phonon configurations ordered by total phonon number, then
 * lexicographically ascending in (n_1..n_L) (n_1 most significant); state
 * index = electron site * nconf + rank, nconf = C(L+nph, nph), so that the
 * configurations of one site are contiguous (the electron hops and phonon
 * partners of neighbouring states then lie close together in memory).
 * g_host, Delta_host: float64[L] host
 * arrays (copied).  The operator is applied matrix-free (the memory-saving
 * scheme of Sect. 3.3): the context builds on the host, and owns on the
 * device, per-state tables of the raised and lowered phonon configuration
 * and the site occupation (9 B per state) instead of the matrix; these also
 * serve chebtd_holstein_obs.  Past 8M states the recursion forms the raised
 * and lowered configurations' ranks itself from a small table of binomials
 * and reads none of the per-state tables (environment CHEBTD_HOL_RANK=1 or
 * 0, read here, forces either way).  L * C(L+nph, nph) must stay below
 * 2^31. */
int chebtd_h_holstein(chebtd_ctx *ctx, int L, int nph, double t, double w0,
                      const double *g_host, const double *Delta_host, int periodic);

/* Host-side builder of the same Holstein matrix as CSR.  Call once with
 * rowptr/col/val = NULL to receive *n_out and *nnz_out, then again with
 * arrays of those sizes (rowptr int64[n+1], col int32[nnz], val complex128
 * [nnz]).  Entries of a row are sorted by column.  Needs no GPU. */
int chebtd_holstein_csr_host(int L, int nph, double t, double w0, const double *g_host,
                             const double *Delta_host, int periodic, int64_t *n_out,
                             int64_t *nnz_out, int64_t *rowptr, int32_t *col, double *val);

/* Occupation table of the Holstein basis above: occ[r*L + j] = phonons on
 * site j in configuration r (uint8[count*L]).  occ = NULL returns only
 * *count_out.  Needs no GPU. */
int chebtd_holstein_occupations(int L, int nph, int64_t *count_out, uint8_t *occ);

/* Dimension of the current Hamiltonian (0 if none). */
int64_t chebtd_dim(const chebtd_ctx *ctx);

/* ======================================================================= */
/* Spectral bounds and plan (Sect. 2.2)                                     */
/* ======================================================================= */

/* Gershgorin bounds of the current H: emin = min_i (H_ii - sum_{j!=i}|H_ij|),
 * emax = max_i (H_ii + sum_{j!=i}|H_ij|), computed on the device.
 * Synchronises the stream.  Does not change the context's bounds. */
int chebtd_gershgorin(chebtd_ctx *ctx, double *emin, double *emax);

/* Set the bounds used for H~ = (H-b)/a: b = (emax+emin)/2,
 * a = (emax - emin + alpha (emax-emin))/2 (the paper uses alpha = 0.01).
 * CHEBTD_E_ARG unless emax > emin and alpha >= 0. */
int chebtd_set_bounds(chebtd_ctx *ctx, double emin, double emax, double alpha);

/* Compute the weights of eq. (U_1) for step dt on the host (Miller's
 * backward recurrence for J_k) and upload them: gamma_0 = e^{-ib dt} J_0,
 * gamma_k = 2 e^{-ib dt} (-i)^k J_k(a dt), k = 1..M, where M is the last
 * order kept: |J_k(a dt)| < tol for every k > M (tol = 1e-15 in the
 * paper's spirit; tol <= 0 selects 1e-15).  Needs bounds.  Allocates the
 * context's work vectors; no later call allocates except where stated. */
int chebtd_plan(chebtd_ctx *ctx, double dt, double tol, int *M_out);

/* Like chebtd_plan but with a caller-chosen order M >= 0. */
int chebtd_plan_order(chebtd_ctx *ctx, double dt, int M);

/* Copy out the current plan: gamma_host complex128[M+1] (may be NULL),
 * a, b, dt and M (each may be NULL). */
int chebtd_get_plan(const chebtd_ctx *ctx, double *gamma_host, double *a, double *b,
                    double *dt, int *M);

/* The passes of one step on the multi-order path (1D chains longer than
 * the whole-run chain kernels, honeycomb ribbons; M >= 2): the Chebyshev
 * orders each pass advances, in launch order.  The first pass is the step
 * head (it also forms v_1 from psi); 2 runs the two-orders kernel, 3..6 the
 * deep kernel (that many orders of the recursion of Sect. 2.2 in one pass
 * over memory), 1 a single-order pass, only ever last.  The split is the
 * cheapest by each pass's time relative to a two-order pass, fixed by M and
 * the lattice (environment CHEBTD_DEPTH=D limits it to passes of 1, 2 and D
 * orders).  passes_out (int[capacity], may be NULL) receives up to capacity
 * entries; count_out receives the number of passes (0 when the plan runs
 * one order per launch).  Needs a plan. */
int chebtd_plan_passes(const chebtd_ctx *ctx, int *passes_out, int capacity, int *count_out);

/* ======================================================================= */
/* Propagation                                                              */
/* ======================================================================= */

/* Advance psi_dev (complex128[n], in/out) by K steps of dt.
 * norm_dev / energy_dev (float64[K] device arrays, or NULL) receive, for
 * s = 0..K-1, <psi_s|psi_s> and <psi_s|H|psi_s> of the state entering step
 * s (psi_s = state after s steps).  Unless CHEBTD_NO_CHECK is set the call
 * synchronises at the end and returns CHEBTD_E_DIVERGED if the final norm
 * is not finite or differs from the initial one by more than the check
 * tolerance (chebtd_set_check_tol, default 1e-6 relative).
 * CHEBTD_KEEP_CHECKPOINTS stores psi_s for the adjoint (CHEBTD_ADJ_REVERSE:
 * also v_{M-1} and v_M of every step); it needs chebtd_reserve_adjoint with
 * K <= its max_steps.
 * A 1D chain of 129 .. 4096 sites runs the whole call in one launch over
 * several workgroups that wait on each other (bounded to two seconds per
 * wait): if a wait runs out (workgroups not all resident, e.g. beside other
 * work filling the GPU) psi is left NaN and, unless CHEBTD_NO_CHECK is set,
 * the call returns CHEBTD_E_TIMEOUT.  Environment CHEBTD_CHAIN_MULTI=0 keeps
 * such runs in one workgroup. */
int chebtd_propagate(chebtd_ctx *ctx, double *psi_dev, int64_t K, double *norm_dev,
                     double *energy_dev, unsigned flags);

/* Time-dependent on-site term (Sect. 2.2: for a time-dependent H the
 * variation of H(t) bounds the step).  H is held constant within each step at
 * the caller's values for that step -- taking them at the step's midpoint
 * makes the scheme second order in dt.  onsite_dev + s*stride (float64)
 * holds, for step s = 0..K-1, V (chain, n values), eps (ribbon, n values) or
 * Delta_i (Holstein, L values); the rest of H is the one built.  The bounds
 * and the plan stay fixed, so they must enclose the spectrum of every step's
 * H.  One launch sequence per step (no graph, no persistent kernel, no
 * checkpoints); norm_dev, energy_dev and flags as chebtd_propagate. */
int chebtd_propagate_td(chebtd_ctx *ctx, double *psi_dev, int64_t K, const double *onsite_dev,
                        int64_t stride, double *norm_dev, double *energy_dev, unsigned flags);

/* Crank-Nicolson, eq. (CN), the comparison method of Sect. 2.2 and Table 1:
 * S steps of (1 + i dt H/2) psi_{s+1} = (1 - i dt H/2) psi_s for the chain
 * built by chebtd_h_chain1d (second order in dt, unitary).  The
 * step-independent tridiagonal factors are computed on the host; one
 * 256-thread workgroup then runs all S steps with the state in registers
 * (n <= 4096, else CHEBTD_E_ARG).  psi_dev: complex128[n] device array,
 * overwritten.  dt > 0, S >= 0 (S = 0 leaves psi unchanged).  Needs no bounds
 * or plan; other kinds of Hamiltonian give CHEBTD_E_STATE.  Synchronises. */
int chebtd_crank_nicolson(chebtd_ctx *ctx, double *psi_dev, double dt, int64_t S);

/* Relative norm tolerance of the end-of-call check (default 1e-6). */
int chebtd_set_check_tol(chebtd_ctx *ctx, double rel_tol);

/* ======================================================================= */
/* Observables (Sect. 3.1 densities, Fig. 3 polaron quantities)             */
/* ======================================================================= */

/* Allocation-free variant of chebtd_region_sum, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Needs no context: n sites of
 * psi_dev (complex128[n]) and mask_dev (uint8[n], 0 or 1), sum into
 * out_dev[0] (float64), enqueued on hip_stream (a hipStream_t of the current
 * HIP device, NULL = null stream).  The per-block partial sums live in a
 * fixed device array of the library, one per GPU, of 33 KB, held until the
 * process ends; it allocates nothing and returns CHEBTD_E_ARG for n outside
 * [1, CHEBTD_NOALLOC_MAX_SITES].  The same kernels as chebtd_region_sum:
 * bit-identical results.  Calls that overlap on one GPU (other streams,
 * other host threads) share that array and race; serialise them.  Errors
 * are reported through chebtd_last_error(NULL). */
#define CHEBTD_NOALLOC_MAX_SITES 16777216
int chebtd_region_sum_noalloc(const double *psi_dev, const uint8_t *mask_dev, int64_t n,
                              double *out_dev, void *hip_stream);

/* rho_dev[i] = |psi_i|^2 (float64[n]). */
int chebtd_density(chebtd_ctx *ctx, const double *psi_dev, double *rho_dev);

/* out_dev[0] = sum_i mask_i |psi_i|^2 with mask_dev uint8[n] (0 or 1),
 * e.g. the transmission into x > 0.  Deterministic reduction. */
int chebtd_region_sum(chebtd_ctx *ctx, const double *psi_dev, const uint8_t *mask_dev,
                      double *out_dev);

/* out2_dev[0] = <psi|psi>, out2_dev[1] = <psi|H|psi> (needs bounds). */
int chebtd_norm_energy(chebtd_ctx *ctx, const double *psi_dev, double *out2_dev);

/* Holstein observables of Fig. 3 for the Hamiltonian built by
 * chebtd_h_holstein: n_dev[i] = <n_i>, nph_dev[i] = <b_i^+ b_i>,
 * chi_dev[i] = <n_i (b_i + b_i^+)> (each float64[L]). */
int chebtd_holstein_obs(chebtd_ctx *ctx, const double *psi_dev, double *n_dev,
                        double *nph_dev, double *chi_dev);

/* ======================================================================= */
/* Batched propagation of many independent ribbons                          */
/* ======================================================================= */

/* One ribbon of a batch (a disorder realisation with its own packet). */
typedef struct {
    int64_t width, length; /* grid, as chebtd_h_honeycomb               */
    int edge;              /* CHEBTD_ZIGZAG or CHEBTD_ARMCHAIR          */
    double t_hop;          /* hopping t                                 */
    const double *eps_dev; /* float64[width*length], borrowed           */
    double emin, emax;     /* spectral bounds (e.g. Gershgorin)         */
    double *psi_dev;       /* complex128[width*length], propagated in   */
                           /* place, borrowed                           */
} chebtd_sys_desc;

/* Prepare a batch of nsys ribbons stepped by the same dt (each with its
 * own a, b, M and weights; alpha and tol as chebtd_set_bounds/plan).
 * Allocates the batch's work vectors (four per system) and schedule tables.
 * Replaces any previous batch on the context. */
int chebtd_batch_create(chebtd_ctx *ctx, int nsys, const chebtd_sys_desc *descs, double dt,
                        double alpha, double tol);

/* Schedules for chebtd_batch_propagate. */
#define CHEBTD_SCHED_LEVELS 0     /* one launch per recursion level over   */
                                  /* every system                           */
#define CHEBTD_SCHED_PERSISTENT 1 /* one persistent launch per step: a     */
                                  /* work queue of (level, system, tile)    */
                                  /* with per-system completion counters    */
#define CHEBTD_SCHED_PAIRS 2      /* one launch per two recursion orders    */
                                  /* over every system still active (needs  */
                                  /* M >= 2 everywhere), plus one tail      */
                                  /* launch for systems with odd M           */
#define CHEBTD_SCHED_DEEP 3       /* passes of D (5; 4..6 by environment  */
                                  /* CHEBTD_BATCH_DEPTH) or D + 1 orders:   */
                                  /* each system takes the fewest that     */
                                  /* cover its M, one launch per pass and   */
                                  /* depth, then two-order and one-order    */
                                  /* passes for what is left (needs M >= D  */
                                  /* everywhere)                            */

/* Fix the schedule: mode, rows per tile (multiple of block, >= block),
 * threads per block (64..1024, multiple of 64), and for the persistent
 * mode the number of resident workgroups per CU (1..8).  The pairs mode
 * walks whole ribbons with 256-thread blocks; its tile and block apply to
 * the odd-M tail and the final copy. */
int chebtd_batch_set_schedule(chebtd_ctx *ctx, int mode, int tile_rows, int block,
                              int wg_per_cu);

/* Time candidate schedules on the real batch (a few steps each, the
 * systems' psi are saved and restored, also when the search fails; a
 * candidate that is refused or times out is skipped) and keep the fastest.  If
 * cache_path is non-NULL the choice is read from / appended to that text
 * file, keyed by the batch's shape.  Synchronises.  best_out (int[4], may be
 * NULL) receives mode, tile_rows, block, wg_per_cu. */
int chebtd_batch_autotune(chebtd_ctx *ctx, const char *cache_path, int *best_out);

/* Advance every system of the batch by K steps.  psi_dev: NULL to propagate
 * the states bound before (at chebtd_batch_create or by an earlier call), or
 * a host array of nsys device pointers (complex128[width*length] each, in
 * place): system s then propagates psi_dev[s], in this call and later ones,
 * without re-planning (the kernels and a captured graph read the states from
 * the batch's device table, which is re-uploaded on the stream when the
 * pointers change).  K = 0 only re-binds.  flags: CHEBTD_GRAPH replays a
 * captured hipGraph per pair of steps; CHEBTD_NO_CHECK skips the final
 * synchronisation that reports CHEBTD_E_TIMEOUT. */
int chebtd_batch_propagate(chebtd_ctx *ctx, double *const *psi_dev, int64_t K, unsigned flags);

/* Number of systems and, per system, its order M (int[nsys], may be NULL). */
int chebtd_batch_info(const chebtd_ctx *ctx, int *nsys, int *M_host);

/* ======================================================================= */
/* Adjoint: dL/dV for the on-site potential (V of chebtd_h_chain1d, eps of  */
/* chebtd_h_honeycomb).  Reverse mode of the recursion above with (a, b)    */
/* held fixed:  u_M = conj(g_M) gbar,                                       */
/*   u_k = conj(g_k) gbar + 2 H~ u_{k+1} - u_{k+2}   (1 <= k < M),          */
/*   u_0 = conj(g_0) gbar + H~ u_1 - u_2,                                   */
/*   dL/dV_i += (1/a) Re[conj(u_1,i) v_0,i + 2 sum_{k=1}^{M-1}              */
/*                        conj(u_{k+1},i) v_k,i],                           */
/* per step in reverse, gbar <- u_0.  gbar follows the convention           */
/* dL = Re sum_i conj(gbar_i) dpsi_i (the gradient torch reports for a     */
/* complex tensor under a real loss).                                       */
/* ======================================================================= */

/* Adjoint memory schedules. */
#define CHEBTD_ADJ_STEP 0  /* recompute each step's M+1 vectors into a     */
                           /* buffer, then sweep back                       */
#define CHEBTD_ADJ_SQRTM 1 /* keep psi_s only; the backward pass rebuilds */
                           /* each step's (v_{j-1}, v_j) pairs about every */
                           /* ceil(sqrt(M)) orders in one forward pass and */
                           /* regenerates the vectors between them         */
                           /* downwards, restarting from each stored pair  */
                           /* (chains and ribbons within the deep walk's   */
                           /* offset limit); elsewhere it recomputes       */
                           /* segment by segment from the pairs             */
#define CHEBTD_ADJ_REVERSE 2 /* keep each step's last two vectors           */
                             /* (v_{M-1}, v_M) beside psi_s and regenerate  */
                             /* v_{M-2} .. v_0 downwards, v_{k-1} =         */
                             /* 2 H~ v_k - v_{k+1}, inside the passes that  */
                             /* run the adjoint levels: nothing is          */
                             /* recomputed forwards.  3 vectors per step;   */
                             /* chains and ribbons within the deep walk's   */
                             /* offset limit ((W + 14) L 16 B <= 2^31)      */

/* Allocate the adjoint's storage: psi checkpoints for up to max_steps steps
 * and the recompute buffers of `mode` (CHEBTD_ADJ_REVERSE: also the step-end
 * pairs, 2 more vectors per step).  Needs a plan (chain or honeycomb);
 * CHEBTD_E_ARG for CHEBTD_ADJ_REVERSE on a lattice past its offset limit. */
int chebtd_reserve_adjoint(chebtd_ctx *ctx, int64_t max_steps, int mode);

/* After chebtd_propagate(..., K, ..., CHEBTD_KEEP_CHECKPOINTS): gbar_dev
 * (complex128[n]) holds dL/dpsi_K on entry and the adjoint of psi_0 on
 * return; dLdV_dev (float64[n]) is accumulated into (+=).  After a run of
 * K = 0 steps both are left as they are.  On ribbons the
 * reverse sweep runs several levels per pass over memory and CHEBTD_ADJ_STEP
 * recomputes several orders per pass; CHEBTD_ADJ_REVERSE regenerates the
 * forward vectors downwards.  The modes group the levels differently and
 * agree to rounding, not bit for bit. */
int chebtd_adjoint(chebtd_ctx *ctx, double *gbar_dev, double *dLdV_dev);

/* Every chebtd_propagate call with CHEBTD_KEEP_CHECKPOINTS overwrites the
 * stored trajectory and numbers the run (1, 2, ... per context).
 * chebtd_checkpoint_run sets *run_id to the number of the run whose
 * checkpoints are stored and valid for the current plan, or 0 if none (no
 * such run since chebtd_reserve_adjoint, or a new Hamiltonian or plan since).
 * chebtd_adjoint_run is chebtd_adjoint for that run only: it returns
 * CHEBTD_E_STATE, touching neither gbar_dev nor dLdV_dev, if run_id is not
 * the stored run (its checkpoints were overwritten by a later run).
 * run_id = 0 accepts the stored run, as chebtd_adjoint does. */
int chebtd_checkpoint_run(const chebtd_ctx *ctx, int64_t *run_id);
int chebtd_adjoint_run(chebtd_ctx *ctx, int64_t run_id, double *gbar_dev, double *dLdV_dev);

/* ======================================================================= */
/* Measurement helpers                                                      */
/* ======================================================================= */

/* Launch the current Hamiltonian's recursion kernel (the hot loop) `launches`
 * times on the context's stream between two hipEvents, on scratch vectors
 * (allocated and freed here), and return the mean time per launch in
 * milliseconds, the kernel's name and the recursion orders one launch
 * advances.  On the multi-order path that is the pass the step runs most
 * often after its head (chebtd_plan_passes; 2 for the two-orders kernel, 3..6
 * for the deep kernel), else 1; CHEBTD_SINGLE_ORDER in `flags` times the
 * one-order kernel.  The Holstein and CSR kernels are timed in the pattern a
 * step runs them: two launches without the accumulator for every one that
 * updates it with three orders.  Needs a plan.  Synchronises.
 * name_out and orders_out may be NULL. */
int chebtd_time_recursion_kernel(chebtd_ctx *ctx, int launches, unsigned flags, double *ms_per_launch,
                                 const char **name_out, int *orders_out);

#ifdef __cplusplus
}
#endif

#endif /* CHEBTD_H */
