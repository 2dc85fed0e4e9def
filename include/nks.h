/*
 * nks.h -- C ABI of libnks, the nested Krylov-Ritz matrix sign function
 * (Bloch & Heybrock, "A nested Krylov subspace method to compute the sign
 * function of large complex matrices") for the lattice operator
 *
 *     A = gamma5 D_w(mu),   D_w(mu) as defined in Sec. 2 of the paper,
 *
 * on AMD MI355X (gfx950).  The library computes y ~ sgn(A) b by
 *   (1) k steps of Lanczos (mu = 0, App. A) or two-sided Lanczos (mu != 0,
 *       App. B) on A from b,
 *   (2) the nested step of Sec. 4.1 / App. C: LU of p H_k, ell steps of
 *       (two-sided) Lanczos on H_k' = (p H_k + (p H_k)^{-1}) / 2 from e_1,
 *       Roberts-Higham iteration (Eq. Roberts) on H_ell,
 *   (3) the lift y = |b| V_k V_ell sgn(H_ell) e_1 (Eq. nested).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - dims = {Lx, Ly, Lz, Lt}, each >= 2, periodic in all four directions.
 *   Site index s = x + Lx*(y + Ly*(z + Lz*t)); V = Lx*Ly*Lz*Lt; n = 12 V.
 * - Vectors (b, x, in, out) are DEVICE pointers to n interleaved complex128
 *   values (re, im), component index 12*s + 3*spin + colour.
 * - Links are a DEVICE pointer to 4*9*V complex128 values, index
 *   ((s*4 + nu)*3 + row)*3 + col, nu = 0..3 for x, y, z, t.  Link U_{s,nu}
 *   transports from site s to s + nu_hat: the hop of D_w(mu) that lands on
 *   y brings psi(y - nu_hat) with (1 + gamma_nu) U_{y-nu_hat,nu} and
 *   psi(y + nu_hat) with (1 - gamma_nu) U_{y,nu}^dagger (Sec. 2).
 * - Dirac matrices: chiral basis, gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]
 *   (k = 1..3), gamma_4 = [[0, 1], [1, 0]], gamma5 = diag(1, 1, -1, -1).
 * - m0 > 0 is the negative Wilson mass: m_w = -m0 in (-2, 0) and
 *   kappa = 1 / (8 + 2 m_w).  mu is the real chemical potential; the forward
 *   time hop carries e^{+mu}, the backward one e^{-mu}.
 * - stream arguments are hipStream_t passed as void* (NULL = default
 *   stream).  Calls are asynchronous on the stream unless stated otherwise;
 *   the caller keeps every buffer alive until the stream has completed.
 * - Ownership: the caller owns b, x, links and workspaces; the library
 *   owns only what it allocates inside nks_ctx / nks_lattice and never
 *   frees caller memory or keeps caller pointers past the call.
 * - Errors: every int-returning function returns NKS_OK or an NKS_E_* code;
 *   nks_last_error(ctx) gives a message for the last failure on ctx.
 *   Outcomes found on the device (breakdown, no convergence) come back in
 *   nks_stats.status.
 * - A context is not thread-safe: use one nks_ctx per host thread.
 */
#ifndef NKS_H
#define NKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NKS_ABI_VERSION 3

/* Largest number of nested levels (Sec. 4.5); see nks_opts.levels. */
#define NKS_MAX_LEVELS 6

enum nks_status {
    NKS_OK = 0,
    NKS_E_INVALID = 1,      /* bad argument (sizes, pointers, m0 out of range) */
    NKS_E_NOMEM = 2,        /* workspace too small or allocation failure */
    NKS_E_HIP = 3,          /* HIP runtime or launch error */
    NKS_E_UNSUPPORTED = 4,  /* valid but not supported (e.g. non-nested k too large) */
    NKS_E_BREAKDOWN = 5,    /* serious two-sided Lanczos breakdown (App. B) */
    NKS_E_NOCONV = 6        /* Roberts-Higham or ell-doubling did not converge */
};

enum nks_precision {
    NKS_FP64 = 0,   /* every vector and scalar in float64 */
    NKS_MIXED = 1   /* float32 stencil and basis vectors, float64 recurrence
                       coefficients, nested step and lift accumulation */
};

enum nks_policy {
    NKS_POLICY_FIXED = 0,     /* use opts.k / opts.ell as given */
    NKS_POLICY_DOUBLING = 1,  /* ell: double from 16 until the coefficient change
                                 is <= tol/10; k: checkpoints every 100 steps until
                                 the change is <= tol/4 (k stays <= opts.k) */
    NKS_POLICY_LEARNED = 2    /* predicted by the network of nks_policy_load
                                 (see there), verified, falls back to DOUBLING */
};

/* Options of one sign application.  Initialise with nks_opts_default(). */
typedef struct nks_opts {
    size_t size;          /* sizeof(nks_opts), for versioning */
    int k;                /* outer Krylov size (the largest k under the k policy); rounded up to even */
    int ell;              /* inner Krylov size (the largest under the ell policy); rounded up to
                             even; ell >= k -> non-nested RHi on H_k.  The dense RHi matrix
                             (ell, or k when non-nested) is limited to 1024 (NKS_E_UNSUPPORTED) */
    double tol;           /* target relative accuracy for the policies */
    int precision;        /* enum nks_precision */
    double p;             /* preconditioner factor of Eq. precond; <= 0 -> p_opt of Eq. popt
                             estimated from the Ritz values of H_k, with z_max capped at
                             1 + kappa (6 sqrt 2 + 2 sqrt(2 cosh 2 mu)) >= ||A|| (a larger
                             |theta| is a spurious two-sided Ritz value); nks_nested_step,
                             which has no lattice, does not cap */
    int k_policy;         /* enum nks_policy */
    int ell_policy;       /* enum nks_policy */
    int max_rhi_iter;     /* Roberts-Higham iteration cap (default 50) */
    double rhi_tol;       /* relative Frobenius change that ends RHi (default 1e-14) */
    unsigned flags;       /* NKS_FLAG_* bits; others give NKS_E_INVALID */
    /* Multi-level nesting (Sec. 4.5, Fig. 12).  levels = L nested levels,
     * 1..NKS_MAX_LEVELS (1 = the nested method; default).  Level 0 is H_k; level
     * i builds the Krylov space of size k_{i+1} of the preconditioned Ritz
     * matrix of level i (Eq. precond with p_i), and RHi runs on the Ritz matrix
     * of the deepest level.  k_1 = ell; ell_deep[i] = k_{i+2} for
     * i < levels - 1 (each >= 1, rounded up to even).  A size that is not
     * below the size of the level above makes that level exact (RHi on its
     * Ritz matrix) and ends the recursion there.  p_deep[i] = p_{i+1} (<= 0:
     * p_opt of Eq. popt from the Ritz values of that level; level 0 uses p).
     * levels > 1 needs the FIXED ell policy and a FIXED or DOUBLING k policy
     * (NKS_E_UNSUPPORTED otherwise). */
    int levels;
    int ell_deep[NKS_MAX_LEVELS - 1];
    double p_deep[NKS_MAX_LEVELS - 1];
} nks_opts;

/* flags: return the overlap operator D_ov(mu) b = b + gamma5 sgn(A) b
 * (Sec. 2, Eq. Dovmu; A = gamma5 D_w(mu), gamma5 = diag(1, 1, -1, -1) in
 * spin) instead of sgn(A) b.  The identity and gamma5 terms are added by
 * the lift kernel; everything else is the sign application. */
#define NKS_FLAG_OVERLAP 1u
/* flags: deflate with the eigenpairs set on the job's lattice
 * (nks_lattice_set_deflation; App. C steps 1 and 6): the method runs on
 * b_m = b - sum_i <l_i, b> r_i and adds sum_i sgn(Re lambda_i) <l_i, b> r_i.
 * NKS_E_INVALID if the lattice has none. */
#define NKS_FLAG_DEFLATE 2u
/* flags: double-pass low-memory mode (Sec. 4.4).  The outer pass keeps only
 * the two newest basis vectors; after the nested step the basis is built a
 * second time from b (the same kernels, bit for bit the same vectors) and
 * summed with the lift weights on the way.  Memory per job O(n) instead of
 * O(n k) (see nks_workspace_size), at twice the outer-pass cost; results are
 * identical to the single-pass ones bit for bit. */
#define NKS_FLAG_DOUBLE_PASS 4u

/* Per-result report (filled after the stream completes). */
typedef struct nks_stats {
    int status;           /* NKS_OK, NKS_E_BREAKDOWN or NKS_E_NOCONV */
    int k_used;           /* outer basis size actually built (lucky breakdown -> smaller) */
    int ell_used;         /* inner basis size actually used (0 = non-nested) */
    int rhi_iters;        /* Roberts-Higham iterations */
    double p_used;        /* preconditioner factor used */
    double z_min, z_max;  /* Ritz-value extremes |theta| used for p, z_max after the cap
                             above (0 if p was given) */
    double b_norm;        /* |b| */
    int breakdown_iter;   /* iteration of a serious breakdown, else 0 */
    double inner_delta;   /* last ell-doubling relative change (policies), else 0 */
    double outer_delta;   /* last k-checkpoint relative change (policies), else 0 */
    float ms_outer, ms_nested, ms_lift;  /* device time per phase (single-job calls; ms_lift
                                            includes the second pass of NKS_FLAG_DOUBLE_PASS) */
    int levels_used;      /* nested levels that ran (0 = non-nested; < opts.levels when a
                             level was exact or the result came from a smaller setting) */
    int ell_deep_used[NKS_MAX_LEVELS - 1];   /* k_{i+2} built at the deeper levels */
    double p_deep_used[NKS_MAX_LEVELS - 1];  /* p_{i+1} used at the deeper levels */
} nks_stats;

typedef struct nks_ctx nks_ctx;
typedef struct nks_lattice nks_lattice;

/* One job of a batched call: x ~ sgn(A) b on lattice lat. */
typedef struct nks_job {
    nks_lattice* lat;
    const void* b;        /* device, n complex128 */
    void* x;              /* device, n complex128 */
    const nks_opts* opts;
} nks_job;

/* Fill *o with defaults: k=200, ell=50, tol=1e-8, FP64, p auto, FIXED policies,
 * one nested level. */
void nks_opts_default(nks_opts* o);

/* Create a context on HIP device `device` (makes it current). */
int nks_create(int device, nks_ctx** out);
void nks_destroy(nks_ctx* ctx);
const char* nks_last_error(nks_ctx* ctx);
const char* nks_status_str(int status);

/* Copy the links (device complex128, layout above) into the lattice's own
 * float64 and float32 structure-of-arrays copies.  Params default to
 * m0 = 1.6, mu = 0.  Blocks until the copy is done. */
int nks_lattice_create(nks_ctx* ctx, const int32_t dims[4], const void* links_dev,
                       nks_lattice** out);
/* Set m0 (m_w = -m0 must lie in (-2, 0)) and mu.  mu == 0 selects Lanczos,
 * mu != 0 two-sided Lanczos. */
int nks_lattice_set_params(nks_lattice* lat, double m0, double mu);
void nks_lattice_destroy(nks_lattice* lat);

/* Deflation data for later NKS_FLAG_DEFLATE jobs on this lattice (App. C
 * step 1): m (0..64) eigenpairs of A.  r_dev, l_dev: device, m complex128
 * vectors each in the caller's layout ([i][12*site + 3*spin + colour]);
 * l_dev NULL means l_i = r_i (A Hermitian).  The caller normalises them
 * biorthonormally, l_i^dagger r_j = delta_ij.  lambda_host: 2m doubles,
 * interleaved complex eigenvalues; Re(lambda_i) = 0 gives NKS_E_INVALID.
 * The vectors are copied into the lattice (2 m 12 V complex128); m = 0
 * switches deflation off.  Waits for the device. */
int nks_lattice_set_deflation(nks_lattice* lat, int m, const void* r_dev, const void* l_dev,
                              const double* lambda_host);

/* Deflation eigenpairs computed on the GPU: the m (1..64) eigenpairs of A
 * with the smallest |lambda| (App. C step 1), by Chebyshev-filtered subspace
 * iteration on A^2 (a block of m + max(8, m) vectors, filter degree 40, the
 * interval bound ||A||^2 <= (1 + kappa (6 sqrt(2) + 2 sqrt(2 cosh 2mu)))^2,
 * Rayleigh-Ritz on A^2 ordered by |theta^2|, then on A within the first m
 * vectors), until every |A r_i - lambda_i r_i| <= tol (r_i unit vectors) or
 * max_iter iterations.  mu = 0: l_i = r_i.  mu != 0: the left eigenvectors
 * come from a second run on A^dagger = A(-mu), paired by eigenvalue and
 * scaled to l_i^dagger r_i = 1; the residuals are the larger of the two
 * runs' and iters counts both; NKS_E_NOCONV also if the two sets do not
 * pair up (a tie in |lambda| at the m-th eigenvalue).  On success the pairs
 * are installed on the lattice as by nks_lattice_set_deflation; on an error
 * the lattice keeps no deflation.  lambda_host (2m doubles, interleaved
 * complex, ascending |lambda|), resid_host (m doubles) and iters may be
 * NULL.  The p x p Cholesky, Jacobi and Hessenberg-QR steps run on the host.
 * Uses the null stream and waits. */
int nks_lattice_eigensolve(nks_lattice* lat, int m, int max_iter, double tol, double* lambda_host,
                           double* resid_host, int* iters);
/* The lattice's deflation eigenvectors (as set or computed above): *m_out =
 * their number; r_dev, l_dev (device, m complex128 vectors each in the
 * caller's layout, either may be NULL) receive copies.  Waits. */
int nks_lattice_get_deflation(nks_lattice* lat, int* m_out, void* r_dev, void* l_dev);

/* out = A in (dagger = 0) or A^dagger in (dagger = 1), A = gamma5 D_w(mu);
 * A(mu)^dagger = gamma5 D_w(-mu).  precision NKS_MIXED runs the float32
 * stencil (inputs and outputs stay complex128).  in and out must not alias. */
int nks_apply_op(nks_lattice* lat, const void* in, void* out, int dagger, int precision,
                 void* stream);

/* Device workspace bytes needed by nks_sign_apply_batch for these jobs (and
 * by nks_sign_apply for one job).  Dominated by the outer basis: n*k*16
 * bytes per FP64 job, n*k*8 per mixed job. */
int nks_workspace_size(nks_ctx* ctx, int njobs, const nks_job* jobs, size_t* bytes);

/* x ~ sgn(A) b (Eq. nested; non-nested when ell >= k).  ws is a device
 * buffer of at least nks_workspace_size bytes.  If stats != NULL the call
 * waits for the stream and fills *stats. */
int nks_sign_apply(nks_ctx* ctx, nks_lattice* lat, const void* b, void* x,
                   const nks_opts* opts, void* ws, size_t ws_bytes, void* stream,
                   nks_stats* stats);

/* nks_sign_apply for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels and result, but the workspace is a static array of
 * NKS_NOALLOC_BYTES that the library holds on every GPU it runs on until the
 * process ends (its address is taken once per GPU by nks_create), and the
 * call makes no allocation of any kind on the device (no hipMalloc, hipFree,
 * stream, event or graph): the job table is copied into the array and the
 * kernels launched eagerly on `stream`.  A job whose workspace
 * (nks_workspace_size) exceeds NKS_NOALLOC_BYTES gives NKS_E_NOMEM with the
 * size in nks_last_error (NKS_FLAG_DOUBLE_PASS needs O(n) memory: 12 MB for
 * one 10^4 job at k = 500).  Every call on one GPU uses the same array, which
 * keeps the last call's contents: calls that overlap on one GPU (on
 * different streams, or from different contexts or threads) race and must
 * be ordered by the caller.  Nothing needs clearing between calls (the
 * kernels initialise what they read).  If stats != NULL the call waits for
 * the stream and fills *stats. */
#define NKS_NOALLOC_BYTES (64u << 20)
int nks_sign_apply_noalloc(nks_ctx* ctx, nks_lattice* lat, const void* b, void* x,
                           const nks_opts* opts, void* stream, nks_stats* stats);

/* Many jobs in one call: jobs on the same lattice (and precision) run in the
 * same stencil and recurrence launches, one workgroup per (site block, job)
 * (each reads the links of its site block itself; launch maps 1 and 3 put
 * the jobs of a site block on one XCD, so that those reads can be served by
 * its L2).  In graph mode (the default, tuning key "graph") a call
 * without stats and without profiling captures its whole launch sequence
 * into a HIP graph on a private stream, keyed by the job table (every
 * pointer, size and option) and the workspace address, and later calls
 * with the same key replay it on `stream` (up to 4 graphs are kept per
 * context).  A call with stats runs eagerly.  stats is NULL or an array of
 * njobs entries (then the call waits for the stream).  The library keeps a
 * host copy of the job table until the next call on the context. */
int nks_sign_apply_batch(nks_ctx* ctx, int njobs, const nks_job* jobs, void* ws,
                         size_t ws_bytes, void* stream, nks_stats* stats);

/* Row-level entry points (the steps of App. C one at a time). */

/* Steps 1-2 of the method: build the outer basis from b and return the
 * tridiagonal Ritz matrix on the host: alpha[k] (H(j,j)), beta[k-1]
 * (H(j+1,j)), gamma[k-1] (H(j,j+1)), each as interleaved complex128
 * (imaginary parts 0 when mu = 0).  Waits for the stream. */
int nks_outer_basis(nks_ctx* ctx, nks_lattice* lat, const void* b, const nks_opts* opts,
                    void* ws, size_t ws_bytes, void* stream, double* alpha_host,
                    double* beta_host, double* gamma_host, nks_stats* stats);

/* Steps 3-5 on a given tridiagonal H_k (host arrays as returned by
 * nks_outer_basis; hermitian != 0 treats it as real symmetric): returns
 * c ~ sgn(H_k) e_1 (k interleaved complex128 on the host), with
 * opts.levels nested levels (Sec. 4.5).  Waits. */
int nks_nested_step(nks_ctx* ctx, int k, const double* alpha_host, const double* beta_host,
                    const double* gamma_host, int hermitian, const nks_opts* opts,
                    double* c_host, nks_stats* stats);

/* Predictor network of the learned ell/k policy: MLP 16 -> 64 -> 64 -> 2
 * with SiLU, parameters as one float32 vector of NKS_MLP_NPARAMS entries
 * (W1[16][64], b1[64], W2[64][64], b2[64], W3[64][2], b3[2]; z = h W + b).
 * Products run on bf16 MFMA with bfloat16 operands (round to nearest even)
 * and float32 accumulation.  All pointers are device pointers; x is
 * [batch][16], y and t are [batch][2].  Asynchronous on the stream. */
#define NKS_MLP_NPARAMS 5378
int nks_mlp_forward(nks_ctx* ctx, const float* params, const float* x, int batch, float* y, void* stream);
/* grad = gradient of 0.5 * mean_b ||y_b - t_b||^2; *loss = that loss. */
int nks_mlp_backward(nks_ctx* ctx, const float* params, const float* x, const float* t, int batch,
                     float* grad, float* loss, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on params with moments
 * m, v; step counts from 1. */
int nks_mlp_adam_step(nks_ctx* ctx, float* params, const float* grad, float* m, float* v, int step,
                      float lr, void* stream);

/* Learned ell/k policy (NKS_POLICY_LEARNED; not part of the paper).
 *
 * After R_{k0} (k0 = NKS_LEARN_K0 outer steps) the nested kernel computes
 * NKS_POLICY_NFEAT features of the Ritz matrix H_{k0}:
 *   f0 = 1, f1 = log10 zmin(H_{k0}), f2 = log10 zmax(H_{k0}),
 *   f3 = log10 zmin(H_{k0/2}), f4 = log10(zmax/zmin), f5 = mu, f6 = log10 tol,
 *   f7 = 1 for the two-sided recurrence else 0, f8 = log10 V,
 *   f9 = mean |alpha_i|, f10 = mean sqrt|beta_i gamma_i|, f11..f15 = 0
 * (zmin, zmax: smallest and largest |Ritz value|, the estimates used for
 * p_opt), normalises them, and evaluates the network (bf16 weights and
 * layer inputs, float32 accumulation) for t = (log10 k*, log10 ell*).
 * The k policy stops at k_t = k* rounded up to a multiple of
 * NKS_LABEL_DK (at least k0 + 20, else no target) and accepts H_{k_t}
 * if the weighted coefficient change against H_{k_t - 40} is <= tol/4;
 * otherwise it continues with the checkpoints of NKS_POLICY_DOUBLING.  The
 * ell policy starts its doubling at the largest power of two <= 1.05 ell*
 * (>= 8), with the DOUBLING acceptance rule.  A learned policy on a job with k <= k0 + 20
 * behaves as DOUBLING.
 *
 * nks_policy_load copies a network to the device, for every later call
 * on ctx.  blob (host) holds NKS_POLICY_NFLOATS float32 values:
 * [NKS_MLP_NPARAMS parameters][16 feature means][16 feature scales]
 * [2 target means][2 target scales]; x_i = (f_i - mean_i) / scale_i and
 * t = y * scale + mean.  Scales must be > 0 and every value finite
 * (NKS_E_INVALID).  Waits for the device before it replaces a network. */
#define NKS_POLICY_NFEAT 16
#define NKS_POLICY_NFLOATS (NKS_MLP_NPARAMS + 2 * NKS_POLICY_NFEAT + 4)
#define NKS_LEARN_K0 100
int nks_policy_load(nks_ctx* ctx, const float* blob, int nfloats);

/* Training labels for the learned policy.  Runs each job's outer loop to
 * opts.k (FIXED policies only, else NKS_E_INVALID; x may be NULL) and
 * writes NKS_LABEL_WORDS doubles per job (labels_host[job][word], host):
 *   [0, 16)    the features above at k0 (f6 from opts.tol),
 *   [16, 76)   e_i, i < NKS_LABEL_NK: weighted relative change
 *              ||c(k_i) - c_ref||_w / ||c_ref||_w with k_i = 20 (i + 1), where
 *              c(k) is the nested result on H_k (ell doubled from 16 to a
 *              1e-13 change) and c_ref the same on H_{k_used};
 *              ||d||_w^2 = sum_i |d_i|^2 ||v_{i+1}||^2 (NaN for k_i > k_used),
 *   [76, 316)  for each k_i, the relative coefficient change of the ell
 *              doublings 16->32, 32->64, 64->128, 128->256 (NaN once the
 *              doubling stopped).
 * Jobs at mu != 0 (two-sided) give NKS_E_UNSUPPORTED: such label runs are
 * switched off until a GPU fault seen in one of them is explained.
 * Every k_i runs in a workgroup of its own with its own scratch (about
 * 61 times the nested scratch of a sign application per job).
 * Allocates its own workspace, uses the null stream and waits. */
#define NKS_LABEL_NK 60
#define NKS_LABEL_NELL 4
#define NKS_LABEL_DK 20
#define NKS_LABEL_WORDS (NKS_POLICY_NFEAT + NKS_LABEL_NK * (1 + NKS_LABEL_NELL))
int nks_policy_label(nks_ctx* ctx, int njobs, const nks_job* jobs, double* labels_host);

/* Launch-shape choices of the outer passes, per context (an autotuner sets
 * them after timing the alternatives):
 *   "xcd_map"    1: 1D grid that keeps every job of a site block on one XCD
 *                2: 1D grid that gives each XCD whole jobs (all site blocks)
 *                3: 1D grid that gives each XCD half of the lattice (in t)
 *                   for a quarter of the jobs
 *                0: 2D grid (site block, job)
 *   "split_dual" 1: the two-sided stencil computes A u and A^dagger t in
 *                separate workgroups; 0: one thread does both.
 *   "min_waves"  1, 3 or 4: register budget of the stencil kernels for that
 *                many resident waves per SIMD (1 = unlimited; more waves
 *                hide more latency, fewer registers may spill)
 *   "collapse"   >= 1 (default 1024): a pass with more workgroups per job
 *                than this sums its per-workgroup partial sums once, in a
 *                launch of its own, instead of in every workgroup of the
 *                next pass (which otherwise re-reads all of them)
 *   "concurrent_groups" 1: the lattice groups of a batched call run on
 *                separate streams forked from (and joined back to) the call's
 *                stream; 0: one after another on the call's stream
 *   "pipeline_groups" 1 (with concurrent groups, calls without stats): each
 *                group's nested step and lift follow its own outer loop on
 *                its stream; 0 (default): one nested launch for all jobs
 *                after the join (measured 1 % faster at 10^4: the lift of one
 *                group competes with the other group's stencil for HBM)
 *   "stagger_groups" 0..100 (with pipelined groups): the group with the
 *                costliest nested step (two-sided first, then the largest k)
 *                starts first and the others wait until it has done this
 *                percentage of its outer loop, so that their outer passes
 *                fill the CUs its nested step leaves idle; 0: all start
 *                together
 *   "graph"      1: capture and replay batched calls as HIP graphs (see
 *                nks_sign_apply_batch); 0: launch eagerly.
 * Read-only counters: "graph_captures", "graph_replays".
 * Results are identical bit for bit under every choice.  Unknown keys give
 * NKS_E_INVALID. */
int nks_tune_set(nks_ctx* ctx, const char* key, int value);
int nks_tune_get(nks_ctx* ctx, const char* key, int* value);

/* Measurement support.  When enabled on a context, sign applications time
 * every 8th launch of each kernel class (every nested and lift launch) with
 * start/stop events that the launch's own dispatch stamps
 * (hipExtLaunchKernelGGL), so a duration is the kernel's execution without
 * the gaps between launches; profiled calls run eagerly (no graph replay).
 * nks_profile_read waits
 * for those events, returns the number of timed launches, their summed
 * device time and their summed algorithmic bytes (what each launch must move
 * at minimum: inputs read once, outputs written once), and resets the class. */
enum nks_kernel_class {
    NKS_K_STENCIL = 0,   /* stencil pass of an outer iteration (A v, two-sided also A^dagger w) */
    NKS_K_RECUR = 1,     /* recurrence pass of an outer iteration */
    NKS_K_NESTED = 2,    /* nested step (steps 3-5), one launch per batch */
    NKS_K_LIFT = 3,      /* lift y = |b| V_k c, one launch per lattice group */
    NKS_K_COUNT = 4
};
int nks_profile_enable(nks_ctx* ctx, int enable);
int nks_profile_read(nks_ctx* ctx, int kernel_class, int* launches, double* total_ms, double* alg_bytes);

#ifdef __cplusplus
}
#endif
#endif /* NKS_H */
