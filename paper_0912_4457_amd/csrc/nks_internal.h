// Internal definitions of libnks: device data layout, job descriptors,
// complex helpers and block reductions shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include <string>

#include "../../include/nks.h"

namespace nks {

// ----------------------------------------------------------------- complex
template <typename R> struct cx;
template <> struct cx<double> { using T = double2; };
template <> struct cx<float> { using T = float2; };
template <typename R> using cx_t = typename cx<R>::T;

__host__ __device__ inline double2 mk(double a, double b) { return make_double2(a, b); }
__host__ __device__ inline float2 mkf(float a, float b) { return make_float2(a, b); }

template <typename V> __host__ __device__ inline V cadd(V a, V b) { V r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename V> __host__ __device__ inline V csub(V a, V b) { V r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename V> __host__ __device__ inline V cmul(V a, V b) {
    V r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
// conj(a) * b
template <typename V> __host__ __device__ inline V cmulc(V a, V b) {
    V r; r.x = a.x * b.x + a.y * b.y; r.y = a.x * b.y - a.y * b.x; return r;
}
template <typename V> __host__ __device__ inline V cconj(V a) { V r; r.x = a.x; r.y = -a.y; return r; }
template <typename V, typename S> __host__ __device__ inline V cscale(V a, S s) { V r; r.x = a.x * s; r.y = a.y * s; return r; }
// i * a and -i * a
template <typename V> __host__ __device__ inline V cmuli(V a) { V r; r.x = -a.y; r.y = a.x; return r; }
template <typename V> __host__ __device__ inline V cmulmi(V a) { V r; r.x = a.y; r.y = -a.x; return r; }
template <typename V> __host__ __device__ inline V cneg(V a) { V r; r.x = -a.x; r.y = -a.y; return r; }
__host__ __device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline double cabs(double2 a) { return sqrt(a.x * a.x + a.y * a.y); }
__host__ __device__ inline double2 cdiv(double2 a, double2 b) {
    // a / b, scaled to avoid overflow in |b|^2
    double s = fabs(b.x) > fabs(b.y) ? fabs(b.x) : fabs(b.y);
    if (s == 0.0) return mk(a.x / 0.0, a.y / 0.0);
    double bx = b.x / s, by = b.y / s;
    double d = bx * bx + by * by;
    double ax = a.x / s, ay = a.y / s;
    return mk((ax * bx + ay * by) / d, (ay * bx - ax * by) / d);
}
__host__ __device__ inline double2 crecip(double2 b) { return cdiv(mk(1.0, 0.0), b); }
// principal square root (branch cut on the negative real axis)
__host__ __device__ inline double2 csqrt_principal(double2 z) {
    double r = sqrt(z.x * z.x + z.y * z.y);
    if (r == 0.0) return mk(0.0, 0.0);
    double a = sqrt(0.5 * (r + fabs(z.x)));
    double b = 0.5 * z.y / a;
    if (z.x >= 0.0) return mk(a, b);
    // z.x < 0: sqrt = (|b|, sign(y) a)
    double im = (z.y >= 0.0) ? a : -a;
    return mk(fabs(b), im);
}

template <typename R> __device__ inline double2 to_d2(cx_t<R> a) { return mk((double)a.x, (double)a.y); }
template <typename R> __device__ inline cx_t<R> from_d2(double2 a);
template <> __device__ inline double2 from_d2<double>(double2 a) { return a; }
template <> __device__ inline float2 from_d2<float>(double2 a) { return mkf((float)a.x, (float)a.y); }

// ----------------------------------------------------------------- geometry
struct Geom {
    int lx, ly, lz, lt;
    int V;
};

// ----------------------------------------------------------------- jobs
// Scalar slots of one job (each an array of double2 of length kcap + 2).
enum ScalarSlot {
    SC_ALPHA = 0,   // H(j,j), j = 1..k
    SC_BETA = 1,    // H(j+1,j), j = 1..k-1
    SC_GAMMA = 2,   // H(j,j+1), j = 1..k-1
    SC_SV = 3,      // v_j = sv_j u_j (u_j: stored unnormalised vector)
    SC_SW = 4,      // w_j = sw_j t_j
    SC_VN = 5,      // ||v_j||
    SC_WN = 6,      // ||w_j||
    SC_COUNT = 7
};

// status words of one job
enum StatusWord {
    ST_DONE = 0,        // outer loop ended early (breakdown or zero source)
    ST_KUSED = 1,       // outer basis size built
    ST_STATUS = 2,      // NKS_OK / NKS_E_BREAKDOWN / NKS_E_NOCONV
    ST_BDITER = 3,      // serious breakdown iteration
    ST_ELL = 4,         // inner size used (0 = non-nested)
    ST_RHI = 5,         // RHi iterations
    ST_CKPT_DONE = 6,   // a k-checkpoint accepted the result (omega already written)
    ST_NCKPT = 7,       // k-checkpoints stored so far
    ST_KCKPT = 8,       // size of the stored checkpoint coefficients
    ST_KTARGET = 9,     // learned policy: predicted outer size (0 = none)
    ST_ELLSTART = 10,   // learned policy: first inner size of the doubling (0 = default)
    ST_FALLBACK = 11,   // learned policy: prediction rejected, plain checkpoints took over
    ST_LEVELS = 12,     // nested levels that ran (multi-level nesting)
    ST_ELL_DEEP = 13,   // .. 13 + NKS_MAX_LEVELS - 2: sizes built at the deeper levels
    ST_COUNT = 24
};

// doubles reported by the nested step
enum ReportWord {
    RP_BNORM = 0,
    RP_P = 1,
    RP_ZMIN = 2,
    RP_ZMAX = 3,
    RP_INNER_DELTA = 4,
    RP_OUTER_DELTA = 5,
    RP_P_DEEP = 8,      // .. 8 + NKS_MAX_LEVELS - 2: p of the deeper levels
    RP_COUNT = 16
};

// Partial-sum slots (each an array of double2 of length pstride: one entry per
// block of the pass that writes it, and a last entry for their total when it
// is collapsed).
enum PartialSlot { PS_S = 0, PS_R0 = 1, PS_R1 = 2, PS_R2 = 3, PS_COUNT = 4 };

// One sign application, as seen by the device.  Lives in the workspace.
struct JobDesc {
    const double2* b;   // caller input, AoS complex128 (12*site + comp)
    double2* x;         // caller output, AoS complex128
    void* vstore;       // outer basis, (kcap + 1) columns of 12V storage-type complex, SoA
    void* lring;        // two-sided left vectors, 2 columns of 12V
    double2* part;      // PS_COUNT * pstride partial sums
    double2* sc;        // SC_COUNT * (kcap + 2) scalars
    int* status;        // ST_COUNT ints
    double* report;     // RP_COUNT doubles
    double2* omega;     // lift weights, kcap
    double2* nest;      // nested-step scratch
    int k;              // requested outer size (even)
    int ell;            // requested inner size (even)
    double p;           // <= 0: estimate
    int max_rhi;
    double rhi_tol;
    int two_sided;
    int nest_cap;       // complex words available in nest
    int lcap;           // inner size capacity of the nest area
    int scstride;       // length of each scalar slot (kcap + 2)
    int nblocks;        // blocks per job of the outer site-parallel kernels
    int pstride;        // length of each partial-sum slot: nblocks + 1
    int collapse;       // a pass with more blocks than this leaves its partials' total in the slot's last entry
    int precision;      // NKS_FP64 / NKS_MIXED
    int k_policy;       // NKS_POLICY_*
    int ell_policy;
    double tol;         // target relative accuracy of the policies
    double2* ckpt;      // coefficients of the last k-checkpoint (kcap)
    double mu;          // chemical potential of the job's lattice
    double zcap;        // bound of |lambda| over A's spectrum (norm_bound); z_max of Eq. popt is
                        // capped there (a larger |theta| of H_k is spurious); <= 0: no cap
    int V;              // lattice volume
    const struct PolicyNet* net;   // learned policy (device), or null
    double* label;      // label mode output (LABEL_WORDS doubles), or null
    int* group;         // GROUP_WORDS ints shared by the jobs of one lattice group (zeroed by pack)
    int overlap;        // 1: the lift writes x = b + gamma5 y (overlap operator) instead of y
    // deflation (App. C steps 1 and 6): dm eigenpairs of A held by the lattice
    int dm;                 // 0 = no deflation
    const double2* dr;      // right eigenvectors, SoA [i][comp][site] (complex128)
    const double2* dl;      // left eigenvectors (= dr when A is Hermitian)
    const double* dsgn;     // sgn(Re lambda_i)
    double2* dcoef;         // <l_i, b> (written by pack_kernel, block 0)
    double2* dpart;         // per-block partial sums of <l_i, b>, [i][block]
    // multi-level nesting (Sec. 4.5): levels >= 1; level i + 1 < levels builds
    // ell_deep[i] vectors (even) with p_deep[i] (<= 0: estimate)
    int levels;
    int ell_deep[NKS_MAX_LEVELS - 1];
    double p_deep[NKS_MAX_LEVELS - 1];
    // double-pass mode (Sec. 4.4): the store holds two columns (u_j in column
    // (j - 1) & 1); the second pass regenerates the basis and sums
    // omega_j u_j into yacc, two SoA complex128 vectors (odd / even j)
    int ring;
    double2* yacc;
};
static_assert(ST_ELL_DEEP + NKS_MAX_LEVELS - 1 <= ST_COUNT && RP_P_DEEP + NKS_MAX_LEVELS - 1 <= RP_COUNT,
              "status / report words of the deeper levels");

constexpr int DEFL_MAX = 64;   // deflated eigenpairs per lattice

// Words shared by a lattice group: the largest learned k target of its jobs.
enum GroupWord { GW_KTARGET_MAX = 0, GROUP_WORDS = 16 };

constexpr int RHI_MAX = 1024;    // largest dense Roberts-Higham matrix (inner ell, or k when non-nested)
constexpr int CKPT_DK = 100;     // outer iterations between plain k-checkpoints
constexpr int LEARN_K0 = 100;    // probe length of the learned policy (features of H_{k0})
constexpr int LEARN_DK = 20;     // granularity of the learned k and of its verification
constexpr int LEARN_VERIFY_DK = 40;   // k* is verified against k* - 40

// Learned policy: network parameters and normalisation, resident on the device.
constexpr int NFEAT = 16;
struct PolicyNet {
    float params[5378];
    float fmean[NFEAT], fstd[NFEAT];   // feature normalisation
    float tmean[2], tstd[2];           // targets: log10 k*, log10 ell*
};

// Label mode output per job (doubles): features of H_{k0}, the weighted error of
// the nested result at k = LABEL_DK * (i + 1) against the job's final result,
// and the ell-doubling changes (16 -> 32, 32 -> 64, 64 -> 128, 128 -> 256) at each k.
// A label job owns 1 + LABEL_NK nested scratch areas of nest_cap words each.
constexpr int LABEL_NK = 60, LABEL_NELL = 4, LABEL_DK = 20;
constexpr double LABEL_TOL = 1e-13;   // ell doubling of the label runs stops at a change <= LABEL_TOL / 10
constexpr int LABEL_WORDS = NFEAT + LABEL_NK + LABEL_NK * LABEL_NELL;
static_assert(LABEL_WORDS == NKS_LABEL_WORDS && NFEAT == NKS_POLICY_NFEAT && LEARN_K0 == NKS_LEARN_K0 &&
                  LABEL_NK == NKS_LABEL_NK && LABEL_NELL == NKS_LABEL_NELL && LABEL_DK == NKS_LABEL_DK,
              "label layout must match the public header");
static_assert(sizeof(PolicyNet) == sizeof(float) * NKS_POLICY_NFLOATS, "PolicyNet layout");

// ----------------------------------------------------------------- reductions
__device__ inline double2 shfl_xor_d2(double2 v, int m) {
    v.x = __shfl_xor(v.x, m, 64);
    v.y = __shfl_xor(v.y, m, 64);
    return v;
}

// Sum over the block; result valid in every thread.  lds: >= NT/64 entries.
template <int NT>
__device__ inline double2 block_sum(double2 v, double2* lds) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = cadd(v, shfl_xor_d2(v, m));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double2 s = lds[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) s = cadd(s, lds[w]);
    return s;
}

// Sum of n partial sums by the 64 lanes of one wavefront: lane l adds entries
// l, l + 64, ..., then a butterfly over the lanes (every lane ends with the
// same bits, addition being commutative).  The one summation order of every
// reader of the outer passes' partial sums, so that a total summed ahead in a
// launch of its own has the same bits.  All 64 lanes must call it.
__device__ inline double2 wave_sum(const double2* part, int n) {
    const int lane = threadIdx.x & 63;
    double2 s = mk(0.0, 0.0);
    int i = lane;
    for (; i + 7 * 64 < n; i += 8 * 64) {   // eight loads in flight, added in index order
        double2 v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = part[i + q * 64];
#pragma unroll
        for (int q = 0; q < 8; ++q) s = cadd(s, v[q]);
    }
    for (; i < n; i += 64) s = cadd(s, part[i]);
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) s = cadd(s, shfl_xor_d2(s, m));
    return s;
}

// Deterministic sum of n partials (same order in every block).  NTS threads
// take part, each summing every NTS-th partial; in a block of NTB >= NTS
// threads the others contribute exact zeros, so the result has the bits of
// the NTS-thread sum whatever the block size.
template <int NTS, int NTB = NTS>
__device__ inline double2 sum_partials(const double2* part, int n, double2* lds) {
    double2 s = mk(0.0, 0.0);
    if (threadIdx.x < NTS)
        for (int i = threadIdx.x; i < n; i += NTS) s = cadd(s, part[i]);
    return block_sum<NTB>(s, lds);
}

// ----------------------------------------------------------------- launchers
// wilson.hip
template <typename R>
void launch_apply(const Geom& g, const cx_t<R>* links, double kappa, double mu, const double2* in,
                  double2* out, cx_t<R>* tmp_in, cx_t<R>* tmp_out, hipStream_t s);

// Launch-shape choices of the outer passes (picked per context; see api.hip).
struct Tuning {
    int xcd_map = 1;      // 1D grid: 1 = all jobs of a site block on one XCD, 2 = whole jobs per XCD
    int split_dual = 1;   // two-sided stencil: A u and A^dagger t in separate blocks
    int min_waves = 1;    // stencil kernels: register budget for 1 (unlimited), 3 or 4 waves per SIMD
    int collapse = 1024;  // passes with more blocks per job than this sum their partials once in a
                          // separate launch instead of in every block of the next pass
    int concurrent = 1;   // lattice groups of a batch on separate streams (1) or one after another (0)
    int pipeline = 0;     // with concurrent groups: each group's nested step and lift follow its own outer loop
    int stagger = 0;      // pipelined groups: the others start once the lead group has done this % of its loop
};

// Start/stop events of a timed launch (nks_profile_enable), stamped by the
// kernel's own dispatch packet (hipExtLaunchKernelGGL), so that they bracket
// its execution and not the gaps between launches.  Null: an ordinary launch.
struct LaunchEvents {
    hipEvent_t a = nullptr, b = nullptr;
};

// outer.hip
struct OuterLaunch {
    Geom g;
    const void* links;    // storage-type links, SoA [nu][row][col][V]
    double kappa, mu;
    JobDesc* jobs;        // device array
    int njobs;
    int kmax;             // max over jobs of k
    int nblocks;          // blocks per job of the site-parallel kernels
    int precision;        // NKS_FP64 / NKS_MIXED
    int two_sided;
    Tuning tune;
    int deflate;           // some job of the group is deflated
    int ring;              // some job of the group runs in double-pass mode
    int pass2;             // 1: the second (regenerating) pass of those jobs
    LaunchEvents ev;       // timing of the next S, R or lift launch
};
// Workgroup size of the site-parallel outer passes: 512 threads (8 wavefronts,
// one workgroup per CU at the stencil's 2 waves per SIMD) cover five x-y
// planes of a 10^4 lattice, so a site's z-neighbours mostly come from the
// CU's own L1 (stencil 49.0 us against 51.0 us with 128 threads).
constexpr int OUTER_NT = 512;

// ||A|| = ||D_w(mu)|| <= 1 + kappa (6 sqrt(2) + 2 sqrt(2 cosh 2 mu)) (Sec. 2 operator):
// per direction the two hops land in the complementary ranges of (1 -+ gamma_nu)/2,
// so their sum has norm <= 2 kappa sqrt(c+^2 + c-^2) with hop factors c+- = 1, or
// e^{+-mu} in time.  Every eigenvalue of A lies in |lambda| <= this bound.
inline double norm_bound(double kappa, double mu) {
    return 1.0 + kappa * (6.0 * std::sqrt(2.0) + 2.0 * std::sqrt(2.0 * std::cosh(2.0 * mu)));
}

// Launch map of the outer passes (tuning key xcd_map).  The hardware hands
// workgroup b of a 1D grid to XCD b % 8, so b -> (site block, job) decides
// which part of the (site block, job) rectangle each XCD's L2 serves:
//   1: a contiguous eighth of the site blocks, all jobs (jobs innermost);
//   2: a contiguous eighth of the (job, site block) pairs, job-major;
//   3: the XCDs split into JP parts of the jobs times 8 / JP contiguous
//      parts of the site blocks (in t), JP = 4 for at least 8 jobs or a
//      multiple of 4, 2 for 2..7 jobs, 1 for one job: at 12 jobs each XCD
//      fetches a t-halo of two slices per half lattice instead of per eighth.
// xcd_slots is the number of workgroups per XCD (grid = 8 * slots);
// map_block returns false for padding workgroups.
__host__ __device__ inline int xcd_job_parts(int njobs) {
    return (njobs >= 8 || njobs % 4 == 0) ? 4 : (njobs >= 2 ? 2 : 1);
}
__host__ __device__ inline int xcd_slots(int nblocks, int njobs, int xcd_map) {
    if (xcd_map == 3) {
        const int jp = xcd_job_parts(njobs), tp = 8 / jp;
        return ((nblocks + tp - 1) / tp) * ((njobs + jp - 1) / jp);
    }
    return (nblocks * njobs + 7) / 8;
}
__host__ __device__ inline bool map_block(int b, int nblocks, int njobs, int xcd_map, int& sb, int& job) {
    const int x = b & 7, i = b >> 3;
    if (xcd_map == 3) {
        const int JP = xcd_job_parts(njobs), TP = 8 / JP;
        const int tp = x % TP, jp = x / TP;
        const int sb_lo = tp * nblocks / TP, sb_hi = (tp + 1) * nblocks / TP;
        const int j_lo = jp * njobs / JP, j_hi = (jp + 1) * njobs / JP;
        const int m = j_hi - j_lo;
        if (m <= 0 || i >= (sb_hi - sb_lo) * m) return false;
        sb = sb_lo + i / m;
        job = j_lo + i % m;
        return true;
    }
    const int total = nblocks * njobs;
    const int q = x * xcd_slots(nblocks, njobs, xcd_map) + i;
    if (q >= total) return false;
    if (xcd_map == 2) {
        job = q / nblocks;
        sb = q - job * nblocks;
    } else {
        sb = q / njobs;
        job = q - sb * njobs;
    }
    return true;
}
void launch_pack(const OuterLaunch& L, hipStream_t s);
void launch_outer_S(const OuterLaunch& L, int j, hipStream_t s);   // stencil pass of iteration j
void launch_outer_R(const OuterLaunch& L, int j, hipStream_t s);   // recurrence pass (j < k only)
void launch_collapse(const OuterLaunch& L, int slot0, int nslots, int nb, hipStream_t s);
void launch_lift(const OuterLaunch& L, hipStream_t s);

// nested.hip
constexpr int NEST_NT = 256;
void launch_finalize(JobDesc* jobs, int njobs, hipStream_t s);
void launch_nested(JobDesc* jobs, int njobs, hipStream_t s, LaunchEvents ev = {});
void launch_checkpoint(JobDesc* jobs, int njobs, int j, hipStream_t s);   // after R_j
void launch_predict(JobDesc* jobs, int njobs, int j, hipStream_t s);      // after R_{k0}
void launch_label(JobDesc* jobs, int njobs, hipStream_t s);               // after the outer loop
size_t nest_words(int k, int ell, int levels, const int* ell_deep);

// eig.hip: m eigenpairs of A(mu) with the smallest |lambda| by a block of
// p >= m vectors: unit right eigenvectors to rvecs_out, left eigenvectors with
// l_i^H r_i = 1 to lvecs_out (both SoA [i][comp][site]; equal for mu = 0),
// eigenvalues as (re, im) pairs to lambda_out.
int eig_chfsi(const Geom& g, const double2* links, double kappa, double mu, int m, int p, int degree, int max_iter,
              double tol, unsigned long long seed, double2* rvecs_out, double2* lvecs_out, double* lambda_out,
              double* resid_out, int* iters_out, std::string& err);

// mlp.hip
int mlp_nparams();
void launch_mlp_forward(const float* P, const float* X, int B, float* Y, hipStream_t s);
void launch_mlp_backward(const float* P, const float* X, const float* T, int B, float* G, float* loss,
                         hipStream_t s);
void launch_mlp_adam(float* P, const float* G, float* M, float* V, int t, float lr, hipStream_t s);

}  // namespace nks
