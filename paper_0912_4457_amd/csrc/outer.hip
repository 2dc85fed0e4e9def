// Outer Krylov basis: Lanczos (App. A, mu = 0) and two-sided Lanczos
// (App. B, mu != 0) with the Wilson stencil fused into the recurrences, and
// the lift y = |b| V_k c of Eq. nested.
//
// The basis is stored unnormalised: column j of the store holds u_j with
// v_j = sv_j u_j (sv_1 = 1/|b|, sv_{j+1} = 1/beta_j), so no pass is spent on
// rescaling.  Per outer iteration j two site-parallel kernels run:
//
//   S_j (stencil):  r = sv_j A u_j - H(j-1,j) v_{j-1}           -> column j+1
//                   [two-sided also l = sw_j A^dag t_j - conj(H(j,j-1)) w_{j-1}]
//                   partial sums of conj(t_j) . r  (alpha_j / sv_j or / conj(sw_j))
//   R_j (recurrence): alpha_j; r -= alpha_j v_j [l -= conj(alpha_j) w_j];
//                   partial sums of |r|^2 [and r^dag l, |l|^2]
//
// Every block of S_{j+1} sums R_j's partials in the same order (one wavefront,
// wave_sum), so all blocks agree on beta_j (and on a breakdown) without a
// grid barrier; block 0 stores the scalars for the nested step.  A pass with
// more blocks per job than the tuning key `collapse` is followed by a
// one-wavefront-per-job launch that sums its partials once, in the same
// order, so that the next pass does not re-read all of them in every block.
// All scalars stay on the device.
//
// Double-pass mode (Sec. 4.4): the store keeps only u_j and u_{j+1} (two
// columns; r overwrites u_{j-1} at its own site, after reading it).  After
// the nested step the same kernels run again from b (pass2 = 1): every sum
// is taken in a fixed order, so they regenerate u_1 .. u_k bit for bit, and
// S_j adds omega_j u_j to one of two accumulators (odd / even j, the
// summation order of the lift).
#include "wilson.h"

#include <hip/hip_ext.h>

namespace nks {

namespace {

constexpr int NT = OUTER_NT;
constexpr double LUCKY_TAU_HERMITIAN = 1e-10;
constexpr double LUCKY_TAU_TWO_SIDED = 1e-8;
constexpr double SERIOUS_TAU = 1e-12;

__device__ inline double2* slot(const JobDesc& J, int s) { return J.sc + (size_t)s * J.scstride; }

template <typename R>
__device__ inline cx_t<R>* column(const JobDesc& J, int j, int n) {   // j is 1-based
    return reinterpret_cast<cx_t<R>*>(J.vstore) + (size_t)(J.ring ? ((j - 1) & 1) : (j - 1)) * n;
}

// Second pass: a job takes part only in double-pass mode, up to its final k.
__device__ inline bool skip_S(const JobDesc& J, int j, int pass2) {
    return pass2 ? (!J.ring || j > J.status[ST_KUSED]) : (j > J.k || J.status[ST_DONE]);
}
__device__ inline bool skip_R(const JobDesc& J, int j, int pass2) {
    return pass2 ? (!J.ring || j >= J.status[ST_KUSED]) : (j >= J.k || J.status[ST_DONE]);
}

// Second pass, S_j: accumulator (j - 1) & 1 += omega_j u_j at element e.
__device__ inline void accumulate(const JobDesc& J, int j, size_t e, int n, double2 u) {
    double2* y = J.yacc + (size_t)((j - 1) & 1) * n + e;
    const double2 prev = (j <= 2) ? mk(0.0, 0.0) : *y;
    *y = cadd(prev, cmul(J.omega[j - 1], u));
}

template <typename R>
__device__ inline cx_t<R>* lvec(const JobDesc& J, int j, int n) {     // t_j in ring slot j % 2
    return reinterpret_cast<cx_t<R>*>(J.lring) + (size_t)(j & 1) * n;
}

// Block -> (site block, job): the 2D grid (xcd_map 0) or the XCD-aware 1D
// maps of map_block.  Returns false for padding blocks.
__device__ inline bool block_coords(int nblocks, int njobs, int xcd_map, int& sb, int& job) {
    if (!xcd_map) { sb = blockIdx.x; job = blockIdx.y; return true; }
    return map_block(blockIdx.x, nblocks, njobs, xcd_map, sb, job);
}

__device__ inline double2* pslot(const JobDesc& J, int s) { return J.part + (size_t)s * J.pstride; }

// The partials of slot s that the next pass re-reduces, written by a pass with
// nb blocks per job: all of them, or the one total that a collapse launch left
// in the slot's last entry (count receives the number).
__device__ inline const double2* partials(const JobDesc& J, int s, int nb, int& count) {
    if (nb > J.collapse) { count = 1; return pslot(J, s) + J.pstride - 1; }
    count = nb;
    return pslot(J, s);
}

// Sum the nb partials of each slot in [slot0, slot0 + nslots) into the slot's
// last entry (wave_sum order), one wavefront per job.  The partials stay as
// they are, so running it again (a job that skipped the pass) gives the same
// total.
__global__ __launch_bounds__(64) void collapse_kernel(JobDesc* jobs, int slot0, int nslots, int nb) {
    const JobDesc& J = jobs[blockIdx.x];
    for (int s = slot0; s < slot0 + nslots; ++s) {
        const double2 t = wave_sum(pslot(J, s), nb);
        if (threadIdx.x == 0) pslot(J, s)[J.pstride - 1] = t;
    }
}

// Per-wavefront butterfly sums of v, combined over the block's nw wavefronts in
// wavefront order; the total is valid in thread 0 only.  lds: nw entries, not
// used for anything else in the kernel.
template <int NW>
__device__ inline double2 block_total(double2 v, double2* lds) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = cadd(v, shfl_xor_d2(v, m));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double2 t = lds[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) t = cadd(t, lds[w]);
    return t;
}

// ------------------------------------------------------------------ deflation dots
// Per-block partial sums of <l_i, b> = sum conj(l_i) b for every deflated job.
__global__ __launch_bounds__(NT) void deflate_dots_kernel(JobDesc* jobs, int V, int nblocks) {
    const JobDesc& J = jobs[blockIdx.y];
    if (J.dm == 0) return;
    __shared__ double2 lds[NT / 64];
    const int site = blockIdx.x * NT + threadIdx.x;
    const int n = 12 * V;
    for (int i = 0; i < J.dm; ++i) {
        double2 acc = mk(0.0, 0.0);
        if (site < V) {
            const double2* l = J.dl + (size_t)i * n;
#pragma unroll
            for (int c = 0; c < 12; ++c) acc = cadd(acc, cmul(cconj(l[(size_t)c * V + site]), J.b[(size_t)12 * site + c]));
        }
        const double2 s = block_sum<NT>(acc, lds);
        if (threadIdx.x == 0) J.dpart[(size_t)i * nblocks + blockIdx.x] = s;
    }
}

// ------------------------------------------------------------------ pack
template <typename R>
__global__ __launch_bounds__(NT) void pack_kernel(JobDesc* jobs, int V, int nblocks, int pass2) {
    const JobDesc& J = jobs[blockIdx.y];
    if (pass2 && !J.ring) return;
    __shared__ double2 lds[NT / 64];
    const int site = blockIdx.x * NT + threadIdx.x;
    const int n = 12 * V;
    if (!pass2 && blockIdx.x == 0 && threadIdx.x < ST_COUNT) {
        int v = 0;
        if (threadIdx.x == ST_KUSED) v = J.k;
        J.status[threadIdx.x] = v;
    }
    if (!pass2 && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < GROUP_WORDS && J.group) J.group[threadIdx.x] = 0;
    // deflation (App. C step 1): b_m = b - sum_i <l_i, b> r_i, with the
    // <l_i, b> re-reduced from deflate_dots' per-block partials by every block
    __shared__ double2 dco[DEFL_MAX];
    if (J.dm > 0) {
        for (int i = 0; i < J.dm; ++i) {
            const double2 d = sum_partials<NT>(J.dpart + (size_t)i * nblocks, nblocks, lds);
            if (threadIdx.x == 0) {
                dco[i] = d;
                if (blockIdx.x == 0) J.dcoef[i] = d;
            }
        }
        __syncthreads();
    }
    double nb2 = 0.0;
    if (site < V) {
        cx_t<R>* u1 = column<R>(J, 1, n);
        cx_t<R>* t1 = J.two_sided ? lvec<R>(J, 1, n) : nullptr;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            double2 bc = J.b[(size_t)12 * site + c];
            for (int i = 0; i < J.dm; ++i) bc = csub(bc, cmul(dco[i], J.dr[(size_t)i * n + (size_t)c * V + site]));
            cx_t<R> v = from_d2<R>(bc);
            u1[(size_t)c * V + site] = v;
            if (t1) t1[(size_t)c * V + site] = v;
            double2 d = to_d2<R>(v);
            nb2 += cabs2(d);
        }
    }
    double2 s = block_sum<NT>(mk(nb2, 0.0), lds);
    if (threadIdx.x == 0) pslot(J, PS_R0)[blockIdx.x] = s;
}

// ------------------------------------------------------------------ scalars of S_j
// Scalars of S_j from R_{j-1}'s partial sums (|b|^2 from pack's when j == 1),
// computed by the 64 lanes of one wavefront; lane 0 of the job's first tile
// (store) writes them to the job's slots.  Hermitian: beta_{j-1}, v_j = svj u_j
// and beta_{j-1} v_{j-1} = cprev u_{j-1}.  Returns false when the job stops
// here (zero source, invariant subspace).
__device__ inline bool herm_scalars(const JobDesc& J, int j, bool store, double& svj, double& cprev) {
    int cnt;
    const double2* pr = partials(J, PS_R0, J.nblocks, cnt);
    const double beta = sqrt(wave_sum(pr, cnt).x);
    if (j == 1) {
        if (beta == 0.0) {                                  // zero source: x = 0
            if (store) { J.status[ST_DONE] = 1; J.status[ST_KUSED] = 0; J.report[RP_BNORM] = 0.0; }
            return false;
        }
        svj = 1.0 / beta;
        cprev = 0.0;
        if (store) { J.report[RP_BNORM] = beta; slot(J, SC_SV)[1] = mk(svj, 0.0); slot(J, SC_VN)[1] = mk(1.0, 0.0); }
        return true;
    }
    const double aprev = slot(J, SC_ALPHA)[j - 1].x;
    const double bprev = (j >= 3) ? slot(J, SC_BETA)[j - 2].x : 0.0;
    if (beta <= LUCKY_TAU_HERMITIAN * (fabs(aprev) + bprev)) {   // invariant subspace
        if (store) { J.status[ST_DONE] = 1; J.status[ST_KUSED] = j - 1; }
        return false;
    }
    svj = 1.0 / beta;
    cprev = beta * slot(J, SC_SV)[j - 1].x;                       // beta_{j-1} v_{j-1} = cprev u_{j-1}
    if (store) {
        slot(J, SC_BETA)[j - 1] = mk(beta, 0.0);
        slot(J, SC_GAMMA)[j - 1] = mk(beta, 0.0);
        slot(J, SC_SV)[j] = mk(svj, 0.0);
        slot(J, SC_VN)[j] = mk(1.0, 0.0);
    }
    return true;
}

// Two-sided (App. B): v_j = sv u_j, w_j = sw t_j, gamma_{j-1} v_{j-1} = cv u_{j-1},
// conj(beta_{j-1}) w_{j-1} = cw t_{j-1}.  Returns false when the job stops
// here (zero source, lucky or serious breakdown).  One wavefront, as above.
__device__ inline bool bi_scalars(const JobDesc& J, int j, bool store, double2& sv, double2& sw, double2& cv,
                                  double2& cw) {
    int cnt;
    if (j == 1) {
        const double2* pr = partials(J, PS_R0, J.nblocks, cnt);
        const double bn = sqrt(wave_sum(pr, cnt).x);
        if (bn == 0.0) {
            if (store) { J.status[ST_DONE] = 1; J.status[ST_KUSED] = 0; J.report[RP_BNORM] = 0.0; }
            return false;
        }
        sv = sw = mk(1.0 / bn, 0.0);
        cv = cw = mk(0.0, 0.0);
        if (store) {
            J.report[RP_BNORM] = bn;
            slot(J, SC_SV)[1] = sv; slot(J, SC_SW)[1] = sw;
            slot(J, SC_VN)[1] = mk(1.0, 0.0); slot(J, SC_WN)[1] = mk(1.0, 0.0);
        }
        return true;
    }
    const double2* p0 = partials(J, PS_R0, J.nblocks, cnt);
    const double2* p1 = partials(J, PS_R1, J.nblocks, cnt);
    const double2* p2 = partials(J, PS_R2, J.nblocks, cnt);
    const double2 delta = wave_sum(p0, cnt);
    const double nr = sqrt(wave_sum(p1, cnt).x);
    const double nl = sqrt(wave_sum(p2, cnt).x);
    const double aprev = cabs(slot(J, SC_ALPHA)[j - 1]);
    const double sprev = (j >= 3) ? sqrt(cabs(cmul(slot(J, SC_BETA)[j - 2], slot(J, SC_GAMMA)[j - 2]))) : 0.0;
    const double S = aprev + sprev;
    if (nr <= LUCKY_TAU_TWO_SIDED * S * slot(J, SC_VN)[j - 1].x ||
        nl <= LUCKY_TAU_TWO_SIDED * S * slot(J, SC_WN)[j - 1].x) {
        if (store) { J.status[ST_DONE] = 1; J.status[ST_KUSED] = j - 1; }
        return false;
    }
    if (cabs(delta) <= SERIOUS_TAU * nr * nl) {
        if (store) {
            J.status[ST_DONE] = 1; J.status[ST_KUSED] = j - 1;
            J.status[ST_STATUS] = NKS_E_BREAKDOWN; J.status[ST_BDITER] = j - 1;
        }
        return false;
    }
    const double2 beta = csqrt_principal(delta);
    const double2 gamma = cdiv(cconj(delta), beta);
    sv = crecip(beta);
    sw = crecip(cconj(gamma));
    cv = cmul(gamma, slot(J, SC_SV)[j - 1]);              // gamma_{j-1} v_{j-1}
    cw = cmul(cconj(beta), slot(J, SC_SW)[j - 1]);        // conj(beta_{j-1}) w_{j-1}
    if (store) {
        slot(J, SC_BETA)[j - 1] = beta; slot(J, SC_GAMMA)[j - 1] = gamma;
        slot(J, SC_SV)[j] = sv; slot(J, SC_SW)[j] = sw;
        slot(J, SC_VN)[j] = mk(nr / cabs(beta), 0.0);
        slot(J, SC_WN)[j] = mk(nl / cabs(gamma), 0.0);
    }
    return true;
}

// ------------------------------------------------------------------ Hermitian step
// MINW: waves per SIMD the register allocation must allow (1 = no limit);
// more resident waves hide more memory latency, at the price of spills.
template <typename R, int MINW>
__global__ __launch_bounds__(NT, MINW) void herm_S(JobDesc* jobs, Geom g, const cx_t<R>* __restrict__ links,
                                                  double kappa, int j, int nblocks, int njobs, int xcd_map,
                                                  int pass2) {
    int sb, job;
    if (!block_coords(nblocks, njobs, xcd_map, sb, job)) return;
    const JobDesc& J = jobs[job];
    if (skip_S(J, j, pass2)) return;
    __shared__ double2 lds[NT / 64];
    __shared__ double2 scal[2];
    __shared__ int go;
    const int n = 12 * g.V;
    // the scalars by wavefront 0 alone; the other wavefront starts its stencil at once
    if (threadIdx.x < 64) {
        double a = 0.0, c = 0.0;
        const bool more = herm_scalars(J, j, sb == 0 && threadIdx.x == 0, a, c);
        if (threadIdx.x == 0) { scal[0] = mk(a, 0.0); scal[1] = mk(c, 0.0); go = more ? 1 : 0; }
    }
    const int site = sb * NT + threadIdx.x;
    cx_t<R> acc[1][12];
    if (site < g.V) {
        const cx_t<R>* uj = column<R>(J, j, n);
        R cf[1][4], cb[1][4];
        hop_coefs<R>(kappa, 0.0, cf[0], cb[0]);
        const cx_t<R>* const fields[1] = {uj};
        wilson_site<R, 1, true>(g, links, fields, cf, cb, site, acc);
    }
    __syncthreads();
    if (!go) return;                                   // zero source or invariant subspace: the job stops
    const double svj = scal[0].x, cprev = scal[1].x;
    double part = 0.0;
    if (site < g.V) {
        const cx_t<R>* uj = column<R>(J, j, n);
        const cx_t<R>* up = (j >= 2) ? column<R>(J, j - 1, n) : nullptr;
        cx_t<R>* rout = (j < J.k) ? column<R>(J, j + 1, n) : nullptr;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const size_t e = (size_t)c * g.V + site;
            double2 r = cscale(to_d2<R>(acc[0][c]), svj);
            if (up) r = csub(r, cscale(to_d2<R>(up[e]), cprev));
            cx_t<R> rs = from_d2<R>(r);
            if (rout) rout[e] = rs;
            const double2 rd = to_d2<R>(rs);
            const double2 u = to_d2<R>(uj[e]);
            part += u.x * rd.x + u.y * rd.y;                          // Re(conj(u_j) r)
            if (pass2) accumulate(J, j, e, n, u);
        }
    }
    const double2 s = block_sum<NT>(mk(part, 0.0), lds);
    if (threadIdx.x == 0) pslot(J, PS_S)[sb] = s;
}

template <typename R>
__global__ __launch_bounds__(NT) void herm_R(JobDesc* jobs, int V, int j, int nblocks, int njobs, int xcd_map,
                                             int pass2) {
    int sb, job;
    if (!block_coords(nblocks, njobs, xcd_map, sb, job)) return;
    const JobDesc& J = jobs[job];
    if (skip_R(J, j, pass2)) return;
    __shared__ double2 lds[NT / 64];
    __shared__ double salpha;
    const int n = 12 * V;
    const int site = sb * NT + threadIdx.x;
    const bool ok = site < V;
    // own-site operands first, then alpha_j from S_j's partials (wavefront 0)
    cx_t<R> rv[12], uv[12];
    cx_t<R>* r = column<R>(J, j + 1, n);
    if (ok) {
        const cx_t<R>* uj = column<R>(J, j, n);
#pragma unroll
        for (int c = 0; c < 12; ++c) { rv[c] = r[(size_t)c * V + site]; uv[c] = uj[(size_t)c * V + site]; }
    }
    const double svj = slot(J, SC_SV)[j].x;
    if (threadIdx.x < 64) {
        int cnt;
        const double2* ps = partials(J, PS_S, J.nblocks, cnt);
        const double alpha = svj * wave_sum(ps, cnt).x;
        if (threadIdx.x == 0) {
            salpha = alpha;
            if (sb == 0) slot(J, SC_ALPHA)[j] = mk(alpha, 0.0);
        }
    }
    __syncthreads();
    const double cu = salpha * svj;
    double nr2 = 0.0;
    if (ok) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const double2 v = csub(to_d2<R>(rv[c]), cscale(to_d2<R>(uv[c]), cu));
            const cx_t<R> vs = from_d2<R>(v);
            r[(size_t)c * V + site] = vs;
            nr2 += cabs2(to_d2<R>(vs));
        }
    }
    const double2 s = block_total<NT / 64>(mk(nr2, 0.0), lds);
    if (threadIdx.x == 0) pslot(J, PS_R0)[sb] = s;
}

// ------------------------------------------------------------------ two-sided step
// SPLIT = false: one thread computes A u_j and A^dagger t_j (links loaded once).
// SPLIT = true: blockIdx.z selects the field (0: A u_j, 1: A^dagger t_j), which
// halves the registers of a thread; the links are then shared through the caches.
template <typename R, bool SPLIT, int MINW>
__global__ __launch_bounds__(NT, MINW) void bi_S(JobDesc* jobs, Geom g, const cx_t<R>* __restrict__ links,
                                                double kappa, double mu, int j, int nblocks, int njobs,
                                                int xcd_map, int pass2) {
    int sb, job;
    if (!block_coords(nblocks, njobs, xcd_map, sb, job)) return;
    const JobDesc& J = jobs[job];
    if (skip_S(J, j, pass2)) return;
    __shared__ double2 lds[NT / 64];
    __shared__ double2 scal[4];
    __shared__ int go;
    const int n = 12 * g.V;
    const int field = SPLIT ? (int)blockIdx.z : 0;
    // v_j = sv u_j, w_j = sw t_j; subtract cv u_{j-1}, cw t_{j-1}: by wavefront 0
    // alone, handed over through LDS at the barrier after the stencil, so the
    // other wavefront starts its stencil at once
    if (threadIdx.x < 64) {
        double2 a0 = mk(0.0, 0.0), a1 = a0, a2 = a0, a3 = a0;
        const bool more = bi_scalars(J, j, sb == 0 && threadIdx.x == 0 && field == 0, a0, a1, a2, a3);
        if (threadIdx.x == 0) { scal[0] = a0; scal[1] = a1; scal[2] = a2; scal[3] = a3; go = more ? 1 : 0; }
    }
    const int site = sb * NT + threadIdx.x;
    const cx_t<R>* uj = column<R>(J, j, n);
    const cx_t<R>* tj = lvec<R>(J, j, n);
    constexpr int NF = SPLIT ? 1 : 2;     // fields of this thread: A u_j (and A^dagger t_j)
    cx_t<R> acc[NF][12];
    if (site < g.V) {
        R cf[NF][4], cb[NF][4];
        if constexpr (!SPLIT) {
            hop_coefs<R>(kappa, mu, cf[0], cb[0]);     // A
            hop_coefs<R>(kappa, -mu, cf[NF - 1], cb[NF - 1]);    // A^dagger = A(-mu)
            const cx_t<R>* const fields[NF] = {uj, tj};
            wilson_site<R, NF>(g, links, fields, cf, cb, site, acc);
        } else {
            hop_coefs<R>(kappa, field == 0 ? mu : -mu, cf[0], cb[0]);
            const cx_t<R>* const fields[NF] = {field == 0 ? uj : tj};
            wilson_site<R, NF>(g, links, fields, cf, cb, site, acc);
        }
    }
    __syncthreads();
    if (!go) return;                                   // zero source or breakdown: the job stops
    const double2 sv = scal[0], sw = scal[1], cv = scal[2], cw = scal[3];
    double2 part = mk(0.0, 0.0);
    if (site < g.V) {
        const cx_t<R>* up = (j >= 2) ? column<R>(J, j - 1, n) : nullptr;
        cx_t<R>* tl = lvec<R>(J, j + 1, n);        // holds t_{j-1}; overwritten by l (own site only)
        cx_t<R>* rout = (j < J.k) ? column<R>(J, j + 1, n) : nullptr;
        if constexpr (!SPLIT) {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const size_t e = (size_t)c * g.V + site;
                double2 r = cmul(sv, to_d2<R>(acc[0][c]));
                double2 l = cmul(sw, to_d2<R>(acc[NF - 1][c]));
                if (up) {
                    r = csub(r, cmul(cv, to_d2<R>(up[e])));
                    l = csub(l, cmul(cw, to_d2<R>(tl[e])));
                }
                const cx_t<R> rs = from_d2<R>(r);
                if (pass2) accumulate(J, j, e, n, to_d2<R>(uj[e]));
                if (rout) { rout[e] = rs; tl[e] = from_d2<R>(l); }
                part = cadd(part, cmulc(to_d2<R>(tj[e]), to_d2<R>(rs)));   // conj(t_j) r
            }
        } else if (field == 0) {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const size_t e = (size_t)c * g.V + site;
                double2 r = cmul(sv, to_d2<R>(acc[0][c]));
                if (up) r = csub(r, cmul(cv, to_d2<R>(up[e])));
                const cx_t<R> rs = from_d2<R>(r);
                if (pass2) accumulate(J, j, e, n, to_d2<R>(uj[e]));
                if (rout) rout[e] = rs;
                part = cadd(part, cmulc(to_d2<R>(tj[e]), to_d2<R>(rs)));   // conj(t_j) r
            }
        } else if (rout) {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const size_t e = (size_t)c * g.V + site;
                double2 l = cmul(sw, to_d2<R>(acc[0][c]));
                if (up) l = csub(l, cmul(cw, to_d2<R>(tl[e])));
                tl[e] = from_d2<R>(l);
            }
        }
    }
    if (field == 0) {
        const double2 s = block_sum<NT>(part, lds);
        if (threadIdx.x == 0) pslot(J, PS_S)[sb] = s;
    }
}

template <typename R>
__global__ __launch_bounds__(NT) void bi_R(JobDesc* jobs, int V, int j, int nblocks, int njobs, int xcd_map,
                                           int pass2) {
    int sb, job;
    if (!block_coords(nblocks, njobs, xcd_map, sb, job)) return;
    const JobDesc& J = jobs[job];
    if (skip_R(J, j, pass2)) return;
    __shared__ double2 lds0[NT / 64], lds1[NT / 64];
    __shared__ double2 salpha;
    const int n = 12 * V;
    const int site = sb * NT + threadIdx.x;
    const bool ok = site < V;
    cx_t<R>* r = column<R>(J, j + 1, n);
    cx_t<R>* l = lvec<R>(J, j + 1, n);
    const cx_t<R>* uj = column<R>(J, j, n);
    const cx_t<R>* tj = lvec<R>(J, j, n);
    // the right-hand vectors' own-site operands first, then alpha_j from S_j's partials (wavefront 0)
    cx_t<R> rv[12], uv[12];
    if (ok) {
#pragma unroll
        for (int c = 0; c < 12; ++c) { rv[c] = r[(size_t)c * V + site]; uv[c] = uj[(size_t)c * V + site]; }
    }
    const double2 sv = slot(J, SC_SV)[j], sw = slot(J, SC_SW)[j];
    if (threadIdx.x < 64) {
        int cnt;
        const double2* ps = partials(J, PS_S, J.nblocks, cnt);
        const double2 alpha = cmul(cconj(sw), wave_sum(ps, cnt));
        if (threadIdx.x == 0) {
            salpha = alpha;
            if (sb == 0) slot(J, SC_ALPHA)[j] = alpha;
        }
    }
    __syncthreads();
    const double2 alpha = salpha;
    const double2 cu = cmul(alpha, sv);                 // alpha v_j = cu u_j
    const double2 ct = cmul(cconj(alpha), sw);          // conj(alpha) w_j = ct t_j
    double2 d = mk(0.0, 0.0);
    double nr2 = 0.0, nl2 = 0.0;
    if (ok) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const size_t e = (size_t)c * V + site;
            const cx_t<R> rn = from_d2<R>(csub(to_d2<R>(rv[c]), cmul(cu, to_d2<R>(uv[c]))));
            const cx_t<R> ln = from_d2<R>(csub(to_d2<R>(l[e]), cmul(ct, to_d2<R>(tj[e]))));
            r[e] = rn;
            l[e] = ln;
            const double2 rd = to_d2<R>(rn), ld = to_d2<R>(ln);
            d = cadd(d, cmulc(rd, ld));                      // r^dagger l
            nr2 += cabs2(rd);
            nl2 += cabs2(ld);
        }
    }
    // the three block sums with one barrier: (r^dagger l) and (|r|^2, |l|^2)
    double2 e0 = d, e1 = mk(nr2, nl2);
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) { e0 = cadd(e0, shfl_xor_d2(e0, m)); e1 = cadd(e1, shfl_xor_d2(e1, m)); }
    if ((threadIdx.x & 63) == 0) { lds0[threadIdx.x >> 6] = e0; lds1[threadIdx.x >> 6] = e1; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double2 t0 = lds0[0], t1 = lds1[0];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) { t0 = cadd(t0, lds0[w]); t1 = cadd(t1, lds1[w]); }
        pslot(J, PS_R0)[sb] = t0;
        pslot(J, PS_R1)[sb] = mk(t1.x, 0.0);
        pslot(J, PS_R2)[sb] = mk(t1.y, 0.0);
    }
}

// ------------------------------------------------------------------ lift
constexpr int LIFT_NT = 256;

template <typename R>
__global__ __launch_bounds__(LIFT_NT) void lift_kernel(JobDesc* jobs, int V) {
    const JobDesc& J = jobs[blockIdx.y];
    const int n = 12 * V;
    const int e = blockIdx.x * LIFT_NT + threadIdx.x;   // e = comp * V + site
    if (e >= n) return;
    const int c = e / V, s = e - c * V;
    const int kused = J.status[ST_KUSED];
    double2 acc0 = mk(0.0, 0.0), acc1 = mk(0.0, 0.0);
    if (J.ring) {
        // double-pass mode: the second pass has summed the basis already
        if (kused >= 1) acc0 = J.yacc[e];
        if (kused >= 2) acc1 = J.yacc[(size_t)n + e];
    } else {
        const cx_t<R>* base = reinterpret_cast<const cx_t<R>*>(J.vstore) + e;
        int jj = 0;
        for (; jj + 1 < kused; jj += 2) {
            const double2 a = to_d2<R>(base[(size_t)jj * n]);
            const double2 b = to_d2<R>(base[(size_t)(jj + 1) * n]);
            acc0 = cadd(acc0, cmul(J.omega[jj], a));
            acc1 = cadd(acc1, cmul(J.omega[jj + 1], b));
        }
        if (jj < kused) acc0 = cadd(acc0, cmul(J.omega[jj], to_d2<R>(base[(size_t)jj * n])));
    }
    double2 y = cadd(acc0, acc1);
    // deflation (App. C step 6): + sum_i sgn(lambda_i) <l_i, b> r_i
    for (int i = 0; i < J.dm; ++i) y = cadd(y, cscale(cmul(J.dcoef[i], J.dr[(size_t)i * n + e]), J.dsgn[i]));
    if (J.overlap) {
        // D_ov(mu) b = b + gamma5 sgn(gamma5 D_w(mu)) b (Sec. 2, Eq. Dovmu); gamma5 = diag(1, 1, -1, -1)
        const double2 bv = J.b[(size_t)12 * s + c];
        y = (c < 6) ? cadd(bv, y) : csub(bv, y);
    }
    J.x[(size_t)12 * s + c] = y;
}

}  // namespace

void launch_pack(const OuterLaunch& L, hipStream_t s) {
    dim3 grid(L.nblocks, L.njobs);
    if (L.deflate && !L.pass2) hipLaunchKernelGGL(deflate_dots_kernel, grid, dim3(NT), 0, s, L.jobs, L.g.V, L.nblocks);
    if (L.precision == NKS_FP64)
        hipLaunchKernelGGL(pack_kernel<double>, grid, dim3(NT), 0, s, L.jobs, L.g.V, L.nblocks, L.pass2);
    else
        hipLaunchKernelGGL(pack_kernel<float>, grid, dim3(NT), 0, s, L.jobs, L.g.V, L.nblocks, L.pass2);
    launch_collapse(L, PS_R0, 1, L.nblocks, s);
}

// A launch of the outer passes: timed through the dispatch packet when L.ev is set.
template <typename F, typename... Args>
static void dispatch(const OuterLaunch& L, F kernel, dim3 grid, dim3 block, hipStream_t s, Args... args) {
    if (L.ev.a) hipExtLaunchKernelGGL(kernel, grid, block, 0, s, L.ev.a, L.ev.b, 0, args...);
    else hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

static dim3 outer_grid(const OuterLaunch& L, int z) {
    if (L.tune.xcd_map) return dim3(8 * xcd_slots(L.nblocks, L.njobs, L.tune.xcd_map), 1, z);
    return dim3(L.nblocks, L.njobs, z);
}

template <typename R, int MINW>
static void outer_S_w(const OuterLaunch& L, int j, hipStream_t s) {
    auto links = static_cast<const cx_t<R>*>(L.links);
    const int xm = L.tune.xcd_map;
    if (!L.two_sided) {
        dispatch(L, herm_S<R, MINW>, outer_grid(L, 1), dim3(NT), s, L.jobs, L.g, links, L.kappa, j, L.nblocks,
                 L.njobs, xm, L.pass2);
    } else if (L.tune.split_dual) {
        dispatch(L, bi_S<R, true, MINW>, outer_grid(L, 2), dim3(NT), s, L.jobs, L.g, links, L.kappa, L.mu, j,
                 L.nblocks, L.njobs, xm, L.pass2);
    } else {
        dispatch(L, bi_S<R, false, MINW>, outer_grid(L, 1), dim3(NT), s, L.jobs, L.g, links, L.kappa, L.mu, j,
                 L.nblocks, L.njobs, xm, L.pass2);
    }
}

template <typename R>
static void outer_S(const OuterLaunch& L, int j, hipStream_t s) {
    switch (L.tune.min_waves) {
        case 3: outer_S_w<R, 3>(L, j, s); break;
        case 4: outer_S_w<R, 4>(L, j, s); break;
        default: outer_S_w<R, 1>(L, j, s); break;
    }
}

template <typename R>
static void outer_R(const OuterLaunch& L, int j, hipStream_t s) {
    const int xm = L.tune.xcd_map;
    if (!L.two_sided)
        dispatch(L, herm_R<R>, outer_grid(L, 1), dim3(NT), s, L.jobs, L.g.V, j, L.nblocks, L.njobs, xm, L.pass2);
    else
        dispatch(L, bi_R<R>, outer_grid(L, 1), dim3(NT), s, L.jobs, L.g.V, j, L.nblocks, L.njobs, xm, L.pass2);
}

void launch_collapse(const OuterLaunch& L, int slot0, int nslots, int nb, hipStream_t s) {
    if (nb <= L.tune.collapse) return;
    hipLaunchKernelGGL(collapse_kernel, dim3(L.njobs), dim3(64), 0, s, L.jobs, slot0, nslots, nb);
}

void launch_outer_S(const OuterLaunch& L, int j, hipStream_t s) {
    if (L.precision == NKS_FP64) outer_S<double>(L, j, s);
    else outer_S<float>(L, j, s);
    launch_collapse(L, PS_S, 1, L.nblocks, s);
}

void launch_outer_R(const OuterLaunch& L, int j, hipStream_t s) {
    if (L.precision == NKS_FP64) outer_R<double>(L, j, s);
    else outer_R<float>(L, j, s);
    launch_collapse(L, PS_R0, L.two_sided ? 3 : 1, L.nblocks, s);
}

void launch_lift(const OuterLaunch& L, hipStream_t s) {
    const int n = 12 * L.g.V;
    dim3 grid((n + LIFT_NT - 1) / LIFT_NT, L.njobs);
    if (L.precision == NKS_FP64)
        dispatch(L, lift_kernel<double>, grid, dim3(LIFT_NT), s, L.jobs, L.g.V);
    else
        dispatch(L, lift_kernel<float>, grid, dim3(LIFT_NT), s, L.jobs, L.g.V);
}

}  // namespace nks
