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
// Every block of S_{j+1} sums R_j's partials in the same order, so all blocks
// agree on beta_j (and on a breakdown) without a grid barrier; block 0 stores
// the scalars for the nested step.  All scalars stay on the device.
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
    if (threadIdx.x == 0) J.part[(size_t)PS_R0 * nblocks + blockIdx.x] = s;
}

// ------------------------------------------------------------------ Hermitian step
// Scalars of S_j from R_{j-1}'s partial sums: beta_{j-1} (|b| when j == 1),
// v_j = svj u_j and beta_{j-1} v_{j-1} = cprev u_{j-1}; block 0 (b0) stores
// them.  Returns false when the job stops here (zero source, invariant subspace).
template <int NTB>
__device__ inline bool herm_scalars(const JobDesc& J, int j, int nblocks, bool b0, double2* lds, double& svj,
                                    double& cprev) {
    const double beta = sqrt(sum_partials<NTB>(J.part + (size_t)PS_R0 * nblocks, nblocks, lds).x);
    if (j == 1) {
        if (beta == 0.0) {                                  // zero source: x = 0
            if (b0) { J.status[ST_DONE] = 1; J.status[ST_KUSED] = 0; J.report[RP_BNORM] = 0.0; }
            return false;
        }
        svj = 1.0 / beta;
        cprev = 0.0;
        if (b0) { J.report[RP_BNORM] = beta; slot(J, SC_SV)[1] = mk(svj, 0.0); slot(J, SC_VN)[1] = mk(1.0, 0.0); }
        return true;
    }
    const double aprev = slot(J, SC_ALPHA)[j - 1].x;
    const double bprev = (j >= 3) ? slot(J, SC_BETA)[j - 2].x : 0.0;
    if (beta <= LUCKY_TAU_HERMITIAN * (fabs(aprev) + bprev)) {   // invariant subspace
        if (b0) { J.status[ST_DONE] = 1; J.status[ST_KUSED] = j - 1; }
        return false;
    }
    svj = 1.0 / beta;
    cprev = beta * slot(J, SC_SV)[j - 1].x;                       // beta_{j-1} v_{j-1} = cprev u_{j-1}
    if (b0) {
        slot(J, SC_BETA)[j - 1] = mk(beta, 0.0);
        slot(J, SC_GAMMA)[j - 1] = mk(beta, 0.0);
        slot(J, SC_SV)[j] = mk(svj, 0.0);
        slot(J, SC_VN)[j] = mk(1.0, 0.0);
    }
    return true;
}

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
    const int n = 12 * g.V;
    double svj, cprev;
    if (!herm_scalars<NT>(J, j, nblocks, sb == 0 && threadIdx.x == 0, lds, svj, cprev)) return;
    const int site = sb * NT + threadIdx.x;
    double part = 0.0;
    if (site < g.V) {
        const cx_t<R>* uj = column<R>(J, j, n);
        R cf[1][4], cb[1][4];
        hop_coefs<R>(kappa, 0.0, cf[0], cb[0]);
        const cx_t<R>* const fields[1] = {uj};
        cx_t<R> acc[1][12];
        wilson_site<R, 1, true>(g, links, fields, cf, cb, site, acc);
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
    if (threadIdx.x == 0) J.part[(size_t)PS_S * nblocks + sb] = s;
}

template <typename R>
__global__ __launch_bounds__(NT) void herm_R(JobDesc* jobs, int V, int j, int nblocks, int njobs, int xcd_map,
                                             int pass2) {
    int sb, job;
    if (!block_coords(nblocks, njobs, xcd_map, sb, job)) return;
    const JobDesc& J = jobs[job];
    if (skip_R(J, j, pass2)) return;
    __shared__ double2 lds[NT / 64];
    const int n = 12 * V;
    const double svj = slot(J, SC_SV)[j].x;
    const double alpha = svj * sum_partials<NT>(J.part + (size_t)PS_S * nblocks, nblocks, lds).x;
    if (sb == 0 && threadIdx.x == 0) slot(J, SC_ALPHA)[j] = mk(alpha, 0.0);
    const double cu = alpha * svj;
    const int site = sb * NT + threadIdx.x;
    double nr2 = 0.0;
    if (site < V) {
        const cx_t<R>* uj = column<R>(J, j, n);
        cx_t<R>* r = column<R>(J, j + 1, n);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const size_t e = (size_t)c * V + site;
            double2 v = csub(to_d2<R>(r[e]), cscale(to_d2<R>(uj[e]), cu));
            cx_t<R> vs = from_d2<R>(v);
            r[e] = vs;
            nr2 += cabs2(to_d2<R>(vs));
        }
    }
    const double2 s = block_sum<NT>(mk(nr2, 0.0), lds);
    if (threadIdx.x == 0) J.part[(size_t)PS_R0 * nblocks + sb] = s;
}

// Scalars of the two-sided S_j from R_{j-1}'s partial sums (App. B):
// v_j = sv u_j, w_j = sw t_j, gamma_{j-1} v_{j-1} = cv u_{j-1},
// conj(beta_{j-1}) w_{j-1} = cw t_{j-1}; block 0 (b0) stores them.  Returns
// false when the job stops here (zero source, lucky or serious breakdown).
template <int NTB>
__device__ inline bool bi_scalars(const JobDesc& J, int j, int nblocks, bool b0, double2* lds, double2& sv,
                                  double2& sw, double2& cv, double2& cw) {
    if (j == 1) {
        const double bn = sqrt(sum_partials<NTB>(J.part + (size_t)PS_R0 * nblocks, nblocks, lds).x);
        if (bn == 0.0) {
            if (b0) { J.status[ST_DONE] = 1; J.status[ST_KUSED] = 0; J.report[RP_BNORM] = 0.0; }
            return false;
        }
        sv = sw = mk(1.0 / bn, 0.0);
        cv = cw = mk(0.0, 0.0);
        if (b0) {
            J.report[RP_BNORM] = bn;
            slot(J, SC_SV)[1] = sv; slot(J, SC_SW)[1] = sw;
            slot(J, SC_VN)[1] = mk(1.0, 0.0); slot(J, SC_WN)[1] = mk(1.0, 0.0);
        }
    } else {
        const double2 delta = sum_partials<NTB>(J.part + (size_t)PS_R0 * nblocks, nblocks, lds);
        const double nr = sqrt(sum_partials<NTB>(J.part + (size_t)PS_R1 * nblocks, nblocks, lds).x);
        const double nl = sqrt(sum_partials<NTB>(J.part + (size_t)PS_R2 * nblocks, nblocks, lds).x);
        const double aprev = cabs(slot(J, SC_ALPHA)[j - 1]);
        const double sprev = (j >= 3) ? sqrt(cabs(cmul(slot(J, SC_BETA)[j - 2], slot(J, SC_GAMMA)[j - 2]))) : 0.0;
        const double S = aprev + sprev;
        if (nr <= LUCKY_TAU_TWO_SIDED * S * slot(J, SC_VN)[j - 1].x ||
            nl <= LUCKY_TAU_TWO_SIDED * S * slot(J, SC_WN)[j - 1].x) {
            if (b0) { J.status[ST_DONE] = 1; J.status[ST_KUSED] = j - 1; }
            return false;
        }
        if (cabs(delta) <= SERIOUS_TAU * nr * nl) {
            if (b0) {
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
        if (b0) {
            slot(J, SC_BETA)[j - 1] = beta; slot(J, SC_GAMMA)[j - 1] = gamma;
            slot(J, SC_SV)[j] = sv; slot(J, SC_SW)[j] = sw;
            slot(J, SC_VN)[j] = mk(nr / cabs(beta), 0.0);
            slot(J, SC_WN)[j] = mk(nl / cabs(gamma), 0.0);
        }
    }
    return true;
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
    const int n = 12 * g.V;
    const int field = SPLIT ? (int)blockIdx.z : 0;
    double2 sv, sw, cv, cw;   // v_j = sv u_j, w_j = sw t_j; subtract cv u_{j-1}, cw t_{j-1}
    if (!bi_scalars<NT>(J, j, nblocks, sb == 0 && threadIdx.x == 0 && field == 0, lds, sv, sw, cv, cw)) return;
    const int site = sb * NT + threadIdx.x;
    double2 part = mk(0.0, 0.0);
    if (site < g.V) {
        const cx_t<R>* uj = column<R>(J, j, n);
        const cx_t<R>* tj = lvec<R>(J, j, n);
        const cx_t<R>* up = (j >= 2) ? column<R>(J, j - 1, n) : nullptr;
        cx_t<R>* tl = lvec<R>(J, j + 1, n);        // holds t_{j-1}; overwritten by l (own site only)
        cx_t<R>* rout = (j < J.k) ? column<R>(J, j + 1, n) : nullptr;
        if constexpr (!SPLIT) {
            R cf[2][4], cb[2][4];
            hop_coefs<R>(kappa, mu, cf[0], cb[0]);     // A
            hop_coefs<R>(kappa, -mu, cf[1], cb[1]);    // A^dagger = A(-mu)
            const cx_t<R>* const fields[2] = {uj, tj};
            cx_t<R> acc[2][12];
            wilson_site<R, 2>(g, links, fields, cf, cb, site, acc);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const size_t e = (size_t)c * g.V + site;
                double2 r = cmul(sv, to_d2<R>(acc[0][c]));
                double2 l = cmul(sw, to_d2<R>(acc[1][c]));
                if (up) {
                    r = csub(r, cmul(cv, to_d2<R>(up[e])));
                    l = csub(l, cmul(cw, to_d2<R>(tl[e])));
                }
                const cx_t<R> rs = from_d2<R>(r);
                if (pass2) accumulate(J, j, e, n, to_d2<R>(uj[e]));
                if (rout) { rout[e] = rs; tl[e] = from_d2<R>(l); }
                part = cadd(part, cmulc(to_d2<R>(tj[e]), to_d2<R>(rs)));   // conj(t_j) r
            }
        } else {
            R cf[1][4], cb[1][4];
            hop_coefs<R>(kappa, field == 0 ? mu : -mu, cf[0], cb[0]);
            const cx_t<R>* const fields[1] = {field == 0 ? uj : tj};
            cx_t<R> acc[1][12];
            wilson_site<R, 1>(g, links, fields, cf, cb, site, acc);
            if (field == 0) {
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
    }
    if (field == 0) {
        const double2 s = block_sum<NT>(part, lds);
        if (threadIdx.x == 0) J.part[(size_t)PS_S * nblocks + sb] = s;
    }
}

template <typename R>
__global__ __launch_bounds__(NT) void bi_R(JobDesc* jobs, int V, int j, int nblocks, int njobs, int xcd_map,
                                           int pass2) {
    int sb, job;
    if (!block_coords(nblocks, njobs, xcd_map, sb, job)) return;
    const JobDesc& J = jobs[job];
    if (skip_R(J, j, pass2)) return;
    __shared__ double2 lds[NT / 64];
    const int n = 12 * V;
    const double2 sv = slot(J, SC_SV)[j], sw = slot(J, SC_SW)[j];
    const double2 alpha = cmul(cconj(sw), sum_partials<NT>(J.part + (size_t)PS_S * nblocks, nblocks, lds));
    if (sb == 0 && threadIdx.x == 0) slot(J, SC_ALPHA)[j] = alpha;
    const double2 cu = cmul(alpha, sv);                 // alpha v_j = cu u_j
    const double2 ct = cmul(cconj(alpha), sw);          // conj(alpha) w_j = ct t_j
    const int site = sb * NT + threadIdx.x;
    double2 d = mk(0.0, 0.0);
    double nr2 = 0.0, nl2 = 0.0;
    if (site < V) {
        const cx_t<R>* uj = column<R>(J, j, n);
        const cx_t<R>* tj = lvec<R>(J, j, n);
        cx_t<R>* r = column<R>(J, j + 1, n);
        cx_t<R>* l = lvec<R>(J, j + 1, n);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const size_t e = (size_t)c * V + site;
            const cx_t<R> rv = from_d2<R>(csub(to_d2<R>(r[e]), cmul(cu, to_d2<R>(uj[e]))));
            const cx_t<R> lv = from_d2<R>(csub(to_d2<R>(l[e]), cmul(ct, to_d2<R>(tj[e]))));
            r[e] = rv;
            l[e] = lv;
            const double2 rd = to_d2<R>(rv), ld = to_d2<R>(lv);
            d = cadd(d, cmulc(rd, ld));                      // r^dagger l
            nr2 += cabs2(rd);
            nl2 += cabs2(ld);
        }
    }
    double2 s = block_sum<NT>(d, lds);
    if (threadIdx.x == 0) J.part[(size_t)PS_R0 * nblocks + sb] = s;
    s = block_sum<NT>(mk(nr2, 0.0), lds);
    if (threadIdx.x == 0) J.part[(size_t)PS_R1 * nblocks + sb] = s;
    s = block_sum<NT>(mk(nl2, 0.0), lds);
    if (threadIdx.x == 0) J.part[(size_t)PS_R2 * nblocks + sb] = s;
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

void launch_outer_S(const OuterLaunch& L, int j, hipStream_t s) {
    if (L.precision == NKS_FP64) outer_S<double>(L, j, s);
    else outer_S<float>(L, j, s);
}

void launch_outer_R(const OuterLaunch& L, int j, hipStream_t s) {
    if (L.precision == NKS_FP64) outer_R<double>(L, j, s);
    else outer_R<float>(L, j, s);
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
