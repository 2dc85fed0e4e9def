// Wilson-Dirac stencil A = gamma5 D_w(mu) for one lattice site (Sec. 2).
//
// (D_w psi)(y) = psi(y) - kappa sum_nu [ c+_nu (1 + gamma_nu) U_{y-nu,nu} psi(y - nu)
//                                      + c-_nu (1 - gamma_nu) U_{y,nu}^dag psi(y + nu) ],
// c+-_nu = 1 for nu = x, y, z and c+-_t = e^{+-mu}.  A^dagger(mu) = A(-mu).
//
// Data layout (structure of arrays, site index fastest so that a wavefront
// reads 64 consecutive sites per load):
//   spinor  [comp = 3*spin + colour][site]
//   links   [nu][row][col][site],  U_{site,nu} transports site -> site + nu_hat
//
// Chiral basis: gamma_nu = [[0, B_nu], [B_nu^dag, 0]] with B = -i sigma_k
// (k = 1..3) and B = 1 for t.  (1 +- gamma) psi has rank two: with
// h = psi_up +- B psi_lo it equals (h, +- B^dag h), so each hop multiplies
// only a two-spin half spinor by the link.
#pragma once

#include "nks_internal.h"

namespace nks {

// (B psi_lo) for the lower spins l0, l1 -> the two upper spin entries
template <typename C>
__device__ __forceinline__ void b_lower(int nu, C l0, C l1, C& o0, C& o1) {
    switch (nu) {
        case 0: o0 = cmulmi(l1); o1 = cmulmi(l0); break;     // -i sigma_1
        case 1: o0 = cneg(l1); o1 = l0; break;               // -i sigma_2
        case 2: o0 = cmulmi(l0); o1 = cmuli(l1); break;      // -i sigma_3
        default: o0 = l0; o1 = l1; break;                    // 1
    }
}

// B^dagger g
template <typename C>
__device__ __forceinline__ void bdag(int nu, C g0, C g1, C& o0, C& o1) {
    switch (nu) {
        case 0: o0 = cmuli(g1); o1 = cmuli(g0); break;
        case 1: o0 = g1; o1 = cneg(g0); break;
        case 2: o0 = cmuli(g0); o1 = cmulmi(g1); break;
        default: o0 = g0; o1 = g1; break;
    }
}

// acc += coef * (1 + SGN gamma_nu) Umat psi(site)  with Umat = U (DAG=false) or U^dagger
template <int SGN, bool DAG, typename R>
__device__ __forceinline__ void hop(int nu, const cx_t<R> (&u)[9], const cx_t<R>* __restrict__ in, int site,
                                    int V, R coef, cx_t<R> (&acc)[12]) {
    using C = cx_t<R>;
    C h[2][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {   // project colour by colour: 4 loads live at a time
        const C p0 = in[(size_t)(0 + a) * V + site];
        const C p1 = in[(size_t)(3 + a) * V + site];
        const C p2 = in[(size_t)(6 + a) * V + site];
        const C p3 = in[(size_t)(9 + a) * V + site];
        C b0, b1;
        b_lower(nu, p2, p3, b0, b1);
        if constexpr (SGN > 0) { h[0][a] = cadd(p0, b0); h[1][a] = cadd(p1, b1); }
        else { h[0][a] = csub(p0, b0); h[1][a] = csub(p1, b1); }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        C g[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            C t;
            if constexpr (!DAG) {
                t = cmul(u[a * 3 + 0], h[s][0]);
                t = cadd(t, cmul(u[a * 3 + 1], h[s][1]));
                t = cadd(t, cmul(u[a * 3 + 2], h[s][2]));
            } else {
                t = cmulc(u[0 * 3 + a], h[s][0]);
                t = cadd(t, cmulc(u[1 * 3 + a], h[s][1]));
                t = cadd(t, cmulc(u[2 * 3 + a], h[s][2]));
            }
            g[a] = cscale(t, coef);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) h[s][a] = g[a];   // h now holds coef * Umat h
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        C o0, o1;
        bdag(nu, h[0][a], h[1][a], o0, o1);
        acc[a] = cadd(acc[a], h[0][a]);
        acc[3 + a] = cadd(acc[3 + a], h[1][a]);
        if constexpr (SGN > 0) { acc[6 + a] = cadd(acc[6 + a], o0); acc[9 + a] = cadd(acc[9 + a], o1); }
        else { acc[6 + a] = csub(acc[6 + a], o0); acc[9 + a] = csub(acc[9 + a], o1); }
    }
}

// The half spinor that one hop contributes: h = coef * Umat (1 + SGN gamma_nu) p
// reduced to its two upper spins (Umat = U, or U^dagger when DAG), for a
// neighbour spinor p already in registers (same operations as hop()).
template <int SGN, bool DAG, typename R>
__device__ __forceinline__ void hop_half(int nu, const cx_t<R> (&u)[9], const cx_t<R> (&p)[12], R coef,
                                         cx_t<R> (&h)[2][3]) {
    using C = cx_t<R>;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        C b0, b1;
        b_lower(nu, p[6 + a], p[9 + a], b0, b1);
        if constexpr (SGN > 0) { h[0][a] = cadd(p[a], b0); h[1][a] = cadd(p[3 + a], b1); }
        else { h[0][a] = csub(p[a], b0); h[1][a] = csub(p[3 + a], b1); }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        C g[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            C t;
            if constexpr (!DAG) {
                t = cmul(u[a * 3 + 0], h[s][0]);
                t = cadd(t, cmul(u[a * 3 + 1], h[s][1]));
                t = cadd(t, cmul(u[a * 3 + 2], h[s][2]));
            } else {
                t = cmulc(u[0 * 3 + a], h[s][0]);
                t = cadd(t, cmulc(u[1 * 3 + a], h[s][1]));
                t = cadd(t, cmulc(u[2 * 3 + a], h[s][2]));
            }
            g[a] = cscale(t, coef);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) h[s][a] = g[a];
    }
}

// Component c (= 3 spin + colour) of the full spinor of a hop's half spinor h:
// the upper spins are h itself, the lower ones SGN B_nu^dagger h.  acc += it.
template <typename C>
__device__ __forceinline__ C hop_component_add(int nu, int sgn, int c, const C& h0, const C& h1, C acc) {
    // h0, h1: h[0][colour], h[1][colour]
    if (c < 6) return cadd(acc, c < 3 ? h0 : h1);
    C o0, o1;
    bdag(nu, h0, h1, o0, o1);
    const C o = c < 9 ? o0 : o1;
    return sgn > 0 ? cadd(acc, o) : csub(acc, o);
}

// hop() on a neighbour spinor already in registers (same operations)
template <int SGN, bool DAG, typename R>
__device__ __forceinline__ void hop_pre(int nu, const cx_t<R> (&u)[9], const cx_t<R> (&p)[12], R coef,
                                        cx_t<R> (&acc)[12]) {
    using C = cx_t<R>;
    C h[2][3];
    hop_half<SGN, DAG, R>(nu, u, p, coef, h);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        C o0, o1;
        bdag(nu, h[0][a], h[1][a], o0, o1);
        acc[a] = cadd(acc[a], h[0][a]);
        acc[3 + a] = cadd(acc[3 + a], h[1][a]);
        if constexpr (SGN > 0) { acc[6 + a] = cadd(acc[6 + a], o0); acc[9 + a] = cadd(acc[9 + a], o1); }
        else { acc[6 + a] = csub(acc[6 + a], o0); acc[9 + a] = csub(acc[9 + a], o1); }
    }
}

// Neighbour of site in direction nu: forward (site + nu_hat) or backward, periodic.
__device__ __forceinline__ int neighbour_site(const Geom& g, int site, int nu, bool forward) {
    const int x = site % g.lx;
    int r = site / g.lx;
    const int y = r % g.ly;
    r /= g.ly;
    const int z = r % g.lz;
    const int t = r / g.lz;
    const int co = nu == 0 ? x : nu == 1 ? y : nu == 2 ? z : t;
    const int ext = nu == 0 ? g.lx : nu == 1 ? g.ly : nu == 2 ? g.lz : g.lt;
    const int st = nu == 0 ? 1 : nu == 1 ? g.lx : nu == 2 ? g.lx * g.ly : g.lx * g.ly * g.lz;
    if (forward) return (co == ext - 1) ? site - (ext - 1) * st : site + st;
    return (co == 0) ? site + (ext - 1) * st : site - st;
}

template <typename R>
__device__ __forceinline__ void load_link(const cx_t<R>* __restrict__ links, int nu, int site, int V,
                                          cx_t<R> (&u)[9]) {
#pragma unroll
    for (int rc = 0; rc < 9; ++rc) u[rc] = links[(size_t)(nu * 9 + rc) * V + site];
}

// acc[f] = (A_f in[f])(site) with A_f = gamma5 D_w(mu_f); mu_f enters via cf/cb:
// cf[f][nu] = -kappa * (nu == 3 ? e^{-mu_f} : 1), cb[f][nu] = -kappa * (nu == 3 ? e^{+mu_f} : 1).
// The direction loop is kept rolled so that only one direction's operands are
// live.  PRE (one field): both hops' links and neighbour spinors are loaded
// before either hop is computed, more loads in flight for the price of about
// 30 registers (a gain where the kernel keeps its occupancy).
template <typename R, int NF, bool PRE = false>
__device__ __forceinline__ void wilson_site(const Geom& g, const cx_t<R>* __restrict__ links,
                                            const cx_t<R>* const (&in)[NF], const R (&cf)[NF][4],
                                            const R (&cb)[NF][4], int site, cx_t<R> (&acc)[NF][12]) {
    const int x = site % g.lx;
    int r = site / g.lx;
    const int y = r % g.ly;
    r /= g.ly;
    const int z = r % g.lz;
    const int t = r / g.lz;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[f][c] = in[f][(size_t)c * g.V + site];
#pragma unroll 1
    for (int nu = 0; nu < 4; ++nu) {
        const int co = nu == 0 ? x : nu == 1 ? y : nu == 2 ? z : t;
        const int ext = nu == 0 ? g.lx : nu == 1 ? g.ly : nu == 2 ? g.lz : g.lt;
        const int st = nu == 0 ? 1 : nu == 1 ? g.lx : nu == 2 ? g.lx * g.ly : g.lx * g.ly * g.lz;
        const int fwd = (co == ext - 1) ? site - (ext - 1) * st : site + st;
        const int bwd = (co == 0) ? site + (ext - 1) * st : site - st;
        if constexpr (PRE && NF == 1) {
            cx_t<R> uf[9], ub[9], pf[12], pb[12];
            load_link<R>(links, nu, site, g.V, uf);   // U_{y,nu}: forward hop, daggered
            load_link<R>(links, nu, bwd, g.V, ub);    // U_{y-nu,nu}: backward hop
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                pf[c] = in[0][(size_t)c * g.V + fwd];
                pb[c] = in[0][(size_t)c * g.V + bwd];
            }
            hop_pre<-1, true, R>(nu, uf, pf, cf[0][nu], acc[0]);
            hop_pre<+1, false, R>(nu, ub, pb, cb[0][nu], acc[0]);
        } else {
            cx_t<R> u[9];
            load_link<R>(links, nu, site, g.V, u);        // U_{y,nu}: forward hop, daggered
#pragma unroll
            for (int f = 0; f < NF; ++f) hop<-1, true, R>(nu, u, in[f], fwd, g.V, cf[f][nu], acc[f]);
            load_link<R>(links, nu, bwd, g.V, u);         // U_{y-nu,nu}: backward hop
#pragma unroll
            for (int f = 0; f < NF; ++f) hop<+1, false, R>(nu, u, in[f], bwd, g.V, cb[f][nu], acc[f]);
        }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int c = 6; c < 12; ++c) acc[f][c] = cneg(acc[f][c]);   // gamma5 = diag(1,1,-1,-1)
}

template <typename R>
__host__ __device__ inline void hop_coefs(double kappa, double mu, R (&cf)[4], R (&cb)[4]) {
    for (int nu = 0; nu < 3; ++nu) { cf[nu] = (R)(-kappa); cb[nu] = (R)(-kappa); }
    cf[3] = (R)(-kappa * exp(-mu));
    cb[3] = (R)(-kappa * exp(mu));
}

}  // namespace nks
