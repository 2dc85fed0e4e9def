// Small dense complex linear algebra on the host (p x p, p <= 128) for the
// Rayleigh-Ritz steps of the eigensolver: Cholesky, the inverse adjoint of
// a triangular factor, Hermitian Jacobi, and the general eigenproblem by
// Hessenberg reduction and shifted QR.  Matrices are column-major
// std::vector<std::complex<double>>, a(i, j) = a[i + j p].  No HIP here, so
// the routines are also built and checked on the CPU alone.
#pragma once

#include <cmath>
#include <complex>
#include <vector>

namespace nks {
namespace dense {

using cd = std::complex<double>;
using Mat = std::vector<cd>;

// In place: the lower Cholesky factor L of the Hermitian positive definite G
// (upper part zeroed); false if G is not numerically positive definite.
inline bool cholesky(Mat& G, int p) {
    for (int j = 0; j < p; ++j) {
        double d = G[j + (size_t)j * p].real();
        for (int k = 0; k < j; ++k) d -= std::norm(G[j + (size_t)k * p]);
        if (!(d > 0.0)) return false;
        const double ljj = std::sqrt(d);
        G[j + (size_t)j * p] = ljj;
        for (int i = j + 1; i < p; ++i) {
            cd s = G[i + (size_t)j * p];
            for (int k = 0; k < j; ++k) s -= G[i + (size_t)k * p] * std::conj(G[j + (size_t)k * p]);
            G[i + (size_t)j * p] = s / ljj;
        }
        for (int i = 0; i < j; ++i) G[i + (size_t)j * p] = 0.0;
    }
    return true;
}

// Z = L^{-H} for the lower triangular L (solve L^H Z = I by back substitution)
inline Mat inverse_adjoint(const Mat& L, int p) {
    Mat Z((size_t)p * p, 0.0);
    for (int c = 0; c < p; ++c)
        for (int i = p - 1; i >= 0; --i) {
            cd s = (i == c) ? 1.0 : 0.0;
            for (int k = i + 1; k < p; ++k) s -= std::conj(L[k + (size_t)i * p]) * Z[k + (size_t)c * p];
            Z[i + (size_t)c * p] = s / std::conj(L[i + (size_t)i * p]);
        }
    return Z;
}

// (H + H^H) / 2 in place
inline void symmetrise(Mat& H, int p) {
    for (int j = 0; j < p; ++j) {
        for (int i = 0; i < j; ++i) {
            const cd v = 0.5 * (H[i + (size_t)j * p] + std::conj(H[j + (size_t)i * p]));
            H[i + (size_t)j * p] = v;
            H[j + (size_t)i * p] = std::conj(v);
        }
        H[j + (size_t)j * p] = H[j + (size_t)j * p].real();
    }
}

// Cyclic Jacobi for the Hermitian H (overwritten): H = W diag(w) W^H.  Each
// rotation first makes the (k, l) entry real by a phase, then zeroes it.
inline void jacobi(Mat& H, int p, std::vector<double>& w, Mat& W) {
    W.assign((size_t)p * p, 0.0);
    for (int i = 0; i < p; ++i) W[i + (size_t)i * p] = 1.0;
    auto at = [&](int i, int j) -> cd& { return H[i + (size_t)j * p]; };
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int j = 0; j < p; ++j)
            for (int i = 0; i < p; ++i) {
                tot += std::norm(at(i, j));
                if (i != j) off += std::norm(at(i, j));
            }
        if (off <= 1e-30 * tot) break;
        for (int k = 0; k < p - 1; ++k)
            for (int l = k + 1; l < p; ++l) {
                const cd g = at(k, l);
                const double ag = std::abs(g);
                if (ag == 0.0) continue;
                const cd ph = g / ag;
                const double a = at(k, k).real(), b = at(l, l).real();
                const double tau = (b - a) / (2.0 * ag);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                // U = [[c, s ph], [-s conj(ph), c]] in the (k, l) plane: H <- U^H H U, W <- W U
                for (int i = 0; i < p; ++i) {
                    const cd hik = at(i, k), hil = at(i, l);
                    at(i, k) = c * hik - s * std::conj(ph) * hil;
                    at(i, l) = s * ph * hik + c * hil;
                }
                for (int j = 0; j < p; ++j) {
                    const cd hkj = at(k, j), hlj = at(l, j);
                    at(k, j) = c * hkj - s * ph * hlj;
                    at(l, j) = s * std::conj(ph) * hkj + c * hlj;
                }
                at(k, l) = 0.0;
                at(l, k) = 0.0;
                for (int i = 0; i < p; ++i) {
                    const cd wik = W[i + (size_t)k * p], wil = W[i + (size_t)l * p];
                    W[i + (size_t)k * p] = c * wik - s * std::conj(ph) * wil;
                    W[i + (size_t)l * p] = s * ph * wik + c * wil;
                }
            }
    }
    w.resize(p);
    for (int i = 0; i < p; ++i) w[i] = at(i, i).real();
}

// General complex eigenproblem A v = lambda v (A p x p, not overwritten):
// Householder reduction to Hessenberg form, shifted QR with Givens rotations
// to the Schur form T = Z^H A Z, eigenvectors of T by back substitution,
// v = Z y normalised to unit length.  False if QR does not converge.
inline bool eig_general(const Mat& A, int p, std::vector<cd>& lam, Mat& V) {
    Mat H = A;
    Mat Z((size_t)p * p, 0.0);
    for (int i = 0; i < p; ++i) Z[i + (size_t)i * p] = 1.0;
    auto h = [&](int i, int j) -> cd& { return H[i + (size_t)j * p]; };
    auto z = [&](int i, int j) -> cd& { return Z[i + (size_t)j * p]; };
    // Hessenberg reduction: P = I - 2 v v^H / (v^H v) on rows / columns k+1..p-1
    std::vector<cd> v(p);
    for (int k = 0; k + 2 < p; ++k) {
        double nx = 0.0;
        for (int i = k + 1; i < p; ++i) nx += std::norm(h(i, k));
        nx = std::sqrt(nx);
        if (nx == 0.0) continue;
        const cd x0 = h(k + 1, k);
        const cd ph = (std::abs(x0) > 0.0) ? x0 / std::abs(x0) : cd(1.0);
        for (int i = 0; i < p; ++i) v[i] = 0.0;
        for (int i = k + 1; i < p; ++i) v[i] = h(i, k);
        v[k + 1] += ph * nx;
        double vv = 0.0;
        for (int i = k + 1; i < p; ++i) vv += std::norm(v[i]);
        if (vv == 0.0) continue;
        for (int j = 0; j < p; ++j) {   // H <- P H
            cd s = 0.0;
            for (int i = k + 1; i < p; ++i) s += std::conj(v[i]) * h(i, j);
            s *= 2.0 / vv;
            for (int i = k + 1; i < p; ++i) h(i, j) -= v[i] * s;
        }
        for (int i = 0; i < p; ++i) {   // H <- H P, Z <- Z P
            cd s = 0.0, t = 0.0;
            for (int j = k + 1; j < p; ++j) {
                s += h(i, j) * v[j];
                t += z(i, j) * v[j];
            }
            s *= 2.0 / vv;
            t *= 2.0 / vv;
            for (int j = k + 1; j < p; ++j) {
                h(i, j) -= s * std::conj(v[j]);
                z(i, j) -= t * std::conj(v[j]);
            }
        }
        for (int i = k + 2; i < p; ++i) h(i, k) = 0.0;
    }
    // shifted QR on the active window [lo, hi]
    const double eps = 2.220446049250313e-16;
    int hi = p - 1, iter = 0, total = 0;
    std::vector<cd> gc(p), gs(p);   // Givens rotations of one sweep
    while (hi > 0) {
        int lo = hi;
        while (lo > 0) {
            const double sc = std::abs(h(lo, lo)) + std::abs(h(lo - 1, lo - 1));
            if (std::abs(h(lo, lo - 1)) <= eps * (sc > 0.0 ? sc : 1.0)) {
                h(lo, lo - 1) = 0.0;
                break;
            }
            --lo;
        }
        if (lo == hi) {   // 1 x 1 block converged
            --hi;
            iter = 0;
            continue;
        }
        if (++total > 60 * p) return false;
        ++iter;
        // Wilkinson shift: the eigenvalue of the trailing 2 x 2 closer to h(hi, hi)
        cd sigma;
        if (iter % 11 == 10) {
            sigma = h(hi, hi) + cd(std::abs(h(hi, hi - 1)), 0.0);   // exceptional shift
        } else {
            const cd a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
            const cd tr = a + d, det = a * d - b * c;
            const cd disc = std::sqrt(tr * tr / 4.0 - det);
            const cd l1 = tr / 2.0 + disc, l2 = tr / 2.0 - disc;
            sigma = (std::abs(l1 - d) < std::abs(l2 - d)) ? l1 : l2;
        }
        for (int i = lo; i <= hi; ++i) h(i, i) -= sigma;
        for (int k = lo; k < hi; ++k) {   // rows: zero h(k+1, k)
            const cd f = h(k, k), g = h(k + 1, k);
            const double r = std::sqrt(std::norm(f) + std::norm(g));
            cd c = 1.0, s = 0.0;
            if (r > 0.0) {
                c = f / r;
                s = g / r;
            }
            gc[k] = c;
            gs[k] = s;
            // [c^* s^*; -s c] applied to rows k, k+1
            for (int j = k; j < p; ++j) {
                const cd x = h(k, j), y = h(k + 1, j);
                h(k, j) = std::conj(c) * x + std::conj(s) * y;
                h(k + 1, j) = -s * x + c * y;
            }
        }
        for (int k = lo; k < hi; ++k) {   // columns: the inverse rotations from the right
            const cd c = gc[k], s = gs[k];
            const int rmax = (k + 2 <= hi) ? k + 2 : hi;
            for (int i = 0; i <= rmax; ++i) {
                const cd x = h(i, k), y = h(i, k + 1);
                h(i, k) = x * c + y * s;
                h(i, k + 1) = -x * std::conj(s) + y * std::conj(c);
            }
            for (int i = 0; i < p; ++i) {
                const cd x = z(i, k), y = z(i, k + 1);
                z(i, k) = x * c + y * s;
                z(i, k + 1) = -x * std::conj(s) + y * std::conj(c);
            }
        }
        for (int i = lo; i <= hi; ++i) h(i, i) += sigma;
    }
    lam.resize(p);
    for (int i = 0; i < p; ++i) lam[i] = h(i, i);
    // eigenvectors of the triangular T, then V = Z Y
    double tn = 0.0;
    for (int j = 0; j < p; ++j)
        for (int i = 0; i <= j; ++i) tn = std::fmax(tn, std::abs(h(i, j)));
    const double small = eps * (tn > 0.0 ? tn : 1.0);
    V.assign((size_t)p * p, 0.0);
    std::vector<cd> y(p);
    for (int k = 0; k < p; ++k) {
        for (int i = 0; i < p; ++i) y[i] = 0.0;
        y[k] = 1.0;
        for (int j = k - 1; j >= 0; --j) {
            cd s = 0.0;
            for (int l = j + 1; l <= k; ++l) s += h(j, l) * y[l];
            cd dd = h(j, j) - lam[k];
            if (std::abs(dd) < small) dd = small;
            y[j] = -s / dd;
        }
        double nv = 0.0;
        for (int i = 0; i < p; ++i) {
            cd s = 0.0;
            for (int l = 0; l <= k; ++l) s += z(i, l) * y[l];
            V[i + (size_t)k * p] = s;
            nv += std::norm(s);
        }
        nv = std::sqrt(nv);
        for (int i = 0; i < p; ++i) V[i + (size_t)k * p] /= nv;
    }
    return true;
}

}  // namespace dense
}  // namespace nks
