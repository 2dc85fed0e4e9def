// Deflation eigenpairs of A = gamma5 D_w(mu) (App. C step 1 needs the
// eigenpairs of A with the smallest |lambda|; the paper takes them from a
// separate eigensolver).  Chebyshev-filtered subspace iteration on a block
// of p vectors:
//
//   filter    X <- T_d(A^2) X, a Chebyshev polynomial of degree d in A^2 that
//             damps [a, b] (a = the largest squared Ritz value of the block in
//             modulus, b >= ||A||^2) and grows below a;
//   orthonormalise  X <- X L^{-H} twice, L the Cholesky factor of X^H X;
//   Rayleigh-Ritz on A^2   order the block by |theta^2|.  Hermitian A:
//             (AX)^H (AX) = W diag(theta^2) W^H, X <- X W.  Otherwise the Ritz
//             vectors of X^H A^2 X in that order, orthonormalised again (which
//             keeps the span of every leading group).  Squared Ritz values sit
//             at the low end of the spectrum of A^2, where Rayleigh-Ritz on the
//             indefinite A itself makes spurious values near 0 (mixtures of
//             +lambda and -lambda modes);
//   eigenpairs  Rayleigh-Ritz on A within the first m vectors, and the
//             residuals |A x - theta x| of the unit Ritz vectors.
//
// For mu != 0 the left eigenvectors are the right eigenvectors of
// A^dagger = A(-mu) (eigenvalues conj(lambda)): a second run on A(-mu), the
// two sets paired by eigenvalue and scaled to l_i^dagger r_i = 1.  The
// stencil, the filter recurrence, the Gram matrices X^H Y and the basis
// rotations X Z run on the GPU; the p x p steps (dense_host.h, p <= 128) run
// on the host in double precision.  Vectors are SoA blocks
// [vector][comp = 3 spin + colour][site] of complex128.
#include <algorithm>
#include <cmath>
#include <complex>
#include <random>
#include <string>
#include <vector>

#include "dense_host.h"
#include "wilson.h"

namespace nks {

namespace {

constexpr int ENT = 128;   // threads per block of the site-parallel kernels
constexpr int GNT = 256;   // threads per block of the reductions
constexpr int ROT = 8;     // outputs per thread of eig_rotate

// out_v = alpha (A(mu) in_v) + beta y_v + gamma z_v for v = blockIdx.y (y, z may be null)
__global__ __launch_bounds__(ENT) void eig_apply(Geom g, const double2* __restrict__ links, double kappa, double mu,
                                                 const double2* __restrict__ in, double2* __restrict__ out,
                                                 double alpha, const double2* __restrict__ y, double beta,
                                                 const double2* __restrict__ z, double gamma) {
    const int site = blockIdx.x * ENT + threadIdx.x;
    if (site >= g.V) return;
    const size_t n = (size_t)12 * g.V;
    const size_t off = (size_t)blockIdx.y * n;
    double cf[1][4], cb[1][4];
    hop_coefs<double>(kappa, mu, cf[0], cb[0]);
    const double2* const fields[1] = {in + off};
    double2 acc[1][12];
    wilson_site<double, 1>(g, links, fields, cf, cb, site, acc);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const size_t e = off + (size_t)c * g.V + site;
        double2 v = cscale(acc[0][c], alpha);
        if (y) v = cadd(v, cscale(y[e], beta));
        if (z) v = cadd(v, cscale(z[e], gamma));
        out[e] = v;
    }
}

// part[(i q + j) nchunk + chunk] = sum over the chunk of conj(X_i) Y_j
__global__ __launch_bounds__(GNT) void eig_gram(const double2* __restrict__ X, const double2* __restrict__ Y,
                                                int q, size_t n, int nchunk, double2* __restrict__ part) {
    __shared__ double2 lds[GNT / 64];
    const int chunk = blockIdx.x, i = blockIdx.y, j = blockIdx.z;
    const size_t len = (n + nchunk - 1) / nchunk;
    const size_t lo = (size_t)chunk * len, hi = (lo + len < n) ? lo + len : n;
    const double2* xi = X + (size_t)i * n;
    const double2* yj = Y + (size_t)j * n;
    double2 s = mk(0.0, 0.0);
    for (size_t e = lo + threadIdx.x; e < hi; e += GNT) s = cadd(s, cmulc(xi[e], yj[e]));
    s = block_sum<GNT>(s, lds);
    if (threadIdx.x == 0) part[((size_t)i * q + j) * nchunk + chunk] = s;
}

// out[r] = sum_c part[r nchunk + c] for r < count (fixed order)
__global__ __launch_bounds__(GNT) void eig_sum(const double2* __restrict__ part, int nchunk, int count,
                                               double2* __restrict__ out) {
    __shared__ double2 lds[GNT / 64];
    const int r = blockIdx.x;
    if (r >= count) return;
    double2 s = mk(0.0, 0.0);
    for (int c = threadIdx.x; c < nchunk; c += GNT) s = cadd(s, part[(size_t)r * nchunk + c]);
    s = block_sum<GNT>(s, lds);
    if (threadIdx.x == 0) out[r] = s;
}

// out_v = sum_{u < pin} X_u Z(u, v) for v < qout (Z column-major, pin x qout); ROT outputs per thread
__global__ __launch_bounds__(GNT) void eig_rotate(const double2* __restrict__ X, const double2* __restrict__ Z,
                                                  double2* __restrict__ out, int pin, int qout, size_t n) {
    const size_t e = (size_t)blockIdx.x * GNT + threadIdx.x;
    if (e >= n) return;
    const int v0 = blockIdx.y * ROT;
    double2 acc[ROT];
#pragma unroll
    for (int k = 0; k < ROT; ++k) acc[k] = mk(0.0, 0.0);
    for (int u = 0; u < pin; ++u) {
        const double2 x = X[(size_t)u * n + e];
#pragma unroll
        for (int k = 0; k < ROT; ++k)
            if (v0 + k < qout) acc[k] = cadd(acc[k], cmul(x, Z[(size_t)(v0 + k) * pin + u]));
    }
#pragma unroll
    for (int k = 0; k < ROT; ++k)
        if (v0 + k < qout) out[(size_t)(v0 + k) * n + e] = acc[k];
}

// part[v nchunk + chunk] = sum over the chunk of |AX_v - theta_v X_v|^2 (in .x)
__global__ __launch_bounds__(GNT) void eig_resid(const double2* __restrict__ AX, const double2* __restrict__ X,
                                                 const double2* __restrict__ theta, size_t n, int nchunk,
                                                 double2* __restrict__ part) {
    __shared__ double2 lds[GNT / 64];
    const int chunk = blockIdx.x, v = blockIdx.y;
    const size_t len = (n + nchunk - 1) / nchunk;
    const size_t lo = (size_t)chunk * len, hi = (lo + len < n) ? lo + len : n;
    const double2 t = theta[v];
    double s = 0.0;
    for (size_t e = lo + threadIdx.x; e < hi; e += GNT)
        s += cabs2(csub(AX[(size_t)v * n + e], cmul(t, X[(size_t)v * n + e])));
    const double2 r = block_sum<GNT>(mk(s, 0.0), lds);
    if (threadIdx.x == 0) part[(size_t)v * nchunk + chunk] = r;
}

using dense::cd;
using dense::Mat;

struct Dev {
    double2 *X = nullptr, *Y = nullptr, *T = nullptr, *U = nullptr, *part = nullptr, *small = nullptr;
    double2* theta = nullptr;
    ~Dev() {
        for (void* q : {(void*)X, (void*)Y, (void*)T, (void*)U, (void*)part, (void*)small, (void*)theta})
            if (q) (void)hipFree(q);
    }
};

// One lattice's device side: the operator A(mu), launch shapes and the block buffers.
struct Run {
    Geom g;
    const double2* links = nullptr;
    double kappa = 0.0, mu = 0.0;
    size_t n = 0;
    int nb = 0, nchunk = 0, p = 0;
    Dev d;

    void apply(const double2* in, double2* out, int count, double alpha = 1.0, const double2* y = nullptr,
               double beta = 0.0, const double2* z = nullptr, double gamma = 0.0) {
        hipLaunchKernelGGL(eig_apply, dim3(nb, count), dim3(ENT), 0, nullptr, g, links, kappa, mu, in, out, alpha, y,
                           beta, z, gamma);
    }
    // out = X^H Y of the first q vectors (host, column-major: out[i + j q] = X_i^H Y_j)
    bool gram(const double2* X, const double2* Y, int q, Mat& out) {
        hipLaunchKernelGGL(eig_gram, dim3(nchunk, q, q), dim3(GNT), 0, nullptr, X, Y, q, n, nchunk, d.part);
        hipLaunchKernelGGL(eig_sum, dim3(q * q), dim3(GNT), 0, nullptr, d.part, nchunk, q * q, d.small);
        std::vector<double2> h((size_t)q * q);
        if (hipMemcpy(h.data(), d.small, sizeof(double2) * q * q, hipMemcpyDeviceToHost) != hipSuccess) return false;
        out.resize((size_t)q * q);
        for (int i = 0; i < q; ++i)
            for (int j = 0; j < q; ++j) out[i + (size_t)j * q] = cd(h[(size_t)i * q + j].x, h[(size_t)i * q + j].y);
        return true;
    }
    // out_v = sum_{u < pin} X_u Z(u, v) for v < qout
    bool rotate(const double2* X, const Mat& Z, double2* out, int pin, int qout) {
        std::vector<double2> h((size_t)pin * qout);
        for (size_t r = 0; r < h.size(); ++r) h[r] = mk(Z[r].real(), Z[r].imag());
        if (hipMemcpy(d.small, h.data(), sizeof(double2) * h.size(), hipMemcpyHostToDevice) != hipSuccess) return false;
        hipLaunchKernelGGL(eig_rotate, dim3((unsigned)((n + GNT - 1) / GNT), (qout + ROT - 1) / ROT), dim3(GNT), 0,
                           nullptr, X, d.small, out, pin, qout, n);
        return hipGetLastError() == hipSuccess;
    }
    // X <- X L^{-H} with X^H X = L L^H, twice
    int orthonormalise(std::string& err) {
        Mat G;
        for (int pass = 0; pass < 2; ++pass) {
            if (!gram(d.X, d.X, p, G)) { err = "eigensolver: gram"; return NKS_E_HIP; }
            if (!dense::cholesky(G, p)) { err = "eigensolver: block lost rank (Cholesky of X^H X failed)"; return NKS_E_NOCONV; }
            if (!rotate(d.X, dense::inverse_adjoint(G, p), d.Y, p, p)) { err = "eigensolver: rotate"; return NKS_E_HIP; }
            std::swap(d.X, d.Y);
        }
        return NKS_OK;
    }
    // X <- T_deg(A^2) X, the Chebyshev filter on [a, b] scaled to 1 at a0 (three-term recurrence)
    bool filter(int deg, double a, double b, double a0) {
        const double e = (b - a) / 2.0, c = (b + a) / 2.0;
        double sigma = e / (a0 - c);
        const double tau = 2.0 / sigma;
        apply(d.X, d.T, p);
        apply(d.T, d.Y, p, sigma / e, d.X, -c * sigma / e);
        double2 *Xp = d.X, *Yc = d.Y, *Yn = d.U;
        for (int i = 2; i <= deg; ++i) {
            const double sigma2 = 1.0 / (tau - sigma);
            apply(Yc, d.T, p);
            apply(d.T, Yn, p, 2.0 * sigma2 / e, Yc, -2.0 * c * sigma2 / e, Xp, -sigma * sigma2);
            double2* t = Xp;
            Xp = Yc;
            Yc = Yn;
            Yn = t;
            sigma = sigma2;
        }
        if (Yc != d.X) {   // the filtered block becomes X; the buffers keep their roles
            double2* old_x = d.X;
            d.X = Yc;
            if (d.Y == Yc) d.Y = old_x;
            else d.U = old_x;
        }
        return hipGetLastError() == hipSuccess;
    }
};

// Indices 0..q-1 in ascending order of key (stable)
template <typename F>
std::vector<int> order_by(int q, F key) {
    std::vector<int> o(q);
    for (int i = 0; i < q; ++i) o[i] = i;
    std::stable_sort(o.begin(), o.end(), [&](int x, int y) { return key(x) < key(y); });
    return o;
}

// Columns of W (q x q) in the order o
Mat permute_columns(const Mat& W, int q, const std::vector<int>& o) {
    Mat out((size_t)q * q);
    for (int j = 0; j < q; ++j)
        for (int i = 0; i < q; ++i) out[i + (size_t)j * q] = W[i + (size_t)o[j] * q];
    return out;
}

// One subspace iteration run on A(R.mu) from a seeded start block: m eigenpairs
// with eigenvalues ascending in |theta|, unit right eigenvectors in the first m
// vectors of R.d.Y, residuals in res.
int solve(Run& R, bool hermitian, int m, int degree, int max_iter, double tol, double bound, unsigned long long seed,
          std::vector<cd>& theta, std::vector<double>& res, int& it, std::string& err) {
    const int p = R.p;
    const size_t n = R.n;
    Dev& d = R.d;
    theta.assign(m, 0.0);
    res.assign(m, INFINITY);
    it = 0;
    {   // seeded Gaussian start block
        std::mt19937_64 rng(seed);
        std::normal_distribution<double> nd;
        std::vector<double2> h(n * p);
        for (auto& v : h) v = mk(nd(rng), nd(rng));
        if (hipMemcpy(d.X, h.data(), sizeof(double2) * n * p, hipMemcpyHostToDevice) != hipSuccess) {
            err = "eigensolver: copy";
            return NKS_E_HIP;
        }
    }
    double a = bound / 10.0, a0 = 0.0;
    Mat H, W;
    while (it < max_iter) {
        if (it > 0 && !R.filter(degree, a, bound, a0)) { err = "eigensolver: filter launch"; return NKS_E_HIP; }
        ++it;
        int rc = R.orthonormalise(err);
        if (rc != NKS_OK) return rc;
        // order the block by |theta^2| (Rayleigh-Ritz on A^2); T = A X after this step
        std::vector<double> t2(p);
        R.apply(d.X, d.T, p);
        if (hermitian) {
            if (!R.gram(d.T, d.T, p, H)) { err = "eigensolver: gram"; return NKS_E_HIP; }
            dense::symmetrise(H, p);
            std::vector<double> w;
            dense::jacobi(H, p, w, W);
            const std::vector<int> o = order_by(p, [&](int i) { return w[i]; });
            for (int j = 0; j < p; ++j) t2[j] = w[o[j]];
            const Mat Wo = permute_columns(W, p, o);
            if (!R.rotate(d.X, Wo, d.Y, p, p) || !R.rotate(d.T, Wo, d.U, p, p)) { err = "eigensolver: rotate"; return NKS_E_HIP; }
            std::swap(d.X, d.Y);
            std::swap(d.T, d.U);
        } else {
            R.apply(d.T, d.U, p);   // A^2 X
            if (!R.gram(d.X, d.U, p, H)) { err = "eigensolver: gram"; return NKS_E_HIP; }
            std::vector<cd> lam;
            if (!dense::eig_general(H, p, lam, W)) { err = "eigensolver: QR of the Ritz matrix of A^2"; return NKS_E_NOCONV; }
            const std::vector<int> o = order_by(p, [&](int i) { return std::abs(lam[i]); });
            for (int j = 0; j < p; ++j) t2[j] = std::abs(lam[o[j]]);
            if (!R.rotate(d.X, permute_columns(W, p, o), d.Y, p, p)) { err = "eigensolver: rotate"; return NKS_E_HIP; }
            std::swap(d.X, d.Y);
            rc = R.orthonormalise(err);
            if (rc != NKS_OK) return rc;
            R.apply(d.X, d.T, m);
        }
        // next filter interval: damp [largest |theta^2| of the block, b]
        a = std::min(t2[p - 1], bound / 2.0);
        a0 = std::max(t2[0], 0.0);
        // Rayleigh-Ritz on A within the first m vectors: eigenpairs into Y, A Y into U
        if (!R.gram(d.X, d.T, m, H)) { err = "eigensolver: gram"; return NKS_E_HIP; }
        std::vector<cd> lam(m);
        if (hermitian) {
            dense::symmetrise(H, m);
            std::vector<double> w;
            dense::jacobi(H, m, w, W);
            for (int i = 0; i < m; ++i) lam[i] = w[i];
        } else if (!dense::eig_general(H, m, lam, W)) {
            err = "eigensolver: QR of the Ritz matrix of A";
            return NKS_E_NOCONV;
        }
        const std::vector<int> o = order_by(m, [&](int i) { return std::abs(lam[i]); });
        std::vector<double2> th(m);
        for (int j = 0; j < m; ++j) {
            theta[j] = lam[o[j]];
            th[j] = mk(theta[j].real(), theta[j].imag());
        }
        const Mat Wm = permute_columns(W, m, o);
        if (!R.rotate(d.X, Wm, d.Y, m, m) || !R.rotate(d.T, Wm, d.U, m, m)) { err = "eigensolver: rotate"; return NKS_E_HIP; }
        if (hipMemcpy(d.theta, th.data(), sizeof(double2) * m, hipMemcpyHostToDevice) != hipSuccess) {
            err = "eigensolver: copy";
            return NKS_E_HIP;
        }
        hipLaunchKernelGGL(eig_resid, dim3(R.nchunk, m), dim3(GNT), 0, nullptr, d.U, d.Y, d.theta, n, R.nchunk, d.part);
        hipLaunchKernelGGL(eig_sum, dim3(m), dim3(GNT), 0, nullptr, d.part, R.nchunk, m, d.small);
        std::vector<double2> hr(m);
        if (hipMemcpy(hr.data(), d.small, sizeof(double2) * m, hipMemcpyDeviceToHost) != hipSuccess) {
            err = "eigensolver: copy";
            return NKS_E_HIP;
        }
        double worst = 0.0;
        for (int i = 0; i < m; ++i) {
            res[i] = std::sqrt(hr[i].x);
            worst = std::max(worst, res[i]);
        }
        if (worst <= tol) return NKS_OK;
    }
    err = "eigensolver: residual above tol after max_iter iterations";
    return NKS_E_NOCONV;
}

}  // namespace

int eig_chfsi(const Geom& g, const double2* links, double kappa, double mu, int m, int p, int degree, int max_iter,
              double tol, unsigned long long seed, double2* rvecs_out, double2* lvecs_out, double* lambda_out,
              double* resid_out, int* iters_out, std::string& err) {
    Run R;
    R.g = g;
    R.links = links;
    R.kappa = kappa;
    R.mu = mu;
    R.n = (size_t)12 * g.V;
    R.nb = (g.V + ENT - 1) / ENT;
    R.nchunk = (int)std::min<size_t>(64, (R.n + 4095) / 4096);
    R.p = p;
    Dev& d = R.d;
    const size_t n = R.n, blk = sizeof(double2) * n * p;
    if (hipMalloc(&d.X, blk) || hipMalloc(&d.Y, blk) || hipMalloc(&d.T, blk) || hipMalloc(&d.U, blk) ||
        hipMalloc(&d.part, sizeof(double2) * (size_t)p * p * R.nchunk) ||
        hipMalloc(&d.small, sizeof(double2) * p * p) || hipMalloc(&d.theta, sizeof(double2) * p)) {
        err = "eigensolver: device allocation failed";
        return NKS_E_NOMEM;
    }
    const double na = norm_bound(kappa, mu);     // ||A||, so ||A^2|| <= na^2
    const double bound = na * na;
    const bool hermitian = mu == 0.0;
    std::vector<cd> th;
    std::vector<double> res;
    int it = 0;
    int rc = solve(R, hermitian, m, degree, max_iter, tol, bound, seed, th, res, it, err);
    if (iters_out) *iters_out = it;
    auto report = [&](const std::vector<double>& r) {
        for (int i = 0; i < m; ++i) {
            if (lambda_out) {
                lambda_out[2 * i] = th[i].real();
                lambda_out[2 * i + 1] = th[i].imag();
            }
            if (resid_out) resid_out[i] = r[i];
        }
    };
    report(res);
    if (rc != NKS_OK) return rc;
    if (hipMemcpy(rvecs_out, d.Y, sizeof(double2) * n * m, hipMemcpyDeviceToDevice) != hipSuccess) {
        err = "eigensolver: copy out";
        return NKS_E_HIP;
    }
    if (hermitian) {
        if (hipMemcpy(lvecs_out, d.Y, sizeof(double2) * n * m, hipMemcpyDeviceToDevice) != hipSuccess) {
            err = "eigensolver: copy out";
            return NKS_E_HIP;
        }
        return NKS_OK;
    }
    // left eigenvectors: the right eigenvectors of A(-mu) = A^dagger, eigenvalues conj(lambda)
    R.mu = -mu;
    std::vector<cd> thl;
    std::vector<double> resl;
    int itl = 0;
    rc = solve(R, false, m, degree, max_iter, tol, bound, seed + 1, thl, resl, itl, err);
    if (iters_out) *iters_out = it + itl;
    for (int i = 0; i < m; ++i) resl[i] = std::max(res[i], resl[i]);
    report(resl);
    if (rc != NKS_OK) return rc;
    // pair l_j with r_i where conj(theta_l_j) = theta_i, then l_i = l_j / conj(l_j^H r_i)
    Mat C;   // C(j, i) = l_j^H r_i
    if (!R.gram(d.Y, rvecs_out, m, C)) { err = "eigensolver: gram"; return NKS_E_HIP; }
    Mat Z((size_t)m * m, 0.0);
    std::vector<bool> used(m, false);
    for (int i = 0; i < m; ++i) {
        int best = -1;
        double bd = INFINITY;
        for (int j = 0; j < m; ++j) {
            const double dd = std::abs(std::conj(thl[j]) - th[i]);
            if (!used[j] && dd < bd) {
                bd = dd;
                best = j;
            }
        }
        if (best < 0 || bd > 1e-6 * std::max(1.0, std::abs(th[i]))) {
            err = "eigensolver: the left and right eigenvalues do not pair up (tie at the m-th |lambda|?)";
            return NKS_E_NOCONV;
        }
        used[best] = true;
        const cd s = C[best + (size_t)i * m];
        if (!(std::abs(s) > 0.0)) {
            err = "eigensolver: l^dagger r = 0 for a computed pair";
            return NKS_E_NOCONV;
        }
        Z[best + (size_t)i * m] = 1.0 / std::conj(s);
    }
    if (!R.rotate(d.Y, Z, lvecs_out, m, m)) { err = "eigensolver: rotate"; return NKS_E_HIP; }
    return NKS_OK;
}

}  // namespace nks
