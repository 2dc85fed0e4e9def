// Deflation eigenpairs of the Hermitian A = gamma5 D_w(0) (App. C step 1
// needs the eigenpairs of A with the smallest |lambda|; the paper takes them
// from a separate eigensolver).  Chebyshev-filtered subspace iteration on a
// block of p vectors:
//
//   filter    X <- T_d(A^2) X, a Chebyshev polynomial of degree d in A^2 that
//             damps [a, b] (a = the largest squared Ritz value of the block,
//             b = (1 + 8 sqrt(2) kappa)^2 >= ||A||^2) and grows below a;
//   orthonormalise  X <- X R^{-1} twice, R from the Cholesky factor of X^H X;
//   Rayleigh-Ritz on A^2   (AX)^H (AX) = W diag(theta^2) W^H, X <- X W: the
//             squared Ritz values are extremal, so none of them is spurious
//             (Rayleigh-Ritz on the indefinite A itself makes spurious
//             values near 0 from mixtures of +lambda and -lambda modes);
//   eigenpairs  Rayleigh-Ritz on A within the m vectors of the smallest
//             squared Ritz values, and the residuals |A x - theta x|.
//
// The stencil, the filter recurrence, the Gram matrices X^H Y and the basis
// rotations X Z run on the GPU; the p x p Cholesky and Jacobi steps (p <= 128)
// run on the host in double precision.  Vectors are SoA blocks
// [vector][comp = 3 spin + colour][site] of complex128.
#include <algorithm>
#include <cmath>
#include <complex>
#include <random>
#include <string>
#include <vector>

#include "wilson.h"

namespace nks {

namespace {

constexpr int ENT = 128;   // threads per block of the site-parallel kernels
constexpr int GNT = 256;   // threads per block of the reductions

// out_v = alpha (A in_v) + beta y_v + gamma z_v for v = blockIdx.y (y, z may be null)
__global__ __launch_bounds__(ENT) void eig_apply(Geom g, const double2* __restrict__ links, double kappa,
                                                 const double2* __restrict__ in, double2* __restrict__ out,
                                                 double alpha, const double2* __restrict__ y, double beta,
                                                 const double2* __restrict__ z, double gamma) {
    const int site = blockIdx.x * ENT + threadIdx.x;
    if (site >= g.V) return;
    const size_t n = (size_t)12 * g.V;
    const size_t off = (size_t)blockIdx.y * n;
    double cf[1][4], cb[1][4];
    hop_coefs<double>(kappa, 0.0, cf[0], cb[0]);
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

// part[(i p + j) nchunk + chunk] = sum over the chunk of conj(X_i) Y_j
__global__ __launch_bounds__(GNT) void eig_gram(const double2* __restrict__ X, const double2* __restrict__ Y,
                                                int p, size_t n, int nchunk, double2* __restrict__ part) {
    __shared__ double2 lds[GNT / 64];
    const int chunk = blockIdx.x, i = blockIdx.y, j = blockIdx.z;
    const size_t len = (n + nchunk - 1) / nchunk;
    const size_t lo = (size_t)chunk * len, hi = (lo + len < n) ? lo + len : n;
    const double2* xi = X + (size_t)i * n;
    const double2* yj = Y + (size_t)j * n;
    double2 s = mk(0.0, 0.0);
    for (size_t e = lo + threadIdx.x; e < hi; e += GNT) s = cadd(s, cmulc(xi[e], yj[e]));
    s = block_sum<GNT>(s, lds);
    if (threadIdx.x == 0) part[((size_t)i * p + j) * nchunk + chunk] = s;
}

// out[q] = sum_c part[q nchunk + c] for q < count (fixed order)
__global__ __launch_bounds__(GNT) void eig_sum(const double2* __restrict__ part, int nchunk, int count,
                                               double2* __restrict__ out) {
    __shared__ double2 lds[GNT / 64];
    const int q = blockIdx.x;
    if (q >= count) return;
    double2 s = mk(0.0, 0.0);
    for (int c = threadIdx.x; c < nchunk; c += GNT) s = cadd(s, part[(size_t)q * nchunk + c]);
    s = block_sum<GNT>(s, lds);
    if (threadIdx.x == 0) out[q] = s;
}

// out_v = sum_u X_u Z(u, v) (Z column-major, p x p); 8 outputs per thread
constexpr int ROT = 8;
__global__ __launch_bounds__(GNT) void eig_rotate(const double2* __restrict__ X, const double2* __restrict__ Z,
                                                  double2* __restrict__ out, int p, size_t n) {
    const size_t e = (size_t)blockIdx.x * GNT + threadIdx.x;
    if (e >= n) return;
    const int v0 = blockIdx.y * ROT;
    double2 acc[ROT];
#pragma unroll
    for (int k = 0; k < ROT; ++k) acc[k] = mk(0.0, 0.0);
    for (int u = 0; u < p; ++u) {
        const double2 x = X[(size_t)u * n + e];
#pragma unroll
        for (int k = 0; k < ROT; ++k)
            if (v0 + k < p) acc[k] = cadd(acc[k], cmul(x, Z[(size_t)(v0 + k) * p + u]));
    }
#pragma unroll
    for (int k = 0; k < ROT; ++k)
        if (v0 + k < p) out[(size_t)(v0 + k) * n + e] = acc[k];
}

// part[v nchunk + chunk] = sum over the chunk of |AX_v - theta_v X_v|^2 (in .x)
__global__ __launch_bounds__(GNT) void eig_resid(const double2* __restrict__ AX, const double2* __restrict__ X,
                                                 const double* __restrict__ theta, size_t n, int nchunk,
                                                 double2* __restrict__ part) {
    __shared__ double2 lds[GNT / 64];
    const int chunk = blockIdx.x, v = blockIdx.y;
    const size_t len = (n + nchunk - 1) / nchunk;
    const size_t lo = (size_t)chunk * len, hi = (lo + len < n) ? lo + len : n;
    const double t = theta[v];
    double s = 0.0;
    for (size_t e = lo + threadIdx.x; e < hi; e += GNT) s += cabs2(csub(AX[(size_t)v * n + e], cscale(X[(size_t)v * n + e], t)));
    const double2 r = block_sum<GNT>(mk(s, 0.0), lds);
    if (threadIdx.x == 0) part[(size_t)v * nchunk + chunk] = r;
}

using cd = std::complex<double>;

// Lower Cholesky factor of the Hermitian positive definite G (p x p, column-major); false if not PD.
bool cholesky(std::vector<cd>& G, int p) {
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

// Z = L^{-H} (upper triangular), L lower triangular, both column-major p x p
std::vector<cd> inverse_adjoint(const std::vector<cd>& L, int p) {
    // solve L^H Z = I column by column (back substitution)
    std::vector<cd> Z((size_t)p * p, 0.0);
    for (int c = 0; c < p; ++c) {
        for (int i = p - 1; i >= 0; --i) {
            cd s = (i == c) ? 1.0 : 0.0;
            for (int k = i + 1; k < p; ++k) s -= std::conj(L[k + (size_t)i * p]) * Z[k + (size_t)c * p];
            Z[i + (size_t)c * p] = s / std::conj(L[i + (size_t)i * p]);
        }
    }
    return Z;
}

// Cyclic Jacobi for the Hermitian H (p x p, column-major, overwritten): H = W diag(w) W^H.
void jacobi(std::vector<cd>& H, int p, std::vector<double>& w, std::vector<cd>& W) {
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
                // phase e^{i phi} = g / |g| makes the 2x2 block real: then a real rotation
                const cd ph = g / ag;
                const double a = at(k, k).real(), b = at(l, l).real();
                const double tau = (b - a) / (2.0 * ag);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                // U = [[c, s ph], [-s conj(ph), c]] in the (k, l) plane; H <- U^H H U, W <- W U
                for (int i = 0; i < p; ++i) {   // columns
                    const cd hik = at(i, k), hil = at(i, l);
                    at(i, k) = c * hik - s * std::conj(ph) * hil;
                    at(i, l) = s * ph * hik + c * hil;
                }
                for (int j = 0; j < p; ++j) {   // rows
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

struct Dev {
    double2 *X = nullptr, *Y = nullptr, *T = nullptr, *U = nullptr, *part = nullptr, *small = nullptr;
    double* theta = nullptr;
    ~Dev() {
        for (void* q : {(void*)X, (void*)Y, (void*)T, (void*)U, (void*)part, (void*)small, (void*)theta})
            if (q) (void)hipFree(q);
    }
};

}  // namespace

// (H + H^H) / 2 in place (rounding of a Hermitian Gram matrix)
static void symmetrise(std::vector<cd>& H, int p) {
    for (int j = 0; j < p; ++j)
        for (int i = 0; i < j; ++i) {
            const cd v = 0.5 * (H[i + (size_t)j * p] + std::conj(H[j + (size_t)i * p]));
            H[i + (size_t)j * p] = v;
            H[j + (size_t)i * p] = std::conj(v);
        }
    for (int i = 0; i < p; ++i) H[i + (size_t)i * p] = H[i + (size_t)i * p].real();
}

// Gram matrix out = X^H Y of the first p vectors (column-major on the host: out[i + j p] = X_i^H Y_j)
static int gram(const double2* X, const double2* Y, int p, size_t n, Dev& d, int nchunk, std::vector<cd>& out) {
    hipLaunchKernelGGL(eig_gram, dim3(nchunk, p, p), dim3(GNT), 0, nullptr, X, Y, p, n, nchunk, d.part);
    hipLaunchKernelGGL(eig_sum, dim3(p * p), dim3(GNT), 0, nullptr, d.part, nchunk, p * p, d.small);
    std::vector<double2> h((size_t)p * p);
    if (hipMemcpy(h.data(), d.small, sizeof(double2) * p * p, hipMemcpyDeviceToHost) != hipSuccess) return 1;
    out.resize((size_t)p * p);
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) out[i + (size_t)j * p] = cd(h[(size_t)i * p + j].x, h[(size_t)i * p + j].y);
    return 0;
}

static int rotate(const double2* X, const std::vector<cd>& Z, double2* out, int p, size_t n, Dev& d) {
    std::vector<double2> h((size_t)p * p);
    for (size_t q = 0; q < h.size(); ++q) h[q] = mk(Z[q].real(), Z[q].imag());
    if (hipMemcpy(d.small, h.data(), sizeof(double2) * p * p, hipMemcpyHostToDevice) != hipSuccess) return 1;
    hipLaunchKernelGGL(eig_rotate, dim3((unsigned)((n + GNT - 1) / GNT), (p + ROT - 1) / ROT), dim3(GNT), 0, nullptr, X,
                       d.small, out, p, n);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

int eig_chfsi(const Geom& g, const double2* links, double kappa, int m, int p, int degree, int max_iter, double tol,
              unsigned long long seed, double2* vecs_out, double* lambda_out, double* resid_out, int* iters_out,
              std::string& err) {
    const size_t n = (size_t)12 * g.V;
    const int nb = (g.V + ENT - 1) / ENT;
    const int nchunk = (int)std::min<size_t>(64, (n + 4095) / 4096);
    Dev d;
    const size_t blk = sizeof(double2) * n * p;
    if (hipMalloc(&d.X, blk) || hipMalloc(&d.Y, blk) || hipMalloc(&d.T, blk) || hipMalloc(&d.U, blk) ||
        hipMalloc(&d.part, sizeof(double2) * (size_t)p * p * nchunk) || hipMalloc(&d.small, sizeof(double2) * p * p) ||
        hipMalloc(&d.theta, sizeof(double) * p)) {
        err = "eigensolver: device allocation failed";
        return NKS_E_NOMEM;
    }
    {   // seeded Gaussian start block
        std::mt19937_64 rng(seed);
        std::normal_distribution<double> nd;
        std::vector<double2> h(n * p);
        for (auto& v : h) v = mk(nd(rng), nd(rng));
        if (hipMemcpy(d.X, h.data(), blk, hipMemcpyHostToDevice) != hipSuccess) { err = "eigensolver: copy"; return NKS_E_HIP; }
    }
    // ||A|| <= 1 + 8 sqrt(2) kappa: per direction the two hops map into the
    // complementary ranges of (1 + gamma)/2 and (1 - gamma)/2, so their sum has norm <= 2 sqrt(2)
    const double bound = (1.0 + 8.0 * std::sqrt(2.0) * kappa) * (1.0 + 8.0 * std::sqrt(2.0) * kappa);
    double a = bound / 10.0, a0 = 0.0;
    std::vector<double> theta(m, 0.0), res(m, INFINITY);
    std::vector<cd> G, H, Hm, W;
    int it = 0;
    for (; it < max_iter; ++it) {
        if (it > 0) {
            // Chebyshev filter of degree `degree` in A^2 on [a, b], scaled to 1 near a0
            const double e = (bound - a) / 2.0, c = (bound + a) / 2.0;
            double sigma = e / (a0 - c);
            const double tau = 2.0 / sigma;
            // Y = (A^2 X - c X) sigma / e
            hipLaunchKernelGGL(eig_apply, dim3(nb, p), dim3(ENT), 0, nullptr, g, links, kappa, d.X, d.T, 1.0,
                               (const double2*)nullptr, 0.0, (const double2*)nullptr, 0.0);
            hipLaunchKernelGGL(eig_apply, dim3(nb, p), dim3(ENT), 0, nullptr, g, links, kappa, d.T, d.Y, sigma / e,
                               (const double2*)d.X, -c * sigma / e, (const double2*)nullptr, 0.0);
            double2 *Xp = d.X, *Yc = d.Y, *Yn = d.U;
            for (int i = 2; i <= degree; ++i) {
                const double sigma2 = 1.0 / (tau - sigma);
                hipLaunchKernelGGL(eig_apply, dim3(nb, p), dim3(ENT), 0, nullptr, g, links, kappa, Yc, d.T, 1.0,
                                   (const double2*)nullptr, 0.0, (const double2*)nullptr, 0.0);
                hipLaunchKernelGGL(eig_apply, dim3(nb, p), dim3(ENT), 0, nullptr, g, links, kappa, d.T, Yn,
                                   2.0 * sigma2 / e, (const double2*)Yc, -2.0 * c * sigma2 / e, (const double2*)Xp,
                                   -sigma * sigma2);
                double2* t = Xp;
                Xp = Yc;
                Yc = Yn;
                Yn = t;
                sigma = sigma2;
            }
            if (Yc != d.X) {
                // the filtered block becomes X (buffers keep their roles by swapping pointers)
                double2* old_x = d.X;
                d.X = Yc;
                if (d.Y == Yc) d.Y = old_x;
                else if (d.U == Yc) d.U = old_x;
            }
            if (hipGetLastError() != hipSuccess) { err = "eigensolver: filter launch"; return NKS_E_HIP; }
        }
        // orthonormalise twice: X <- X L^{-H} with G = X^H X = L L^H
        for (int pass = 0; pass < 2; ++pass) {
            if (gram(d.X, d.X, p, n, d, nchunk, G)) { err = "eigensolver: gram"; return NKS_E_HIP; }
            if (!cholesky(G, p)) { err = "eigensolver: block lost rank (Cholesky of X^H X failed)"; return NKS_E_NOCONV; }
            if (rotate(d.X, inverse_adjoint(G, p), d.Y, p, n, d)) { err = "eigensolver: rotate"; return NKS_E_HIP; }
            std::swap(d.X, d.Y);
        }
        // Rayleigh-Ritz on A^2 (extremal, no spurious interior values): H2 = (AX)^H (AX)
        hipLaunchKernelGGL(eig_apply, dim3(nb, p), dim3(ENT), 0, nullptr, g, links, kappa, d.X, d.T, 1.0,
                           (const double2*)nullptr, 0.0, (const double2*)nullptr, 0.0);
        if (gram(d.T, d.T, p, n, d, nchunk, H)) { err = "eigensolver: gram"; return NKS_E_HIP; }
        symmetrise(H, p);
        std::vector<double> w2;
        jacobi(H, p, w2, W);
        std::vector<int> ord(p);
        for (int i = 0; i < p; ++i) ord[i] = i;
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return w2[x] < w2[y]; });
        std::vector<cd> Wo((size_t)p * p);
        for (int j = 0; j < p; ++j)
            for (int i = 0; i < p; ++i) Wo[i + (size_t)j * p] = W[i + (size_t)ord[j] * p];
        if (rotate(d.X, Wo, d.Y, p, n, d) || rotate(d.T, Wo, d.U, p, n, d)) { err = "eigensolver: rotate"; return NKS_E_HIP; }
        std::swap(d.X, d.Y);
        std::swap(d.T, d.U);
        // next filter interval: damp [largest squared Ritz value of the block, b]
        a = std::min(w2[ord[p - 1]], bound / 2.0);
        a0 = std::max(w2[ord[0]], 0.0);
        // Rayleigh-Ritz on A within the m vectors of the smallest squared Ritz
        // values: the eigenpairs and their residuals (into Y, U: m vectors)
        if (gram(d.X, d.T, m, n, d, nchunk, Hm)) { err = "eigensolver: gram"; return NKS_E_HIP; }
        symmetrise(Hm, m);
        std::vector<double> wa;
        jacobi(Hm, m, wa, W);
        std::vector<int> om(m);
        for (int i = 0; i < m; ++i) om[i] = i;
        std::stable_sort(om.begin(), om.end(), [&](int x, int y) { return std::fabs(wa[x]) < std::fabs(wa[y]); });
        std::vector<cd> Wm((size_t)m * m);
        theta.resize(m);
        for (int j = 0; j < m; ++j) {
            theta[j] = wa[om[j]];
            for (int i = 0; i < m; ++i) Wm[i + (size_t)j * m] = W[i + (size_t)om[j] * m];
        }
        if (rotate(d.X, Wm, d.Y, m, n, d) || rotate(d.T, Wm, d.U, m, n, d)) { err = "eigensolver: rotate"; return NKS_E_HIP; }
        if (hipMemcpy(d.theta, theta.data(), sizeof(double) * m, hipMemcpyHostToDevice) != hipSuccess) { err = "copy"; return NKS_E_HIP; }
        hipLaunchKernelGGL(eig_resid, dim3(nchunk, m), dim3(GNT), 0, nullptr, d.U, d.Y, d.theta, n, nchunk, d.part);
        hipLaunchKernelGGL(eig_sum, dim3(m), dim3(GNT), 0, nullptr, d.part, nchunk, m, d.small);
        std::vector<double2> hr(m);
        if (hipMemcpy(hr.data(), d.small, sizeof(double2) * m, hipMemcpyDeviceToHost) != hipSuccess) { err = "copy"; return NKS_E_HIP; }
        double worst = 0.0;
        for (int i = 0; i < m; ++i) {
            res[i] = std::sqrt(hr[i].x);
            worst = std::max(worst, res[i]);
        }
        if (worst <= tol) { ++it; break; }
    }
    if (iters_out) *iters_out = it;
    for (int i = 0; i < m; ++i) {
        if (lambda_out) lambda_out[i] = theta[i];
        if (resid_out) resid_out[i] = res[i];
    }
    if (hipMemcpy(vecs_out, d.Y, sizeof(double2) * n * m, hipMemcpyDeviceToDevice) != hipSuccess) {
        err = "eigensolver: copy out";
        return NKS_E_HIP;
    }
    double worst = 0.0;
    for (int i = 0; i < m; ++i) worst = std::max(worst, res[i]);
    if (!(worst <= tol)) {
        err = "eigensolver: residual above tol after max_iter iterations";
        return NKS_E_NOCONV;
    }
    return NKS_OK;
}

}  // namespace nks
