// Nested step of the method (Sec. 4.1, App. C steps 3-5) on the device,
// one workgroup per job:
//
//   3. p (given, or p_opt = (z_min z_max)^{-1/2} of Eq. popt from estimated
//      Ritz-value extremes of H_k) and the LU of p H_k with row interchanges,
//      exactly as LAPACK ?gttrf builds it;
//   4. ell steps of Lanczos (mu = 0, real arithmetic) or two-sided Lanczos on
//      H_k' = (p H_k + (p H_k)^{-1}) / 2 from e_1: (p H_k)^{-1} v by the LU
//      back substitution (?gttrs, trans 'C' for the adjoint) plus the
//      tridiagonal product p H_k v;
//   5. Roberts-Higham iteration S <- (S + S^{-1}) / 2 (Eq. Roberts) on the
//      dense ell x ell Ritz matrix, inverses by Gauss-Jordan with partial
//      pivoting;
//   then c = V_ell sgn(H_ell) e_1 and the lift weights omega_j = |b| c_j sv_j.
//
// With ell >= k_used the RHi runs on H_k itself (non-nested method).
#include "nks_internal.h"

#include <hip/hip_ext.h>

namespace nks {

namespace {

constexpr int NT = NEST_NT;
constexpr double RHI_NEAR = 1e-8;          // one more step once the change is below this
constexpr double LUCKY_TAU_HERMITIAN = 1e-10;
constexpr double LUCKY_TAU_TWO_SIDED = 1e-8;
constexpr double SERIOUS_TAU = 1e-12;
constexpr int ELL0 = 16;                   // first inner size of ell-doubling
constexpr int HOT_BYTES = 96 * 1024;       // LDS for the k-length arrays of the nested step

// ---- scalar helpers for T = double (real) or double2 (complex)
__device__ inline double s_mul(double a, double b) { return a * b; }
__device__ inline double2 s_mul(double2 a, double2 b) { return cmul(a, b); }
__device__ inline double s_add(double a, double b) { return a + b; }
__device__ inline double2 s_add(double2 a, double2 b) { return cadd(a, b); }
__device__ inline double s_sub(double a, double b) { return a - b; }
__device__ inline double2 s_sub(double2 a, double2 b) { return csub(a, b); }
__device__ inline double s_div(double a, double b) { return a / b; }
__device__ inline double2 s_div(double2 a, double2 b) { return cdiv(a, b); }
__device__ inline double s_conj(double a) { return a; }
__device__ inline double2 s_conj(double2 a) { return cconj(a); }
__device__ inline double s_abs1(double a) { return fabs(a); }                 // LAPACK cabs1
__device__ inline double s_abs1(double2 a) { return fabs(a.x) + fabs(a.y); }
__device__ inline double s_abs(double a) { return fabs(a); }
__device__ inline double s_abs(double2 a) { return cabs(a); }
__device__ inline double s_abs2(double a) { return a * a; }
__device__ inline double s_abs2(double2 a) { return cabs2(a); }
__device__ inline double s_scale(double a, double s) { return a * s; }
__device__ inline double2 s_scale(double2 a, double s) { return cscale(a, s); }
__device__ inline double2 s_d2(double a) { return mk(a, 0.0); }
__device__ inline double2 s_d2(double2 a) { return a; }
template <typename T> __device__ inline T s_from(double2 a);
template <> __device__ inline double s_from<double>(double2 a) { return a.x; }
template <> __device__ inline double2 s_from<double2>(double2 a) { return a; }
template <typename T> __device__ inline T s_zero() { return s_from<T>(mk(0.0, 0.0)); }
template <typename T> __device__ inline T s_one() { return s_from<T>(mk(1.0, 0.0)); }
// conj(a) * b
__device__ inline double s_dotterm(double a, double b) { return a * b; }
__device__ inline double2 s_dotterm(double2 a, double2 b) { return cmulc(a, b); }
__device__ inline double2 s_sqrt(double2 z) { return csqrt_principal(z); }

// ---- block reductions of doubles
__device__ inline double block_max(double v, double* lds) {
    for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = lds[0];
    for (int w = 1; w < NT / 64; ++w) r = fmax(r, lds[w]);
    return r;
}
__device__ inline double block_min(double v, double* lds) {
    return -block_max(-v, lds);
}
// argmax of v with the smallest index on ties; returns the index
__device__ inline int block_argmax(double v, int idx, double* ldsv, int* ldsi) {
    for (int m = 32; m >= 1; m >>= 1) {
        double ov = __shfl_xor(v, m, 64);
        int oi = __shfl_xor(idx, m, 64);
        if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) { ldsv[threadIdx.x >> 6] = v; ldsi[threadIdx.x >> 6] = idx; }
    __syncthreads();
    double bv = ldsv[0];
    int bi = ldsi[0];
    for (int w = 1; w < NT / 64; ++w)
        if (ldsv[w] > bv || (ldsv[w] == bv && ldsi[w] < bi)) { bv = ldsv[w]; bi = ldsi[w]; }
    return bi;
}

template <typename T>
__device__ inline T block_dot(const T* a, const T* b, int n, double2* lds) {   // sum conj(a) b
    double2 s = mk(0.0, 0.0);
    for (int i = threadIdx.x; i < n; i += NT) s = cadd(s, s_d2(s_dotterm(a[i], b[i])));
    return s_from<T>(block_sum<NT>(s, lds));
}
template <typename T>
__device__ inline double block_norm2(const T* a, int n, double2* lds) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) s += s_abs2(a[i]);
    return block_sum<NT>(mk(s, 0.0), lds).x;
}

// ---- LAPACK-style tridiagonal LU with partial pivoting (serial, one thread)
// dl: multipliers (n-1), d: U diagonal (n), du: first super-diagonal (n-1),
// du2: second super-diagonal (n-2), ipiv: 0-based pivot rows.  Returns info.
// The running d[i] and du[i] are carried in registers, so no step waits on
// reading back what the previous one stored.
template <typename T>
__device__ int gttrf(int n, T* __restrict__ dl, T* __restrict__ d, T* __restrict__ du, T* __restrict__ du2,
                     int* __restrict__ ipiv) {
    for (int i = 0; i < n; ++i) ipiv[i] = i;
    for (int i = 0; i + 2 < n; ++i) du2[i] = s_zero<T>();
    T dc = d[0];                                   // d[i] as updated by the steps before i
    T uc = (n > 1) ? du[0] : s_zero<T>();          // du[i] likewise
    for (int i = 0; i + 1 < n; ++i) {
        const T l = dl[i];
        T dn = d[i + 1];                           // d[i+1] and du[i+1] are still the input values
        const T un = (i + 2 < n) ? du[i + 1] : s_zero<T>();
        T un_next = un;
        if (s_abs1(dc) >= s_abs1(l)) {
            if (s_abs1(dc) != 0.0) {
                const T fact = s_div(l, dc);
                dl[i] = fact;
                dn = s_sub(dn, s_mul(fact, uc));
            }
            d[i] = dc;
            du[i] = uc;
        } else {                                   // interchange rows i and i+1
            const T fact = s_div(dc, l);
            d[i] = l;
            dl[i] = fact;
            du[i] = dn;
            dn = s_sub(uc, s_mul(fact, dn));
            if (i + 2 < n) {
                du2[i] = un;
                un_next = s_scale(s_mul(fact, un), -1.0);
            }
            ipiv[i] = i + 1;
        }
        dc = dn;
        uc = un_next;
    }
    d[n - 1] = dc;
    for (int i = 0; i < n; ++i)
        if (s_abs1(d[i]) == 0.0) return i + 1;
    return 0;
}

// ---- block-parallel solves with the LU factors of gttrf
//
// Every sweep of ?gttrs is a linear recurrence: the row interchanges of L
// make the forward (and the L^H backward) sweep a first-order recurrence
// c -> a c + b with |a| <= ~1, and U (U^H) with two super-diagonals is a
// second-order one, s -> M s + g on s = (x_i, x_{i+1}).  Each thread composes
// the affine maps of a contiguous chunk of steps, a Hillis-Steele scan over
// the block gives every chunk its incoming state, and each thread replays
// its chunk.  The arithmetic per step is the one of the serial sweep; only
// the association of the chunk products differs.
template <typename T> struct Aff1 { T a, b; };                   // c -> a c + b
template <typename T> struct Aff2 { T m00, m01, m10, m11, g0, g1; };   // s -> M s + g

template <typename T> __device__ inline Aff1<T> ident1() { return {s_one<T>(), s_zero<T>()}; }
template <typename T> __device__ inline Aff2<T> ident2() {
    return {s_one<T>(), s_zero<T>(), s_zero<T>(), s_one<T>(), s_zero<T>(), s_zero<T>()};
}
// later o earlier
template <typename T> __device__ inline Aff1<T> compose(const Aff1<T>& l, const Aff1<T>& e) {
    return {s_mul(l.a, e.a), s_add(s_mul(l.a, e.b), l.b)};
}
template <typename T> __device__ inline Aff2<T> compose(const Aff2<T>& l, const Aff2<T>& e) {
    Aff2<T> r;
    r.m00 = s_add(s_mul(l.m00, e.m00), s_mul(l.m01, e.m10));
    r.m01 = s_add(s_mul(l.m00, e.m01), s_mul(l.m01, e.m11));
    r.m10 = s_add(s_mul(l.m10, e.m00), s_mul(l.m11, e.m10));
    r.m11 = s_add(s_mul(l.m10, e.m01), s_mul(l.m11, e.m11));
    r.g0 = s_add(s_add(s_mul(l.m00, e.g0), s_mul(l.m01, e.g1)), l.g0);
    r.g1 = s_add(s_add(s_mul(l.m10, e.g0), s_mul(l.m11, e.g1)), l.g1);
    return r;
}

// Lane shuffles of the scalar types and of the affine maps
__device__ inline double shfl_s(double v, int src) { return __shfl(v, src, 64); }
__device__ inline double2 shfl_s(double2 v, int src) { return mk(__shfl(v.x, src, 64), __shfl(v.y, src, 64)); }
template <typename T> __device__ inline Aff1<T> shfl_map(const Aff1<T>& x, int src) {
    return {shfl_s(x.a, src), shfl_s(x.b, src)};
}
template <typename T> __device__ inline Aff2<T> shfl_map(const Aff2<T>& x, int src) {
    return {shfl_s(x.m00, src), shfl_s(x.m01, src), shfl_s(x.m10, src),
            shfl_s(x.m11, src), shfl_s(x.g0, src), shfl_s(x.g1, src)};
}

// Exclusive scan over scan positions 0..NT-1 (position pos composes after
// positions < pos); pos is tid (rev = false) or NT-1-tid (rev = true).
// Returns the composition of all maps at positions < pos.  Within a
// wavefront a Hillis-Steele scan over lane shuffles, then every wavefront
// composes the totals of the wavefronts before it (two barriers in all).
template <typename Map>
__device__ Map block_exclusive_scan(Map x, bool rev, Map* lds, Map id) {
    const int lane = threadIdx.x & 63;
    const int r = rev ? 63 - lane : lane;                           // rank in position order
    const int wv = rev ? (NT / 64 - 1 - (int)(threadIdx.x >> 6)) : (int)(threadIdx.x >> 6);
    for (int off = 1; off < 64; off <<= 1) {
        const int src = rev ? min(lane + off, 63) : max(lane - off, 0);
        const Map y = shfl_map(x, src);
        if (r >= off) x = compose(x, y);
    }
    if (r == 63) lds[wv] = x;                                        // wavefront total
    const Map in = shfl_map(x, rev ? min(lane + 1, 63) : max(lane - 1, 0));
    __syncthreads();
    Map pre = id;
    for (int w = 0; w < wv; ++w) pre = compose(lds[w], pre);
    __syncthreads();
    return (r == 0) ? pre : compose(in, pre);
}

struct LUF {   // LU factors of p H_k (gttrf layout) in the nest area
    const void *dl, *d, *du, *du2;
    const int* ipiv;
};

// x = (L U)^{-1} P b   (LAPACK trans 'N');  b, t, x distinct; all threads
template <typename T>
__device__ void solve_n(const LUF& F, int n, const T* b, T* t, T* x, void* scan_lds) {
    const T* dl = (const T*)F.dl;
    const T* d = (const T*)F.d;
    const T* du = (const T*)F.du;
    const T* du2 = (const T*)F.du2;
    const int tid = threadIdx.x;
    const int steps = n - 1;
    const int m = (steps + NT - 1) / NT;
    const int i0 = tid * m, i1 = min(steps, i0 + m);
    // forward sweep with interchanges: carry c_i = current b[i]
    {
        Aff1<T> f = ident1<T>();
        for (int i = i0; i < i1; ++i) {
            const T e = b[i + 1];
            Aff1<T> st = (F.ipiv[i] == i) ? Aff1<T>{s_scale(dl[i], -1.0), e}
                                          : Aff1<T>{s_one<T>(), s_scale(s_mul(dl[i], e), -1.0)};
            f = compose(st, f);
        }
        Aff1<T> ex = block_exclusive_scan<Aff1<T>>(f, false, (Aff1<T>*)scan_lds, ident1<T>());
        T c = s_add(s_mul(ex.a, b[0]), ex.b);
        for (int i = i0; i < i1; ++i) {
            const T e = b[i + 1];
            if (F.ipiv[i] == i) { t[i] = c; c = s_sub(e, s_mul(dl[i], c)); }
            else { t[i] = e; c = s_sub(c, s_mul(dl[i], e)); }
        }
        if (steps == 0 && tid == 0) t[0] = b[0];
        else if (i1 == steps && i0 < i1) t[steps] = c;
    }
    __syncthreads();
    // backward sweep with U: s_i = (x_i, x_{i+1}) = M_i s_{i+1} + g_i, i = n-2 .. 0
    {
        Aff2<T> f = ident2<T>();
        for (int i = i1 - 1; i >= i0; --i) {
            const T inv = s_div(s_one<T>(), d[i]);
            Aff2<T> st{s_scale(s_mul(du[i], inv), -1.0),
                       (i + 2 < n) ? s_scale(s_mul(du2[i], inv), -1.0) : s_zero<T>(),
                       s_one<T>(), s_zero<T>(), s_mul(t[i], inv), s_zero<T>()};
            f = compose(st, f);
        }
        Aff2<T> ex = block_exclusive_scan<Aff2<T>>(f, true, (Aff2<T>*)scan_lds, ident2<T>());
        const T xl = s_div(t[n - 1], d[n - 1]);
        T s0 = s_add(s_mul(ex.m00, xl), ex.g0);
        T s1 = s_add(s_mul(ex.m10, xl), ex.g1);
        for (int i = i1 - 1; i >= i0; --i) {
            const T inv = s_div(s_one<T>(), d[i]);
            const T dd2 = (i + 2 < n) ? du2[i] : s_zero<T>();
            const T xi = s_mul(s_sub(s_sub(t[i], s_mul(du[i], s0)), s_mul(dd2, s1)), inv);
            s1 = s0;
            s0 = xi;
            x[i] = xi;
        }
        if (tid == 0) x[n - 1] = xl;
    }
    __syncthreads();
}

// x = ((L U)^H)^{-1} b   (LAPACK trans 'C');  b, t, x distinct; all threads
template <typename T>
__device__ void solve_c(const LUF& F, int n, const T* b, T* t, T* x, void* scan_lds) {
    const T* dl = (const T*)F.dl;
    const T* d = (const T*)F.d;
    const T* du = (const T*)F.du;
    const T* du2 = (const T*)F.du2;
    const int tid = threadIdx.x;
    const int steps = n - 1;
    const int m = (steps + NT - 1) / NT;
    const int i0 = 1 + tid * m, i1 = min(n, i0 + m);   // rows 1..n-1
    // forward sweep with U^H: s_i = (x_i, x_{i-1}) = N_i s_{i-1} + h_i
    {
        Aff2<T> f = ident2<T>();
        for (int i = i0; i < i1; ++i) {
            const T inv = s_div(s_one<T>(), s_conj(d[i]));
            Aff2<T> st{s_scale(s_mul(s_conj(du[i - 1]), inv), -1.0),
                       (i >= 2) ? s_scale(s_mul(s_conj(du2[i - 2]), inv), -1.0) : s_zero<T>(),
                       s_one<T>(), s_zero<T>(), s_mul(b[i], inv), s_zero<T>()};
            f = compose(st, f);
        }
        Aff2<T> ex = block_exclusive_scan<Aff2<T>>(f, false, (Aff2<T>*)scan_lds, ident2<T>());
        const T x0 = s_div(b[0], s_conj(d[0]));
        T s0 = s_add(s_mul(ex.m00, x0), ex.g0);
        T s1 = s_add(s_mul(ex.m10, x0), ex.g1);
        for (int i = i0; i < i1; ++i) {
            const T inv = s_div(s_one<T>(), s_conj(d[i]));
            const T c2 = (i >= 2) ? s_conj(du2[i - 2]) : s_zero<T>();
            const T xi = s_mul(s_sub(s_sub(b[i], s_mul(s_conj(du[i - 1]), s0)), s_mul(c2, s1)), inv);
            s1 = s0;
            s0 = xi;
            t[i] = xi;
        }
        if (tid == 0) t[0] = x0;
    }
    __syncthreads();
    // backward sweep with L^H and the interchanges: carry c, steps i = n-2 .. 0
    {
        const int j0 = tid * m, j1 = min(steps, j0 + m);   // steps j0..j1-1, run descending
        Aff1<T> f = ident1<T>();
        for (int i = j1 - 1; i >= j0; --i) {
            Aff1<T> st = (F.ipiv[i] == i) ? Aff1<T>{s_scale(s_conj(dl[i]), -1.0), t[i]}
                                          : Aff1<T>{s_one<T>(), s_zero<T>()};
            f = compose(st, f);
        }
        Aff1<T> ex = block_exclusive_scan<Aff1<T>>(f, true, (Aff1<T>*)scan_lds, ident1<T>());
        T c = s_add(s_mul(ex.a, t[n - 1]), ex.b);
        for (int i = j1 - 1; i >= j0; --i) {
            if (F.ipiv[i] == i) { x[i + 1] = c; c = s_sub(t[i], s_mul(s_conj(dl[i]), c)); }
            else { x[i + 1] = s_sub(t[i], s_mul(s_conj(dl[i]), c)); }
        }
        if (steps == 0) { if (tid == 0) x[0] = t[0]; }
        else if (j0 == 0 && j0 < j1) x[0] = c;
    }
    __syncthreads();
}

// ---- two independent solves in one pass: their scans share the shuffle
// rounds and barriers; each component keeps the association of its own solve,
// so the results are those of two separate calls
template <typename A, typename B> struct MPair { A a; B b; };
template <typename A, typename B>
__device__ inline MPair<A, B> compose(const MPair<A, B>& l, const MPair<A, B>& e) {
    return {compose(l.a, e.a), compose(l.b, e.b)};
}
template <typename A, typename B> __device__ inline MPair<A, B> shfl_map(const MPair<A, B>& x, int src) {
    return {shfl_map(x.a, src), shfl_map(x.b, src)};
}

// x1 = (L U)^{-1} P b1 and x2 = (L U)^{-1} P b2 (trans 'N' twice); t1 != t2; all threads
template <typename T>
__device__ void solve_nn(const LUF& F, int n, const T* b1, T* t1, T* x1, const T* b2, T* t2, T* x2,
                         void* scan_lds) {
    const T* dl = (const T*)F.dl;
    const T* d = (const T*)F.d;
    const T* du = (const T*)F.du;
    const T* du2 = (const T*)F.du2;
    const int tid = threadIdx.x;
    const int steps = n - 1;
    const int m = (steps + NT - 1) / NT;
    const int i0 = tid * m, i1 = min(steps, i0 + m);
    {
        MPair<Aff1<T>, Aff1<T>> f{ident1<T>(), ident1<T>()};
        for (int i = i0; i < i1; ++i) {
            const bool keep = F.ipiv[i] == i;
            const T e1 = b1[i + 1], e2 = b2[i + 1];
            const Aff1<T> s1 = keep ? Aff1<T>{s_scale(dl[i], -1.0), e1} : Aff1<T>{s_one<T>(), s_scale(s_mul(dl[i], e1), -1.0)};
            const Aff1<T> s2 = keep ? Aff1<T>{s_scale(dl[i], -1.0), e2} : Aff1<T>{s_one<T>(), s_scale(s_mul(dl[i], e2), -1.0)};
            f.a = compose(s1, f.a);
            f.b = compose(s2, f.b);
        }
        const MPair<Aff1<T>, Aff1<T>> ex = block_exclusive_scan<MPair<Aff1<T>, Aff1<T>>>(
            f, false, (MPair<Aff1<T>, Aff1<T>>*)scan_lds, {ident1<T>(), ident1<T>()});
        T c1 = s_add(s_mul(ex.a.a, b1[0]), ex.a.b);
        T c2 = s_add(s_mul(ex.b.a, b2[0]), ex.b.b);
        for (int i = i0; i < i1; ++i) {
            const T e1 = b1[i + 1], e2 = b2[i + 1];
            if (F.ipiv[i] == i) {
                t1[i] = c1; c1 = s_sub(e1, s_mul(dl[i], c1));
                t2[i] = c2; c2 = s_sub(e2, s_mul(dl[i], c2));
            } else {
                t1[i] = e1; c1 = s_sub(c1, s_mul(dl[i], e1));
                t2[i] = e2; c2 = s_sub(c2, s_mul(dl[i], e2));
            }
        }
        if (steps == 0 && tid == 0) { t1[0] = b1[0]; t2[0] = b2[0]; }
        else if (i1 == steps && i0 < i1) { t1[steps] = c1; t2[steps] = c2; }
    }
    __syncthreads();
    {
        MPair<Aff2<T>, Aff2<T>> f{ident2<T>(), ident2<T>()};
        for (int i = i1 - 1; i >= i0; --i) {
            const T inv = s_div(s_one<T>(), d[i]);
            const T a0 = s_scale(s_mul(du[i], inv), -1.0);
            const T a1 = (i + 2 < n) ? s_scale(s_mul(du2[i], inv), -1.0) : s_zero<T>();
            const Aff2<T> s1{a0, a1, s_one<T>(), s_zero<T>(), s_mul(t1[i], inv), s_zero<T>()};
            const Aff2<T> s2{a0, a1, s_one<T>(), s_zero<T>(), s_mul(t2[i], inv), s_zero<T>()};
            f.a = compose(s1, f.a);
            f.b = compose(s2, f.b);
        }
        const MPair<Aff2<T>, Aff2<T>> ex = block_exclusive_scan<MPair<Aff2<T>, Aff2<T>>>(
            f, true, (MPair<Aff2<T>, Aff2<T>>*)scan_lds, {ident2<T>(), ident2<T>()});
        const T xl1 = s_div(t1[n - 1], d[n - 1]), xl2 = s_div(t2[n - 1], d[n - 1]);
        T p0 = s_add(s_mul(ex.a.m00, xl1), ex.a.g0), p1 = s_add(s_mul(ex.a.m10, xl1), ex.a.g1);
        T q0 = s_add(s_mul(ex.b.m00, xl2), ex.b.g0), q1 = s_add(s_mul(ex.b.m10, xl2), ex.b.g1);
        for (int i = i1 - 1; i >= i0; --i) {
            const T inv = s_div(s_one<T>(), d[i]);
            const T dd2 = (i + 2 < n) ? du2[i] : s_zero<T>();
            const T y1 = s_mul(s_sub(s_sub(t1[i], s_mul(du[i], p0)), s_mul(dd2, p1)), inv);
            const T y2 = s_mul(s_sub(s_sub(t2[i], s_mul(du[i], q0)), s_mul(dd2, q1)), inv);
            p1 = p0; p0 = y1; x1[i] = y1;
            q1 = q0; q0 = y2; x2[i] = y2;
        }
        if (tid == 0) { x1[n - 1] = xl1; x2[n - 1] = xl2; }
    }
    __syncthreads();
}

// xn = (L U)^{-1} P bn (trans 'N') and xc = ((L U)^H)^{-1} bc (trans 'C'); tn != tc; all threads
template <typename T>
__device__ void solve_nc(const LUF& F, int n, const T* bn, T* tn, T* xn, const T* bc, T* tc, T* xc,
                         void* scan_lds) {
    const T* dl = (const T*)F.dl;
    const T* d = (const T*)F.d;
    const T* du = (const T*)F.du;
    const T* du2 = (const T*)F.du2;
    const int tid = threadIdx.x;
    const int steps = n - 1;
    const int m = (steps + NT - 1) / NT;
    const int i0 = tid * m, i1 = min(steps, i0 + m);           // 'N' steps; 'C' backward steps too
    const int c0 = 1 + tid * m, c1 = min(n, c0 + m);            // 'C' forward rows
    // forward: L with interchanges ('N'), U^H ('C')
    {
        MPair<Aff1<T>, Aff2<T>> f{ident1<T>(), ident2<T>()};
        for (int i = i0; i < i1; ++i) {
            const T e = bn[i + 1];
            const Aff1<T> st = (F.ipiv[i] == i) ? Aff1<T>{s_scale(dl[i], -1.0), e}
                                                : Aff1<T>{s_one<T>(), s_scale(s_mul(dl[i], e), -1.0)};
            f.a = compose(st, f.a);
        }
        for (int i = c0; i < c1; ++i) {
            const T inv = s_div(s_one<T>(), s_conj(d[i]));
            const Aff2<T> st{s_scale(s_mul(s_conj(du[i - 1]), inv), -1.0),
                             (i >= 2) ? s_scale(s_mul(s_conj(du2[i - 2]), inv), -1.0) : s_zero<T>(),
                             s_one<T>(), s_zero<T>(), s_mul(bc[i], inv), s_zero<T>()};
            f.b = compose(st, f.b);
        }
        const MPair<Aff1<T>, Aff2<T>> ex = block_exclusive_scan<MPair<Aff1<T>, Aff2<T>>>(
            f, false, (MPair<Aff1<T>, Aff2<T>>*)scan_lds, {ident1<T>(), ident2<T>()});
        T c = s_add(s_mul(ex.a.a, bn[0]), ex.a.b);
        for (int i = i0; i < i1; ++i) {
            const T e = bn[i + 1];
            if (F.ipiv[i] == i) { tn[i] = c; c = s_sub(e, s_mul(dl[i], c)); }
            else { tn[i] = e; c = s_sub(c, s_mul(dl[i], e)); }
        }
        if (steps == 0 && tid == 0) tn[0] = bn[0];
        else if (i1 == steps && i0 < i1) tn[steps] = c;
        const T x0 = s_div(bc[0], s_conj(d[0]));
        T s0 = s_add(s_mul(ex.b.m00, x0), ex.b.g0);
        T s1 = s_add(s_mul(ex.b.m10, x0), ex.b.g1);
        for (int i = c0; i < c1; ++i) {
            const T inv = s_div(s_one<T>(), s_conj(d[i]));
            const T cc2 = (i >= 2) ? s_conj(du2[i - 2]) : s_zero<T>();
            const T xi = s_mul(s_sub(s_sub(bc[i], s_mul(s_conj(du[i - 1]), s0)), s_mul(cc2, s1)), inv);
            s1 = s0;
            s0 = xi;
            tc[i] = xi;
        }
        if (tid == 0) tc[0] = x0;
    }
    __syncthreads();
    // backward: U ('N'), L^H with interchanges ('C')
    {
        MPair<Aff2<T>, Aff1<T>> f{ident2<T>(), ident1<T>()};
        for (int i = i1 - 1; i >= i0; --i) {
            const T inv = s_div(s_one<T>(), d[i]);
            const Aff2<T> st{s_scale(s_mul(du[i], inv), -1.0),
                             (i + 2 < n) ? s_scale(s_mul(du2[i], inv), -1.0) : s_zero<T>(),
                             s_one<T>(), s_zero<T>(), s_mul(tn[i], inv), s_zero<T>()};
            f.a = compose(st, f.a);
        }
        for (int i = i1 - 1; i >= i0; --i) {
            const Aff1<T> st = (F.ipiv[i] == i) ? Aff1<T>{s_scale(s_conj(dl[i]), -1.0), tc[i]}
                                                : Aff1<T>{s_one<T>(), s_zero<T>()};
            f.b = compose(st, f.b);
        }
        const MPair<Aff2<T>, Aff1<T>> ex = block_exclusive_scan<MPair<Aff2<T>, Aff1<T>>>(
            f, true, (MPair<Aff2<T>, Aff1<T>>*)scan_lds, {ident2<T>(), ident1<T>()});
        const T xl = s_div(tn[n - 1], d[n - 1]);
        T s0 = s_add(s_mul(ex.a.m00, xl), ex.a.g0);
        T s1 = s_add(s_mul(ex.a.m10, xl), ex.a.g1);
        for (int i = i1 - 1; i >= i0; --i) {
            const T inv = s_div(s_one<T>(), d[i]);
            const T dd2 = (i + 2 < n) ? du2[i] : s_zero<T>();
            const T xi = s_mul(s_sub(s_sub(tn[i], s_mul(du[i], s0)), s_mul(dd2, s1)), inv);
            s1 = s0;
            s0 = xi;
            xn[i] = xi;
        }
        if (tid == 0) xn[n - 1] = xl;
        T c = s_add(s_mul(ex.b.a, tc[n - 1]), ex.b.b);
        for (int i = i1 - 1; i >= i0; --i) {
            if (F.ipiv[i] == i) { xc[i + 1] = c; c = s_sub(tc[i], s_mul(s_conj(dl[i]), c)); }
            else { xc[i + 1] = s_sub(tc[i], s_mul(s_conj(dl[i]), c)); }
        }
        if (steps == 0) { if (tid == 0) xc[0] = tc[0]; }
        else if (i0 == 0 && i0 < i1) xc[0] = c;
    }
    __syncthreads();
}

// ---- nest-area layout
struct NestPtrs {
    void *d, *sub, *sup;        // H_k diagonals (k)
    void *lf, *u0, *u1, *u2;    // LU factors (k each)
    int* piv;                   // k
    void* vl;                   // inner basis, L columns of k
    void *v, *vp, *w, *wp, *r, *l, *y, *t, *t2;   // work vectors (k)
    void *cc, *cp;              // current and previous coefficient vectors (k)
    void *al, *bl, *gl;         // H_ell (L)
    void *S, *B;                // dense L x L
    void *prow, *fcol;          // L
    int* perm;                  // L
};

__host__ __device__ inline size_t nest_words_impl(int k, int L) {
    // complex words (16 bytes); int arrays rounded up
    return (size_t)3 * k + 4 * (size_t)k + ((size_t)k + 3) / 4 + (size_t)k * L + 11 * (size_t)k + 3 * (size_t)L +
           2 * (size_t)L * L + 2 * (size_t)L + ((size_t)L + 3) / 4 + 8;
}

__device__ inline NestPtrs nest_ptrs(double2* base, int k, int L) {
    NestPtrs P;
    double2* q = base;
    auto take = [&](size_t n) { double2* r = q; q += n; return (void*)r; };
    P.d = take(k); P.sub = take(k); P.sup = take(k);
    P.lf = take(k); P.u0 = take(k); P.u1 = take(k); P.u2 = take(k);
    P.piv = (int*)take(((size_t)k + 3) / 4);
    P.vl = take((size_t)k * L);
    P.v = take(k); P.vp = take(k); P.w = take(k); P.wp = take(k); P.r = take(k); P.l = take(k); P.y = take(k);
    P.t = take(k); P.t2 = take(k); P.cc = take(k); P.cp = take(k);
    P.al = take(L); P.bl = take(L); P.gl = take(L);
    P.S = take((size_t)L * L); P.B = take((size_t)L * L);
    P.prow = take(L); P.fcol = take(L);
    P.perm = (int*)take(((size_t)L + 3) / 4);
    return P;
}

// y = 0.5 * ((pH)^{-1} v + p H v) (ADJ: with H^dagger); v, y length k; all threads
template <typename T, bool ADJ>
__device__ void apply_hprime(const NestPtrs& P, int k, double p, const T* v, T* y, void* scan_lds) {
    const T* d = (const T*)P.d;
    const T* sub = (const T*)P.sub;
    const T* sup = (const T*)P.sup;
    const LUF F{P.lf, P.u0, P.u1, P.u2, P.piv};
    if (!ADJ) solve_n<T>(F, k, v, (T*)P.t, y, scan_lds);
    else solve_c<T>(F, k, v, (T*)P.t, y, scan_lds);
    for (int i = threadIdx.x; i < k; i += NT) {
        T hv;
        if (!ADJ) {
            hv = s_mul(d[i], v[i]);
            if (i > 0) hv = s_add(hv, s_mul(sub[i - 1], v[i - 1]));
            if (i + 1 < k) hv = s_add(hv, s_mul(sup[i], v[i + 1]));
        } else {
            hv = s_mul(s_conj(d[i]), v[i]);
            if (i > 0) hv = s_add(hv, s_mul(s_conj(sup[i - 1]), v[i - 1]));
            if (i + 1 < k) hv = s_add(hv, s_mul(s_conj(sub[i]), v[i + 1]));
        }
        y[i] = s_scale(s_add(y[i], s_scale(hv, p)), 0.5);
    }
    __syncthreads();
}

// yv = H_k' v and yw = H_k'^dagger w with both solves in one pass (two-sided step)
template <typename T>
__device__ void apply_hprime2(const NestPtrs& P, int k, double p, const T* v, T* yv, const T* w, T* yw,
                              void* scan_lds) {
    const T* d = (const T*)P.d;
    const T* sub = (const T*)P.sub;
    const T* sup = (const T*)P.sup;
    const LUF F{P.lf, P.u0, P.u1, P.u2, P.piv};
    solve_nc<T>(F, k, v, (T*)P.t, yv, w, (T*)P.t2, yw, scan_lds);
    for (int i = threadIdx.x; i < k; i += NT) {
        T hv = s_mul(d[i], v[i]);
        if (i > 0) hv = s_add(hv, s_mul(sub[i - 1], v[i - 1]));
        if (i + 1 < k) hv = s_add(hv, s_mul(sup[i], v[i + 1]));
        yv[i] = s_scale(s_add(yv[i], s_scale(hv, p)), 0.5);
        T hw = s_mul(s_conj(d[i]), w[i]);
        if (i > 0) hw = s_add(hw, s_mul(s_conj(sup[i - 1]), w[i - 1]));
        if (i + 1 < k) hw = s_add(hw, s_mul(s_conj(sub[i]), w[i + 1]));
        yw[i] = s_scale(s_add(yw[i], s_scale(hw, p)), 0.5);
    }
    __syncthreads();
}

// Sturm count: number of eigenvalues < x of the real symmetric tridiagonal (d, e^2)
__device__ inline int sturm_count(const double* d, const double* sub, int k, double x, double pivmin) {
    int cnt = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
    for (int i = 1; i < k; ++i) {
        const double e = sub[i - 1];
        q = d[i] - x - e * e / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// Eigenvalues number ms[0..nt) (1-based, nt <= 8) of the symmetric
// tridiagonal by multisection of [-G, G]: one NT-point round shared by all
// targets, then the threads split into nt groups, each refining its own
// target's bracket, for as many rounds as bring every bracket below the
// resolution of four NT-point rounds, 2G / (NT+1)^4.  A bracket keeps the
// largest point with fewer than m eigenvalues below it and the smallest with
// at least m.  lds: NT ints and 16 doubles.  All threads; results in out.
__device__ void find_eigs(const double* d, const double* sub, int k, const int* ms, int nt, double G,
                          double pivmin, void* lds, double* out) {
    int* cnt = static_cast<int*>(lds);
    double* lo = reinterpret_cast<double*>(cnt + NT);
    double* hi = lo + 8;
    const int tid = threadIdx.x;
    cnt[tid] = sturm_count(d, sub, k, -G + 2.0 * G * (double)(tid + 1) / (double)(NT + 1), pivmin);
    __syncthreads();
    if (tid < nt) {
        double l = -G, h = G;
        for (int t = 0; t < NT; ++t) {
            const double xt = -G + 2.0 * G * (double)(t + 1) / (double)(NT + 1);
            if (cnt[t] < ms[tid]) l = fmax(l, xt);
            else h = fmin(h, xt);
        }
        lo[tid] = l;
        hi[tid] = h;
    }
    __syncthreads();
    const int per = NT / nt;
    int rounds = 0;
    for (double f = 1.0; f < (double)(NT + 1) * (NT + 1) * (NT + 1); f *= (double)(per + 1)) ++rounds;
    const int g = tid / per, j = tid - (tid / per) * per;
    for (int r = 0; r < rounds; ++r) {
        if (g < nt) cnt[tid] = sturm_count(d, sub, k, lo[g] + (hi[g] - lo[g]) * (double)(j + 1) / (double)(per + 1), pivmin);
        __syncthreads();
        if (tid < nt) {
            const double ol = lo[tid], oh = hi[tid];
            double l = ol, h = oh;
            for (int t = 0; t < per; ++t) {
                const double xt = ol + (oh - ol) * (double)(t + 1) / (double)(per + 1);
                if (cnt[tid * per + t] < ms[tid]) l = fmax(l, xt);
                else h = fmin(h, xt);
            }
            lo[tid] = l;
            hi[tid] = h;
        }
        __syncthreads();
    }
    for (int i = 0; i < nt; ++i) out[i] = 0.5 * (lo[i] + hi[i]);
    __syncthreads();
}

// Pivot search key: rows already used never win; every unused row is a
// candidate even when its entry is NaN (then it only wins if nothing else
// can), so the chosen pivot row is always a valid unused row and a NaN matrix
// fails the sweep (ok = false) instead of indexing row n.
__device__ inline double pivot_weight(int used_as, double a) {
    if (used_as >= 0) return -1.0;
    return (a >= 0.0) ? a : -0.5;
}

// In-place Gauss-Jordan inversion with partial pivoting and implicit row
// interchanges (the pivot rows are recorded, not moved).  After the sweep
// B[perm[k]][pinv[m]] = (A^{-1})[k][m], with perm[k] the pivot row of column
// k (global, n ints) and pinv its inverse (LDS, n ints).  fcol (LDS, n
// entries) holds the pivot column, prow (n entries) the scaled pivot row.
// Threads own columns, so row accesses are coalesced.  Returns false on a
// zero pivot.  Used when the blocked form's panel does not fit in LDS.
template <typename T>
__device__ bool gj_invert_unblocked(T* __restrict__ B, int n, T* __restrict__ prow, int* __restrict__ perm,
                                    T* __restrict__ fcol, int* __restrict__ pinv, double* ldsd, int* ldsi) {
    const int tid = threadIdx.x;
    const int nc = n < NT ? n : NT;          // columns per pass
    const int groups = NT / nc;              // threads per column
    const int g = tid / nc, jc = tid - (tid / nc) * nc;
    bool ok = true;
    for (int i = tid; i < n; i += NT) pinv[i] = -1;
    __syncthreads();
    for (int kk = 0; kk < n; ++kk) {
        double best = -1.0;
        int bidx = n;
        for (int i = tid; i < n; i += NT) {
            const T v = B[(size_t)i * n + kk];
            fcol[i] = v;
            const double a = pivot_weight(pinv[i], s_abs(v));
            if (a > best) { best = a; bidx = i; }
        }
        const int p = block_argmax(best, bidx, ldsd, ldsi);   // synchronises
        const T piv = fcol[p];
        if (!(s_abs1(piv) > 0.0) || !isfinite(s_abs1(piv))) ok = false;
        const T pivinv = s_div(s_one<T>(), piv);
        for (int j = tid; j < n; j += NT) prow[j] = (j == kk) ? pivinv : s_mul(B[(size_t)p * n + j], pivinv);
        __syncthreads();
        if (tid == 0) { perm[kk] = p; pinv[p] = kk; }
        if (g < groups) {
            for (int j = jc; j < n; j += nc) {
                const T pj = prow[j];
                T* col = B + j;
                for (int i = g; i < n; i += groups) {
                    T* e = col + (size_t)i * n;
                    if (i == p) *e = pj;
                    else *e = s_sub((j == kk) ? s_zero<T>() : *e, s_mul(fcol[i], pj));
                }
            }
        }
        __syncthreads();
    }
    return ok;
}

// Blocked form of the same sweep.  Columns are taken NB at a time: the panel
// B[:, k0:k0+nb] is eliminated in LDS (W), then the rest of B gets the
// panel's combined effect in one pass,
//   B[i][j] <- (i a pivot row of the panel ? 0 : B[i][j]) + sum_s W[i][s] R[s][j],
// where R[s] is pivot row perm[k0+s] before the pass.  Each element of B is
// read and written once per panel instead of once per column.
constexpr int GJ_NB = 8;                 // widest panel
constexpr int GJ_PANEL_BYTES = 32768;
constexpr int GJ_CH = 8;                 // rows per prefetched chunk

// Column j, rows i0, i0 + step, ... : the rank-nb update with the next chunk
// of B loaded before the current one is stored.
template <typename T, int NB>
__device__ inline void panel_update_column(T* __restrict__ B, int n, int j, int i0, int step, int k0, int nb,
                                           const T* __restrict__ W, const int* __restrict__ pinv, const T* R) {
    T* col = B + j;
    T cur[GJ_CH];
#pragma unroll
    for (int r = 0; r < GJ_CH; ++r) {
        const int i = i0 + r * step;
        cur[r] = i < n ? col[(size_t)i * n] : s_zero<T>();
    }
    for (int base = i0; base < n; base += GJ_CH * step) {
        T nxt[GJ_CH];
        const int nb0 = base + GJ_CH * step;
#pragma unroll
        for (int r = 0; r < GJ_CH; ++r) {
            const int i = nb0 + r * step;
            nxt[r] = i < n ? col[(size_t)i * n] : s_zero<T>();
        }
#pragma unroll
        for (int r = 0; r < GJ_CH; ++r) {
            const int i = base + r * step;
            if (i < n) {
                const int q = pinv[i];
                T acc = (q >= k0 && q < k0 + nb) ? s_zero<T>() : cur[r];
                const T* w = W + i * NB;
#pragma unroll
                for (int s2 = 0; s2 < NB; ++s2) acc = s_add(acc, s_mul(w[s2], R[s2]));
                col[(size_t)i * n] = acc;
            }
        }
#pragma unroll
        for (int r = 0; r < GJ_CH; ++r) cur[r] = nxt[r];
    }
}

template <typename T, int NB>
__device__ bool gj_invert_blocked(T* __restrict__ B, int n, int* __restrict__ perm, T* __restrict__ fcol,
                                  int* __restrict__ pinv, T* __restrict__ W, double* ldsd, int* ldsi) {
    const int tid = threadIdx.x;
    T* pr = fcol - GJ_NB;                    // scaled pivot row of the panel (kept just before fcol)
    bool ok = true;
    __shared__ int gj_ok;                    // a zero pivot seen by the single-wavefront panel
    if (tid == 0) gj_ok = 1;
    for (int i = tid; i < n; i += NT) pinv[i] = -1;
    __syncthreads();
    const int nc = n < NT ? n : NT;
    const int groups = NT / nc;
    const int g = tid / nc, jc = tid - (tid / nc) * nc;
    for (int k0 = 0; k0 < n; k0 += NB) {
        const int nb = min(NB, n - k0);
        for (int e = tid; e < n * NB; e += NT) {
            const int i = e / NB, sidx = e - i * NB;
            W[e] = sidx < nb ? B[(size_t)i * n + k0 + sidx] : s_zero<T>();
        }
        __syncthreads();
        if (n <= 64) {
            // n <= 64: the first wavefront eliminates the panel alone, one row per
            // lane held in registers; the pivot search and the pivot row travel
            // by lane shuffles (same pivots and operations, no barriers; the
            // complex products may be fused into FMAs differently)
            if (tid < 64) {
                const int i = tid;
                int used = (i < n) ? pinv[i] : 0;
                T w[NB];
#pragma unroll
                for (int s2 = 0; s2 < NB; ++s2) w[s2] = (i < n) ? W[i * NB + s2] : s_zero<T>();
#pragma unroll
                for (int t = 0; t < NB; ++t) {
                    if (t >= nb) break;
                    double best = -1.0;
                    int bidx = n;
                    if (i < n) {
                        const double a = pivot_weight(used, s_abs(w[t]));
                        if (a > best) { best = a; bidx = i; }
                    }
                    for (int m = 32; m >= 1; m >>= 1) {
                        const double ov = __shfl_xor(best, m, 64);
                        const int oi = __shfl_xor(bidx, m, 64);
                        if (ov > best || (ov == best && oi < bidx)) { best = ov; bidx = oi; }
                    }
                    const int p = bidx;   // an unused row exists, so p < n <= 64
                    T prv[NB];
#pragma unroll
                    for (int s2 = 0; s2 < NB; ++s2) prv[s2] = shfl_s(w[s2], p);
                    const T piv = prv[t];
                    if (!(s_abs1(piv) > 0.0) || !isfinite(s_abs1(piv))) ok = false;
                    const T pivinv = s_div(s_one<T>(), piv);
#pragma unroll
                    for (int s2 = 0; s2 < NB; ++s2) prv[s2] = (s2 == t) ? pivinv : s_mul(prv[s2], pivinv);
                    if (tid == 0) perm[k0 + t] = p;
                    if (i < n) {
                        if (i == p) {
                            used = k0 + t;
#pragma unroll
                            for (int s2 = 0; s2 < NB; ++s2) w[s2] = prv[s2];
                        } else {
                            const T f = w[t];
#pragma unroll
                            for (int s2 = 0; s2 < NB; ++s2) w[s2] = s_sub(s2 == t ? s_zero<T>() : w[s2], s_mul(f, prv[s2]));
                        }
                    }
                }
                if (i < n) {
                    pinv[i] = used;
#pragma unroll
                    for (int s2 = 0; s2 < NB; ++s2) W[i * NB + s2] = w[s2];
                }
                if (tid == 0 && !ok) gj_ok = 0;
            }
            __syncthreads();
        } else if (n <= NT) {
            // 64 < n <= NT: one row per thread, held in registers; per pivot the
            // wavefront maxima meet in LDS (the tie rule of block_argmax) and the
            // pivot row's owner publishes it: two barriers per pivot
            const int i = tid;
            int used = (i < n) ? pinv[i] : 0;
            T w[NB];
#pragma unroll
            for (int s2 = 0; s2 < NB; ++s2) w[s2] = (i < n) ? W[i * NB + s2] : s_zero<T>();
#pragma unroll
            for (int t = 0; t < NB; ++t) {
                if (t >= nb) break;
                double best = -1.0;
                int bidx = n;
                if (i < n) {
                    const double a = pivot_weight(used, s_abs(w[t]));
                    if (a > best) { best = a; bidx = i; }
                }
                for (int m = 32; m >= 1; m >>= 1) {
                    const double ov = __shfl_xor(best, m, 64);
                    const int oi = __shfl_xor(bidx, m, 64);
                    if (ov > best || (ov == best && oi < bidx)) { best = ov; bidx = oi; }
                }
                if ((tid & 63) == 0) { ldsd[tid >> 6] = best; ldsi[tid >> 6] = bidx; }
                __syncthreads();
                double bv = ldsd[0];
                int p = ldsi[0];
                for (int q = 1; q < NT / 64; ++q)
                    if (ldsd[q] > bv || (ldsd[q] == bv && ldsi[q] < p)) { bv = ldsd[q]; p = ldsi[q]; }
                if (i == p) {
#pragma unroll
                    for (int s2 = 0; s2 < NB; ++s2) pr[s2] = w[s2];
                }
                __syncthreads();
                T prv[NB];
#pragma unroll
                for (int s2 = 0; s2 < NB; ++s2) prv[s2] = pr[s2];
                const T piv = prv[t];
                if (!(s_abs1(piv) > 0.0) || !isfinite(s_abs1(piv))) ok = false;
                const T pivinv = s_div(s_one<T>(), piv);
#pragma unroll
                for (int s2 = 0; s2 < NB; ++s2) prv[s2] = (s2 == t) ? pivinv : s_mul(prv[s2], pivinv);
                if (tid == 0) perm[k0 + t] = p;
                if (i < n) {
                    if (i == p) {
                        used = k0 + t;
#pragma unroll
                        for (int s2 = 0; s2 < NB; ++s2) w[s2] = prv[s2];
                    } else {
                        const T f = w[t];
#pragma unroll
                        for (int s2 = 0; s2 < NB; ++s2) w[s2] = s_sub(s2 == t ? s_zero<T>() : w[s2], s_mul(f, prv[s2]));
                    }
                }
            }
            if (i < n) {
                pinv[i] = used;
#pragma unroll
                for (int s2 = 0; s2 < NB; ++s2) W[i * NB + s2] = w[s2];
            }
            __syncthreads();
        } else {
            // eliminate the panel in LDS
            for (int t = 0; t < nb; ++t) {
                double best = -1.0;
                int bidx = n;
                for (int i = tid; i < n; i += NT) {
                    const double a = pivot_weight(pinv[i], s_abs(W[i * NB + t]));
                    if (a > best) { best = a; bidx = i; }
                }
                const int p = block_argmax(best, bidx, ldsd, ldsi);   // synchronises
                const T piv = W[p * NB + t];
                if (!(s_abs1(piv) > 0.0) || !isfinite(s_abs1(piv))) ok = false;
                const T pivinv = s_div(s_one<T>(), piv);
                if (tid < NB) pr[tid] = (tid == t) ? pivinv : s_mul(W[p * NB + tid], pivinv);
                __syncthreads();
                if (tid == 0) { perm[k0 + t] = p; pinv[p] = k0 + t; }
                for (int i = tid; i < n; i += NT) {
                    T* w = W + i * NB;
                    if (i == p) {
    #pragma unroll
                        for (int s2 = 0; s2 < NB; ++s2) w[s2] = pr[s2];
                    } else {
                        const T f = w[t];
    #pragma unroll
                        for (int s2 = 0; s2 < NB; ++s2) w[s2] = s_sub(s2 == t ? s_zero<T>() : w[s2], s_mul(f, pr[s2]));
                    }
                }
                __syncthreads();
            }
        }
        // rank-nb update of the columns outside the panel
        if (groups > 1) {
            // one column per thread: read its pivot-row entries before any thread writes
            const int j = jc;
            const bool mine = g < groups && !(j >= k0 && j < k0 + nb);
            T R[NB];
#pragma unroll
            for (int s2 = 0; s2 < NB; ++s2)
                R[s2] = (s2 < nb && mine) ? B[(size_t)perm[k0 + s2] * n + j] : s_zero<T>();
            __syncthreads();
            if (mine) panel_update_column<T, NB>(B, n, j, g, groups, k0, nb, W, pinv, R);
        } else if (g == 0) {
            // each column has one owner thread, so it reads and updates the column alone
            for (int j = jc; j < n; j += nc) {
                if (j >= k0 && j < k0 + nb) continue;
                T R[NB];
#pragma unroll
                for (int s2 = 0; s2 < NB; ++s2) R[s2] = s2 < nb ? B[(size_t)perm[k0 + s2] * n + j] : s_zero<T>();
                panel_update_column<T, NB>(B, n, j, 0, 1, k0, nb, W, pinv, R);
            }
        }
        __syncthreads();
        // the panel columns take W
        for (int e = tid; e < n * nb; e += NT) {
            const int i = e / nb, sidx = e - i * nb;
            B[(size_t)i * n + k0 + sidx] = W[i * NB + sidx];
        }
        __syncthreads();
    }
    return ok && gj_ok != 0;
}

// The widest panel that fits in GJ_PANEL_BYTES of LDS.
template <typename T>
__device__ bool gj_invert(T* __restrict__ B, int n, T* __restrict__ prow, int* __restrict__ perm,
                          T* __restrict__ fcol, int* __restrict__ pinv, T* __restrict__ W, double* ldsd,
                          int* ldsi) {
    const size_t row = (size_t)n * sizeof(T);
    if (row * 8 <= (size_t)GJ_PANEL_BYTES) return gj_invert_blocked<T, 8>(B, n, perm, fcol, pinv, W, ldsd, ldsi);
    if (row * 4 <= (size_t)GJ_PANEL_BYTES) return gj_invert_blocked<T, 4>(B, n, perm, fcol, pinv, W, ldsd, ldsi);
    if (row * 2 <= (size_t)GJ_PANEL_BYTES) return gj_invert_blocked<T, 2>(B, n, perm, fcol, pinv, W, ldsd, ldsi);
    return gj_invert_unblocked<T>(B, n, prow, perm, fcol, pinv, ldsd, ldsi);
}

static_assert((RHI_MAX + GJ_NB) * sizeof(double2) + RHI_MAX * sizeof(int) <= NT * sizeof(Aff2<double2>),
              "the RHi pivot row, pivot column and permutation live in the scan LDS");

template <typename T>
__device__ int rhi(T* S, T* B, int n, int maxit, double tol, T* prow, int* perm, void* lds, void* panel,
                   double2* red, double* ldsd, int* ldsi) {
    if (n > RHI_MAX) return -1;
    T* fcol = (T*)lds + GJ_NB;              // the blocked sweep keeps its pivot row just before
    int* pinv = (int*)(fcol + n);
    bool last = false;
    for (int it = 1; it <= maxit; ++it) {
        for (int e = threadIdx.x; e < n * n; e += NT) B[e] = S[e];
        __syncthreads();
        const bool ok = gj_invert<T>(B, n, prow, perm, fcol, pinv, (T*)panel, ldsd, ldsi);
        if (!ok) return -it;
        double ch = 0.0, nm = 0.0;
        for (int k = 0; k < n; ++k) {
            const T* inv_row = B + (size_t)perm[k] * n;     // row k of S^{-1}, columns permuted
            T* srow = S + (size_t)k * n;
            for (int m = threadIdx.x; m < n; m += NT) {
                const T sn = s_scale(s_add(srow[m], inv_row[pinv[m]]), 0.5);
                ch += s_abs2(s_sub(sn, srow[m]));
                nm += s_abs2(sn);
                srow[m] = sn;
            }
        }
        const double2 r = block_sum<NT>(mk(ch, nm), red);
        const double change = sqrt(r.x) / sqrt(r.y);
        if (change <= tol || last) return it;
        if (change <= RHI_NEAR) last = true;
    }
    return -maxit;
}

struct Smem {
    double2* red;     // NT/64
    double* redd;     // NT/64
    int* redi;        // NT/64
    void* scan;       // NT affine maps
    void* panel;      // GJ_PANEL_BYTES: the Gauss-Jordan panel of RHi
    void* hot = nullptr;   // HOT_BYTES (null: the nest area stays in global memory)
};

// Every inner step is a chain of short phases (tridiagonal solves, products,
// reductions), each reading what the previous one wrote, and the LU is a
// serial sweep by one thread; from global memory each phase waits on L2
// latency.  The k-length arrays of the job's own level move to LDS, in this
// order, as many as fit: LU factors and pivots, solve and work vectors, then
// H_k itself.  Only the space used within one launch moves (c, the bases and
// the RHi matrices stay in the nest area), and the arithmetic is unchanged.
template <typename T>
__device__ void place_hot(NestPtrs& P, int k, const Smem& sm) {
    constexpr bool CPLX = sizeof(T) == sizeof(double2);
    if (!sm.hot) return;
    char* q = static_cast<char*>(sm.hot);
    size_t left = HOT_BYTES;
    const size_t vb = ((size_t)k * sizeof(T) + 15) & ~(size_t)15;
    const size_t ib = ((size_t)k * sizeof(int) + 15) & ~(size_t)15;
    auto take = [&](void*& a, size_t n) {
        if (n > left) return false;
        a = q;
        q += n;
        left -= n;
        return true;
    };
    void* piv = P.piv;
    if (!take(P.lf, vb) || !take(P.u0, vb) || !take(P.u1, vb) || !take(P.u2, vb) || !take(piv, ib)) return;
    P.piv = static_cast<int*>(piv);
    if (!take(P.t, vb) || !take(P.t2, vb) || !take(P.v, vb) || !take(P.r, vb) || !take(P.vp, vb)) return;
    if (CPLX && (!take(P.w, vb) || !take(P.l, vb) || !take(P.wp, vb))) return;
    if (!take(P.d, vb) || !take(P.sub, vb) || !take(P.sup, vb)) return;
}

// ---------------------------------------------------------------- step 3: p
// Estimated Ritz-value extremes of the tridiagonal in P.d/sub/sup (H_k, or
// the Ritz matrix of a deeper level).
template <typename T>
__device__ void estimate_extremes(const NestPtrs& P, int k, const Smem& sm, double& zmin, double& zmax) {
    constexpr bool CPLX = sizeof(T) == sizeof(double2);
    const int tid = threadIdx.x;
    const T* d = (const T*)P.d;
    const T* sub = (const T*)P.sub;
    const T* sup = (const T*)P.sup;
    if (!CPLX) {
        // Ritz values of the real symmetric matrix by Sturm multisection
        const double* dd = (const double*)P.d;
        const double* ee = (const double*)P.sub;
        double g = 0.0, emax = 0.0;
        for (int i = tid; i < k; i += NT) {
            const double el = (i > 0) ? fabs(ee[i - 1]) : 0.0;
            const double er = (i + 1 < k) ? fabs(ee[i]) : 0.0;
            g = fmax(g, fabs(dd[i]) + el + er);
            emax = fmax(emax, er);
        }
        const double G = block_max(g, sm.redd) * 1.001 + 1e-300;
        const double em = block_max(emax, sm.redd);
        const double pivmin = 2.2250738585072014e-308 * fmax(1.0, em * em);
        __shared__ int c0s;
        if (tid == 0) c0s = sturm_count(dd, ee, k, 0.0, pivmin);
        __syncthreads();
        const int c0 = c0s;
        __syncthreads();
        // the extremes and the Ritz values next to the origin (indices c0 - 1 .. c0 + 2)
        int ms[6], nt = 0;
        auto add = [&](int m) {
            if (m < 1 || m > k) return;
            for (int i = 0; i < nt; ++i)
                if (ms[i] == m) return;
            ms[nt++] = m;
        };
        add(1);
        add(k);
        for (int m = c0 - 1; m <= c0 + 2; ++m) add(m);
        double ev[6];
        find_eigs(dd, ee, k, ms, nt, G, pivmin, sm.scan, ev);
        auto eig = [&](int m) {
            for (int i = 0; i < nt; ++i)
                if (ms[i] == m) return ev[i];
            return 0.0;
        };
        const double l1 = eig(1), lk = eig(k);
        zmax = fmax(fabs(l1), fabs(lk));
        if (k == 1) { zmin = fabs(l1); return; }
        // z_min: the second smallest |theta|.  Between two Ritz values lies an
        // eigenvalue of A, so the gap of A around 0 holds at most one Ritz value,
        // which may sit anywhere in it; the second smallest lies outside.  The
        // two smallest |theta| are among the two largest negative and the two
        // smallest positive Ritz values (indices c0 - 1 .. c0 + 2).
        double z1 = INFINITY, z2 = INFINITY;
        for (int m = c0 - 1; m <= c0 + 2; ++m) {
            if (m < 1 || m > k) continue;
            const double a = fabs(eig(m));
            if (a < z1) { z2 = z1; z1 = a; }
            else if (a < z2) z2 = a;
        }
        zmin = z2;
        return;
    }
    // power iteration for z_max, inverse iteration (LU of H_k) for z_min; each
    // estimate is the geometric mean of the per-step growth over the second
    // half of the iterations, which damps the transient growth of a non-normal H_k
    constexpr int NIT = 48, NAVG = 24;
    T* x = (T*)P.v;
    T* y = (T*)P.w;
    T* lf = (T*)P.lf;
    T* u0 = (T*)P.u0;
    T* u1 = (T*)P.u1;
    T* u2 = (T*)P.u2;
    for (int i = tid; i < k; i += NT) x[i] = s_from<T>(mk(1.0 + 0.5 * (double)i / (double)k, 0.0));
    __syncthreads();
    double nx = sqrt(block_norm2<T>(x, k, sm.red));
    for (int i = tid; i < k; i += NT) x[i] = s_scale(x[i], 1.0 / nx);
    __syncthreads();
    double lsum = 0.0;
    for (int it = 0; it < NIT; ++it) {
        for (int i = tid; i < k; i += NT) {
            T hv = s_mul(d[i], x[i]);
            if (i > 0) hv = s_add(hv, s_mul(sub[i - 1], x[i - 1]));
            if (i + 1 < k) hv = s_add(hv, s_mul(sup[i], x[i + 1]));
            y[i] = hv;
        }
        __syncthreads();
        const double ny = sqrt(block_norm2<T>(y, k, sm.red));
        if (it >= NIT - NAVG) lsum += log(ny);
        for (int i = tid; i < k; i += NT) x[i] = s_scale(y[i], 1.0 / ny);
        __syncthreads();
    }
    zmax = exp(lsum / NAVG);
    for (int i = tid; i < k; i += NT) {
        u0[i] = d[i];
        if (i + 1 < k) { lf[i] = sub[i]; u1[i] = sup[i]; }
    }
    __syncthreads();
    __shared__ int info0;
    if (tid == 0) info0 = gttrf<T>(k, lf, u0, u1, u2, P.piv);
    __syncthreads();
    // z_min: the second smallest |theta| (a single Ritz value can stray near
    // the origin), by inverse subspace iteration on two vectors with
    // Gram-Schmidt: the diagonal of R grows like 1/|theta_1|, 1/|theta_2|
    T* x2 = (T*)P.vp;
    T* y2 = (T*)P.wp;
    for (int i = tid; i < k; i += NT) {
        x[i] = s_from<T>(mk(1.0 + 0.5 * (double)i / (double)k, 0.0));
        x2[i] = s_from<T>(mk((i & 1) ? -1.0 : 1.0, 0.25 * (double)(i % 3)));
    }
    __syncthreads();
    if (info0 == 0 && k >= 2) {
        const LUF F{P.lf, P.u0, P.u1, P.u2, P.piv};
        double l2sum = 0.0;
        // orthonormal start
        nx = sqrt(block_norm2<T>(x, k, sm.red));
        for (int i = tid; i < k; i += NT) x[i] = s_scale(x[i], 1.0 / nx);
        __syncthreads();
        {
            const T h = block_dot<T>(x, x2, k, sm.red);
            for (int i = tid; i < k; i += NT) x2[i] = s_sub(x2[i], s_mul(h, x[i]));
            __syncthreads();
            const double n2 = sqrt(block_norm2<T>(x2, k, sm.red));
            for (int i = tid; i < k; i += NT) x2[i] = s_scale(x2[i], 1.0 / n2);
            __syncthreads();
        }
        lsum = 0.0;
        for (int it = 0; it < NIT; ++it) {
            solve_nn<T>(F, k, x, (T*)P.t, y, x2, (T*)P.t2, y2, sm.scan);
            const double n1 = sqrt(block_norm2<T>(y, k, sm.red));
            for (int i = tid; i < k; i += NT) y[i] = s_scale(y[i], 1.0 / n1);
            __syncthreads();
            const T h = block_dot<T>(y, y2, k, sm.red);
            for (int i = tid; i < k; i += NT) y2[i] = s_sub(y2[i], s_mul(h, y[i]));
            __syncthreads();
            const double n2 = sqrt(block_norm2<T>(y2, k, sm.red));
            // (a second vector that vanished is left as it is: its log then
            // spoils only the z_min estimate, which p_opt checks)
            if (n2 > 0.0) for (int i = tid; i < k; i += NT) y2[i] = s_scale(y2[i], 1.0 / n2);
            __syncthreads();
            if (it >= NIT - NAVG) { lsum += log(n1); l2sum += log(n2); }
            T* sw_ = x; x = y; y = sw_;
            sw_ = x2; x2 = y2; y2 = sw_;
        }
        zmin = exp(-l2sum / NAVG);
    } else if (info0 == 0) {
        zmin = s_abs(d[0]);
    } else {
        zmin = zmax * 1e-3;
    }
    __syncthreads();
}

// LU of p H_k into the nest area; returns the ?gttrf info (0 = nonsingular)
template <typename T>
__device__ int lu_pH(const NestPtrs& P, int k, double p) {
    const T* d = (const T*)P.d;
    const T* sub = (const T*)P.sub;
    const T* sup = (const T*)P.sup;
    for (int i = threadIdx.x; i < k; i += NT) {
        ((T*)P.u0)[i] = s_scale(d[i], p);
        if (i + 1 < k) { ((T*)P.lf)[i] = s_scale(sub[i], p); ((T*)P.u1)[i] = s_scale(sup[i], p); }
    }
    __syncthreads();
    __shared__ int info;
    if (threadIdx.x == 0) info = gttrf<T>(k, (T*)P.lf, (T*)P.u0, (T*)P.u1, (T*)P.u2, P.piv);
    __syncthreads();
    const int r = info;
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------- step 4: inner Krylov space
// The inner (two-sided) Lanczos process on H_k' from e_1, resumable so that
// ell-doubling extends the same space instead of restarting it.
struct Inner {
    int i = 0;          // basis vectors built so far (H_i is i x i)
    bool ended = false; // lucky or serious breakdown: the space cannot grow
    bool serious = false;
    double vn = 1.0, wn = 1.0;
};

template <typename T>
__device__ void inner_init(const NestPtrs& P, int k, double p, Inner& st, const Smem& sm) {
    constexpr bool CPLX = sizeof(T) == sizeof(double2);
    T* v = (T*)P.v;
    T* vp = (T*)P.vp;
    T* w = (T*)P.w;
    T* wp = (T*)P.wp;
    for (int i = threadIdx.x; i < k; i += NT) {
        v[i] = (i == 0) ? s_one<T>() : s_zero<T>();
        vp[i] = s_zero<T>();
        if (CPLX) { w[i] = v[i]; wp[i] = s_zero<T>(); }
    }
    __syncthreads();
    if (CPLX) apply_hprime2<T>(P, k, p, v, (T*)P.r, w, (T*)P.l, sm.scan);
    else apply_hprime<T, false>(P, k, p, v, (T*)P.r, sm.scan);
    st = Inner{};
}

// Grow the inner space to m vectors (or until it breaks down).
template <typename T>
__device__ void inner_extend(const NestPtrs& P, int k, double p, int m, Inner& st, const Smem& sm) {
    constexpr bool CPLX = sizeof(T) == sizeof(double2);
    const int tid = threadIdx.x;
    T* v = (T*)P.v;
    T* vp = (T*)P.vp;
    T* w = (T*)P.w;
    T* wp = (T*)P.wp;
    T* r = (T*)P.r;
    T* l = (T*)P.l;
    T* al = (T*)P.al;
    T* bl = (T*)P.bl;
    T* gl = (T*)P.gl;
    T* vl = (T*)P.vl;
    while (st.i < m && !st.ended) {
        const int i = st.i;   // vectors so far; next vector is number i+1
        if (i > 0) {
            // finish step i: beta_i, gamma_i and v_{i+1}
            if (!CPLX) {
                const double a = s_d2(al[i - 1]).x;
                const double b = sqrt(block_norm2<T>(r, k, sm.red));
                const double bprev = (i >= 2) ? s_d2(bl[i - 2]).x : 0.0;
                if (b <= LUCKY_TAU_HERMITIAN * (fabs(a) + bprev)) { st.ended = true; break; }
                if (tid == 0) { bl[i - 1] = s_from<T>(mk(b, 0.0)); gl[i - 1] = bl[i - 1]; }
                for (int q = tid; q < k; q += NT) {
                    vp[q] = v[q];
                    v[q] = s_scale(r[q], 1.0 / b);
                }
                __syncthreads();
                apply_hprime<T, false>(P, k, p, v, r, sm.scan);
                for (int q = tid; q < k; q += NT) r[q] = s_sub(r[q], s_scale(vp[q], b));
                __syncthreads();
            } else {
                const double2 a = s_d2(al[i - 1]);
                const double2 delta = s_d2(block_dot<T>(r, l, k, sm.red));
                const double nr = sqrt(block_norm2<T>(r, k, sm.red));
                const double nl = sqrt(block_norm2<T>(l, k, sm.red));
                const double S_ = cabs(a) + ((i >= 2) ? sqrt(cabs(cmul(s_d2(bl[i - 2]), s_d2(gl[i - 2])))) : 0.0);
                if (nr <= LUCKY_TAU_TWO_SIDED * S_ * st.vn || nl <= LUCKY_TAU_TWO_SIDED * S_ * st.wn) {
                    st.ended = true;
                    break;
                }
                if (cabs(delta) <= SERIOUS_TAU * nr * nl) { st.ended = true; st.serious = true; break; }
                const double2 beta = csqrt_principal(delta);
                const double2 gamma = cdiv(cconj(delta), beta);
                if (tid == 0) { bl[i - 1] = s_from<T>(beta); gl[i - 1] = s_from<T>(gamma); }
                const double2 ib = crecip(beta), ig = crecip(cconj(gamma));
                for (int q = tid; q < k; q += NT) {
                    vp[q] = v[q];
                    wp[q] = w[q];
                    v[q] = s_mul(r[q], s_from<T>(ib));
                    w[q] = s_mul(l[q], s_from<T>(ig));
                }
                st.vn = nr / cabs(beta);
                st.wn = nl / cabs(gamma);
                __syncthreads();
                apply_hprime2<T>(P, k, p, v, r, w, l, sm.scan);
                for (int q = tid; q < k; q += NT) {
                    r[q] = s_sub(r[q], s_mul(s_from<T>(gamma), vp[q]));
                    l[q] = s_sub(l[q], s_mul(s_from<T>(cconj(beta)), wp[q]));
                }
                __syncthreads();
            }
        }
        // step i+1: store v_{i+1}, alpha_{i+1}, r -= alpha v (l -= conj(alpha) w)
        for (int q = tid; q < k; q += NT) vl[(size_t)i * k + q] = v[q];
        __syncthreads();
        if (!CPLX) {
            const double a = s_d2(block_dot<T>(v, r, k, sm.red)).x;
            if (tid == 0) al[i] = s_from<T>(mk(a, 0.0));
            for (int q = tid; q < k; q += NT) r[q] = s_sub(r[q], s_scale(v[q], a));
        } else {
            const double2 a = s_d2(block_dot<T>(w, r, k, sm.red));
            if (tid == 0) al[i] = s_from<T>(a);
            for (int q = tid; q < k; q += NT) {
                r[q] = s_sub(r[q], s_mul(s_from<T>(a), v[q]));
                l[q] = s_sub(l[q], s_mul(s_from<T>(cconj(a)), w[q]));
            }
        }
        __syncthreads();
        st.i = i + 1;
    }
    __syncthreads();
}

// ---------------------------------------------------------------- step 5: RHi and c
// c = V_m sgn(H_m) e_1 for the leading m x m inner Ritz matrix -> out (k).
// lds_b: the inner space will not grow again, so the LDS of the level's
// k-length arrays is free and holds the inverted matrix B, and S as well,
// when they fit.
template <typename T>
__device__ int inner_coeffs(const JobDesc& J, const NestPtrs& P, int k, int m, T* out, const Smem& sm,
                            bool lds_b = false) {
    const int tid = threadIdx.x;
    const size_t mm = (size_t)m * m;
    const bool b_lds = lds_b && sm.hot && mm * sizeof(T) <= (size_t)HOT_BYTES;
    const bool s_lds = b_lds && 2 * mm * sizeof(T) <= (size_t)HOT_BYTES;
    T* B = b_lds ? (T*)sm.hot : (T*)P.B;
    T* S = s_lds ? (T*)sm.hot + mm : (T*)P.S;
    const T* al = (const T*)P.al;
    const T* bl = (const T*)P.bl;
    const T* gl = (const T*)P.gl;
    const T* vl = (const T*)P.vl;
    T* s_e1 = (T*)P.y;
    for (int e = tid; e < m * m; e += NT) {
        const int i = e / m, j = e - i * m;
        T val = s_zero<T>();
        if (i == j) val = al[i];
        else if (i == j + 1) val = bl[j];
        else if (j == i + 1) val = gl[i];
        S[e] = val;
    }
    __syncthreads();
    const int it = rhi<T>(S, B, m, J.max_rhi, J.rhi_tol, (T*)P.prow, P.perm, sm.scan, sm.panel, sm.red, sm.redd, sm.redi);
    __syncthreads();
    for (int j = tid; j < m; j += NT) s_e1[j] = S[(size_t)j * m];
    __syncthreads();
    for (int q = tid; q < k; q += NT) {
        T acc = s_zero<T>();
        for (int j = 0; j < m; ++j) acc = s_add(acc, s_mul(vl[(size_t)j * k + q], s_e1[j]));
        out[q] = acc;
    }
    __syncthreads();
    return it;
}

// non-nested: c = sgn(H_k) e_1 by RHi on H_k itself -> out (k)
template <typename T>
__device__ int nonnested_coeffs(const JobDesc& J, const NestPtrs& P, int k, T* out, const Smem& sm) {
    const int tid = threadIdx.x;
    T* S = (T*)P.S;
    T* B = (T*)P.B;
    const T* d = (const T*)P.d;
    const T* sub = (const T*)P.sub;
    const T* sup = (const T*)P.sup;
    for (int e = tid; e < k * k; e += NT) {
        const int i = e / k, j = e - i * k;
        T v = s_zero<T>();
        if (i == j) v = d[i];
        else if (i == j + 1) v = sub[j];
        else if (j == i + 1) v = sup[i];
        S[e] = v;
    }
    __syncthreads();
    const int it = rhi<T>(S, B, k, J.max_rhi, J.rhi_tol, (T*)P.prow, P.perm, sm.scan, sm.panel, sm.red, sm.redd, sm.redi);
    __syncthreads();
    for (int i = tid; i < k; i += NT) out[i] = S[(size_t)i * k];
    __syncthreads();
    return it;
}

template <typename T>
__device__ double rel_change(const T* a, const T* b, int k, const Smem& sm) {   // |a - b| / |a|
    double dn = 0.0, an = 0.0;
    for (int i = threadIdx.x; i < k; i += NT) {
        dn += s_abs2(s_sub(a[i], b[i]));
        an += s_abs2(a[i]);
    }
    const double2 r = block_sum<NT>(mk(dn, an), sm.red);
    return sqrt(r.x) / sqrt(r.y);
}

struct NestResult {
    int ell = 0;        // inner size of the accepted result (0 = non-nested)
    int levels = 0;     // nested levels that ran (0 = non-nested)
    int rhi = 0;        // RHi iterations (negative: no convergence)
    int status = NKS_OK;
    double p = 0.0, zmin = 0.0, zmax = 0.0, inner_delta = 0.0;
};

// ---------------------------------------------------------------- multi-level nesting (Sec. 4.5)
// Words of the deeper levels' nest areas, after level 0's.  Level i >= 1
// holds a tridiagonal of at most cap_i (cap_1 = the level-1 capacity) and
// builds min(ell_deep[i - 1], cap_i) inner vectors; a size that is not below
// cap_i ends the chain, as it makes level i exact.
__host__ __device__ inline size_t deep_words_impl(int cap1, int levels, const int* ell_deep) {
    size_t w = 0;
    int cap = cap1;
    for (int i = 1; i < levels; ++i) {
        const int want = ell_deep[i - 1] < cap ? ell_deep[i - 1] : cap;
        if (want >= cap) break;
        w += nest_words_impl(cap, want);
        cap = want;
    }
    return w;
}

// Nest area of deeper level i (1 <= i < levels, within the chain above).
__device__ inline NestPtrs deep_ptrs(const JobDesc& J, int i) {
    double2* base = J.nest + nest_words_impl(J.k, J.lcap);
    int cap = J.lcap;
    for (int l = 1; l < i; ++l) {
        const int want = min(J.ell_deep[l - 1], cap);
        base += nest_words_impl(cap, want);
        cap = want;
    }
    return nest_ptrs(base, cap, min(J.ell_deep[i - 1], cap));
}

// out (k) = W s with the inner basis W of a level (m columns of length k)
template <typename T>
__device__ void basis_times(const NestPtrs& P, int k, int m, const T* s, T* out) {
    const T* vl = (const T*)P.vl;
    for (int q = threadIdx.x; q < k; q += NT) {
        T acc = s_zero<T>();
        for (int j = 0; j < m; ++j) acc = s_add(acc, s_mul(vl[(size_t)j * k + q], s[j]));
        out[q] = acc;
    }
    __syncthreads();
}

// Level 0 has built its inner space: T_1 (size m) in P0.al/bl/gl and W_0 in
// P0.vl.  Each deeper level i runs steps 3 and 4 on T_i (p_i given, or p_opt
// from T_i's Ritz extremes): the LU of p_i T_i and the (two-sided) Lanczos
// process on T_i' from e_1, giving T_{i+1} and W_i.  RHi runs on the deepest
// T_L and the result is lifted through every basis,
// c = W_0 W_1 ... W_{L-1} sgn(T_L) e_1 -> out (k0).  Returns the RHi
// iterations; levels, sizes and p go to res and the job's report words.
template <typename T>
__device__ int deep_coeffs(const JobDesc& J, const NestPtrs& P0, int k0, int m, T* out, const Smem& sm,
                           NestResult& res) {
    const int tid = threadIdx.x;
    __shared__ int nsz[NKS_MAX_LEVELS + 1];
    if (tid == 0) {
        nsz[0] = k0;
        nsz[1] = m;
        for (int i = 0; i + 1 < NKS_MAX_LEVELS; ++i) {
            J.status[ST_ELL_DEEP + i] = 0;
            J.report[RP_P_DEEP + i] = 0.0;
        }
    }
    __syncthreads();
    int depth = 1;   // levels whose inner space exists
    int cap = J.lcap;
    for (int i = 1; i < J.levels; ++i) {
        const int ni = nsz[i];
        const int want = min(J.ell_deep[i - 1], ni);
        const int want_cap = min(J.ell_deep[i - 1], cap);
        if (want >= ni || want_cap >= cap) break;   // level i is exact
        cap = want_cap;
        const NestPtrs Q = deep_ptrs(J, i);
        const NestPtrs U = (i == 1) ? P0 : deep_ptrs(J, i - 1);
        T* d = (T*)Q.d;
        T* sub = (T*)Q.sub;
        T* sup = (T*)Q.sup;
        for (int q = tid; q < ni; q += NT) {
            d[q] = ((const T*)U.al)[q];
            if (q + 1 < ni) { sub[q] = ((const T*)U.bl)[q]; sup[q] = ((const T*)U.gl)[q]; }
        }
        __syncthreads();
        double p = J.p_deep[i - 1];
        if (p <= 0.0) {
            double zmin, zmax;
            estimate_extremes<T>(Q, ni, sm, zmin, zmax);
            p = 1.0 / sqrt(zmin * zmax);
            if (!(p > 0.0) || !isfinite(p)) p = 1.0;
        }
        if (lu_pH<T>(Q, ni, p) != 0) { res.status = NKS_E_NOCONV; break; }
        Inner in;
        inner_init<T>(Q, ni, p, in, sm);
        inner_extend<T>(Q, ni, p, want, in, sm);
        if (in.serious) res.status = NKS_E_BREAKDOWN;
        if (tid == 0) {
            nsz[i + 1] = in.i;
            J.status[ST_ELL_DEEP + i - 1] = in.i;
            J.report[RP_P_DEEP + i - 1] = p;
        }
        __syncthreads();
        depth = i + 1;
    }
    res.levels = depth;
    // RHi on T_depth, lifted through W_{depth-1}, then through the bases above
    const NestPtrs B = (depth == 1) ? P0 : deep_ptrs(J, depth - 1);
    const int it = inner_coeffs<T>(J, B, nsz[depth - 1], nsz[depth], depth == 1 ? out : (T*)B.cc, sm);
    for (int i = depth - 2; i >= 0; --i) {
        const NestPtrs Pi = (i == 0) ? P0 : deep_ptrs(J, i);
        const NestPtrs Pn = deep_ptrs(J, i + 1);
        basis_times<T>(Pi, nsz[i], nsz[i + 1], (const T*)Pn.cc, i == 0 ? out : (T*)Pi.cc);
    }
    return it;
}

// H_k (k = kk) from the job's scalars into the nest area
template <typename T>
__device__ void load_H(const JobDesc& J, const NestPtrs& P, int kk) {
    const double2* sc = J.sc;
    const size_t st = J.scstride;
    T* d = (T*)P.d;
    T* sub = (T*)P.sub;
    T* sup = (T*)P.sup;
    for (int i = threadIdx.x; i < kk; i += NT) {
        d[i] = s_from<T>(sc[SC_ALPHA * st + i + 1]);
        if (i + 1 < kk) { sub[i] = s_from<T>(sc[SC_BETA * st + i + 1]); sup[i] = s_from<T>(sc[SC_GAMMA * st + i + 1]); }
    }
    __syncthreads();
}

// Steps 3-5 on H_k (k = kk); the result c is left in P.cc.  ell-doubling runs
// when the job's ell policy asks for it or force_doubling; it starts at
// ell_start (0: ELL0), stops at tol/10 (tol < 0: the job's), and records each
// doubling's change in trace[0..ntrace).
template <typename T>
__device__ NestResult nested_coeffs(const JobDesc& J, const NestPtrs& P, int kk, const Smem& sm, int ell_start = 0,
                                    double tol = -1.0, bool force_doubling = false, double* trace = nullptr,
                                    int ntrace = 0) {
    const int tid = threadIdx.x;
    load_H<T>(J, P, kk);
    T* cc = (T*)P.cc;
    T* cp = (T*)P.cp;
    NestResult res;
    if (tol < 0.0) tol = J.tol;
    const int cap = min(J.lcap, kk);   // largest inner size allowed
    const bool doubling = force_doubling || J.ell_policy != NKS_POLICY_FIXED;
    const int ell0 = doubling ? (ell_start > 0 ? ell_start : ELL0) : J.ell;
    if (ell0 >= kk || (doubling && ell0 >= cap && cap >= kk)) {
        res.rhi = nonnested_coeffs<T>(J, P, kk, cc, sm);
        res.ell = 0;
        return res;
    }
    double p = J.p;
    if (p <= 0.0) {
        estimate_extremes<T>(P, kk, sm, res.zmin, res.zmax);
        // no eigenvalue of A lies beyond J.zcap: a larger |theta| is a spurious
        // Ritz value of the oblique projection (two-sided, without
        // reorthogonalisation), and taking it for z_max would mistune p
        if (J.zcap > 0.0 && res.zmax > J.zcap) res.zmax = J.zcap;
        p = 1.0 / sqrt(res.zmin * res.zmax);
        if (!(p > 0.0) || !isfinite(p)) p = 1.0;   // degenerate estimate: p = 1 is one RHi step
    }
    res.p = p;
    if (lu_pH<T>(P, kk, p) != 0) { res.status = NKS_E_NOCONV; return res; }
    Inner in;
    inner_init<T>(P, kk, p, in, sm);
    res.levels = 1;
    if (!doubling) {
        inner_extend<T>(P, kk, p, min(ell0, cap), in, sm);
        if (J.levels > 1) res.rhi = deep_coeffs<T>(J, P, kk, in.i, cc, sm, res);
        else res.rhi = inner_coeffs<T>(J, P, kk, in.i, cc, sm, true);
        res.ell = in.i;
    } else {
        int ell = min(ell0, cap);
        inner_extend<T>(P, kk, p, ell, in, sm);
        res.rhi = inner_coeffs<T>(J, P, kk, in.i, cp, sm);
        res.ell = in.i;
        int step = 0;
        while (true) {
            const int ell2 = 2 * ell;
            if (ell2 >= cap && cap >= kk) {          // the inner space would be the whole of H_k
                res.rhi = nonnested_coeffs<T>(J, P, kk, cc, sm);
                res.inner_delta = rel_change<T>(cc, cp, kk, sm);
                res.ell = 0;
                res.levels = 0;
                if (trace && step < ntrace && tid == 0) trace[step] = res.inner_delta;
                break;
            }
            const int target = min(ell2, cap);
            inner_extend<T>(P, kk, p, target, in, sm);
            res.rhi = inner_coeffs<T>(J, P, kk, in.i, cc, sm);
            res.ell = in.i;
            res.inner_delta = rel_change<T>(cc, cp, kk, sm);
            if (trace && step < ntrace && tid == 0) trace[step] = res.inner_delta;
            ++step;
            if (res.inner_delta <= tol / 10 || target >= cap || in.ended) break;
            for (int i = tid; i < kk; i += NT) cp[i] = cc[i];
            __syncthreads();
            ell = ell2;
        }
    }
    if (in.serious) res.status = NKS_E_BREAKDOWN;
    return res;
}

// weighted change |c - [c_prev; 0]|_w / |c|_w with ||d||_w^2 = sum |d_i|^2 ||v_{i+1}||^2
template <typename T>
__device__ double weighted_change(const JobDesc& J, const T* c, int kk, const double2* prev, int kprev,
                                  const Smem& sm) {
    const double2* VN = J.sc + SC_VN * J.scstride;
    double dn = 0.0, cn = 0.0;
    for (int i = threadIdx.x; i < kk; i += NT) {
        const double w2 = cabs2(VN[i + 1]);
        const double2 ci = s_d2(c[i]);
        const double2 di = (i < kprev) ? csub(ci, prev[i]) : ci;
        dn += cabs2(di) * w2;
        cn += cabs2(ci) * w2;
    }
    const double2 r = block_sum<NT>(mk(dn, cn), sm.red);
    return sqrt(r.x) / sqrt(r.y);
}

// ---------------------------------------------------------------- learned policy
// Features of the probe Ritz matrix H_{k0} (all threads get them).
template <typename T>
__device__ void job_features(const JobDesc& J, const NestPtrs& P, int k0, const Smem& sm, double* f) {
    double zmin, zmax, zmin2, zmax2;
    load_H<T>(J, P, k0);
    estimate_extremes<T>(P, k0, sm, zmin, zmax);
    const int kh = max(2, k0 / 2);
    load_H<T>(J, P, kh);
    estimate_extremes<T>(P, kh, sm, zmin2, zmax2);
    const double2* sc = J.sc;
    const size_t st = J.scstride;
    double sa = 0.0, sb = 0.0;
    for (int i = threadIdx.x; i < k0; i += NT) {
        sa += cabs(sc[SC_ALPHA * st + i + 1]);
        if (i + 1 < k0) sb += sqrt(cabs(cmul(sc[SC_BETA * st + i + 1], sc[SC_GAMMA * st + i + 1])));
    }
    const double2 r = block_sum<NT>(mk(sa, sb), sm.red);
    for (int i = 0; i < NFEAT; ++i) f[i] = 0.0;
    f[0] = 1.0;
    f[1] = log10(zmin);
    f[2] = log10(zmax);
    f[3] = log10(zmin2);
    f[4] = log10(zmax / zmin);
    f[5] = J.mu;
    f[6] = log10(J.tol);
    f[7] = J.two_sided ? 1.0 : 0.0;
    f[8] = log10((double)J.V);
    f[9] = r.x / k0;
    f[10] = r.y / max(k0 - 1, 1);
}

__device__ inline float bf16r(float x) {   // round to the nearest bfloat16 (ties to even)
    unsigned int u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}
__device__ inline float silu_f(float z) { return z / (1.0f + expf(-z)); }

// Network inference for one feature vector (same rounding as the training
// kernels: bf16 weights and layer inputs, float32 accumulation).  Result in out[2].
__device__ void net_forward(const PolicyNet* net, const double* f, float* out) {
    __shared__ float x[NFEAT], h1[64], h2[64];
    const int tid = threadIdx.x;
    const float* P = net->params;
    if (tid < NFEAT) x[tid] = bf16r(((float)f[tid] - net->fmean[tid]) / net->fstd[tid]);
    __syncthreads();
    if (tid < 64) {
        float z = P[16 * 64 + tid];
        for (int i = 0; i < 16; ++i) z += x[i] * bf16r(P[i * 64 + tid]);
        h1[tid] = bf16r(silu_f(z));
    }
    __syncthreads();
    if (tid < 64) {
        const float* W2 = P + 16 * 64 + 64;
        float z = W2[64 * 64 + tid];
        for (int i = 0; i < 64; ++i) z += h1[i] * bf16r(W2[i * 64 + tid]);
        h2[tid] = bf16r(silu_f(z));
    }
    __syncthreads();
    if (tid < 2) {
        const float* W3 = P + 16 * 64 + 64 + 64 * 64 + 64;
        float z = W3[64 * 2 + tid];
        for (int i = 0; i < 64; ++i) z += h2[i] * bf16r(W3[i * 2 + tid]);
        out[tid] = z * net->tstd[tid] + net->tmean[tid];
    }
    __syncthreads();
}

enum NestMode { NEST_FINAL = 0, NEST_CHECKPOINT = 1, NEST_PREDICT = 2, NEST_LABEL = 3 };

// Final result (or an accepted checkpoint): lift weights and the job report.
template <typename T>
__device__ void write_result(const JobDesc& J, const T* cc, int kk, const NestResult& res, double outer_delta,
                             bool accept, bool kpol) {
    const int tid = threadIdx.x;
    const double2* SV = J.sc + SC_SV * J.scstride;
    const double bnorm = J.report[RP_BNORM];
    for (int q = tid; q < kk; q += NT) J.omega[q] = cscale(cmul(s_d2(cc[q]), SV[q + 1]), bnorm);
    if (tid == 0) {
        if (accept) {
            J.status[ST_DONE] = 1;
            J.status[ST_KUSED] = kk;
            J.status[ST_CKPT_DONE] = 1;
        }
        int status = J.status[ST_STATUS];
        if (status == NKS_OK && res.status != NKS_OK) status = res.status;
        if (status == NKS_OK && res.rhi < 0) status = NKS_E_NOCONV;
        // (a final non-nested step, ell = 0, is exact in ell and never counts)
        if (status == NKS_OK && J.ell_policy != NKS_POLICY_FIXED && res.ell != 0 && res.inner_delta > J.tol / 10)
            status = NKS_E_NOCONV;
        // a k policy that ran to its cap without meeting tol (a lucky breakdown is exact)
        if (status == NKS_OK && kpol && !accept && J.status[ST_DONE] == 0 &&
            (outer_delta < 0.0 || outer_delta > J.tol / 4))
            status = NKS_E_NOCONV;
        J.status[ST_STATUS] = status;
        J.status[ST_ELL] = res.ell;
        J.status[ST_LEVELS] = res.levels;
        J.status[ST_RHI] = res.rhi < 0 ? -res.rhi : res.rhi;
        J.report[RP_P] = res.p;
        J.report[RP_ZMIN] = res.zmin;
        J.report[RP_ZMAX] = res.zmax;
        J.report[RP_INNER_DELTA] = res.inner_delta;
        if (outer_delta >= 0.0) J.report[RP_OUTER_DELTA] = outer_delta;
    }
    __syncthreads();
}

template <typename T>
__device__ void store_checkpoint(const JobDesc& J, const T* cc, int kk, double outer_delta) {
    for (int i = threadIdx.x; i < kk; i += NT) J.ckpt[i] = s_d2(cc[i]);
    __syncthreads();
    if (threadIdx.x == 0) {
        J.status[ST_KCKPT] = kk;
        J.status[ST_NCKPT] += 1;
        if (outer_delta >= 0.0) J.report[RP_OUTER_DELTA] = outer_delta;
    }
    __syncthreads();
}

template <typename T>
__device__ void nested_job(const JobDesc& J, int mode, int j, const Smem& sm, float* net_out) {
    const int tid = threadIdx.x;
    const bool learned = J.k_policy == NKS_POLICY_LEARNED;
    const bool kpol = J.k_policy != NKS_POLICY_FIXED;
    NestPtrs P = nest_ptrs(J.nest, J.k, J.lcap);
    place_hot<T>(P, J.k, sm);
    const T* cc = (const T*)P.cc;
    const int ell_start = J.ell_policy == NKS_POLICY_LEARNED ? J.status[ST_ELLSTART] : 0;

    if (mode == NEST_PREDICT) {
        // learned policy: features of H_{k0} -> network -> k*, ell*
        if (!J.net || J.status[ST_DONE] || j >= J.k) return;
        __shared__ double f[NFEAT];
        double fl[NFEAT];
        job_features<T>(J, P, j, sm, fl);
        if (tid < NFEAT) f[tid] = fl[tid];
        __syncthreads();
        net_forward(J.net, f, net_out);
        if (tid == 0) {
            // (a non-finite output gives no k target and the smallest ell start)
            const double ks0 = pow(10.0, (double)net_out[0]);
            const double ks = (ks0 >= 0.0 && ks0 < 1e7) ? ks0 : 1e7;
            const double ls0 = pow(10.0, (double)net_out[1]);
            const double ls = (ls0 >= 0.0 && ls0 < 1e7) ? ls0 : 0.0;
            int kt = (int)ceil(ks / LEARN_DK) * LEARN_DK;
            kt = max(kt, j + LEARN_DK);
            if (learned && kt < J.k) {
                J.status[ST_KTARGET] = kt;
                if (J.group) atomicMax(J.group + GW_KTARGET_MAX, kt);
            }
            // largest power of two not above ell* (at least 8): a start below the
            // needed size costs one more doubling at small size, one above a
            // dense RHi step eight times dearer per doubling
            int es = 8;
            while (2.0 * es <= 1.05 * ls && es < J.lcap) es *= 2;
            J.status[ST_ELLSTART] = es;
        }
        __syncthreads();
        return;
    }

    if (mode == NEST_LABEL) {
        // features of H_{k0} and the reference c_ref = c(k_used) (label_kernel does the rest)
        if (!J.label) return;
        const int kused = J.status[ST_KUSED];
        double* L = J.label;
        for (int i = tid; i < LABEL_WORDS; i += NT) L[i] = nan("");
        __syncthreads();
        if (kused < LEARN_K0 + LABEL_DK) return;
        double fl[NFEAT];
        job_features<T>(J, P, LEARN_K0, sm, fl);
        if (tid < NFEAT) L[tid] = fl[tid];
        __syncthreads();
        nested_coeffs<T>(J, P, kused, sm, 0, LABEL_TOL, true);
        for (int i = tid; i < kused; i += NT) J.ckpt[i] = s_d2(cc[i]);
        __syncthreads();
        return;
    }

    if (mode == NEST_CHECKPOINT) {
        if (!kpol || J.status[ST_DONE] || j >= J.k) return;
        if (learned && !J.status[ST_FALLBACK] && J.status[ST_KTARGET] > 0) {
            // Every job of the group is verified in the same launch, at the
            // group's largest target (or this job's last checkpoint before
            // its own k cap), each on its own H_{k*}: a leading section of
            // the longer basis.  One launch instead of one per distinct k*.
            const int kt = J.status[ST_KTARGET];
            const int jlast = ((J.k - 1) / LEARN_DK) * LEARN_DK;
            const int jv = J.group ? min(J.group[GW_KTARGET_MAX], jlast) : kt;
            if (j != jv) return;
            // verify k* against k* - LEARN_VERIFY_DK
            const int kv = kt - LEARN_VERIFY_DK;
            nested_coeffs<T>(J, P, kv, sm, ell_start);
            store_checkpoint<T>(J, cc, kv, -1.0);
            NestResult res = nested_coeffs<T>(J, P, kt, sm, ell_start);
            const double delta = weighted_change<T>(J, cc, kt, J.ckpt, kv, sm);
            if (delta <= J.tol / 4 && res.status == NKS_OK) {
                write_result<T>(J, cc, kt, res, delta, true, true);
            } else {
                // fall back to the plain checkpoints from here on
                store_checkpoint<T>(J, cc, kt, delta);
                if (tid == 0) {
                    J.status[ST_FALLBACK] = 1;
                    J.status[ST_KTARGET] = 0;
                }
                __syncthreads();
            }
            return;
        }
        if (j % CKPT_DK != 0) return;
        NestResult res = nested_coeffs<T>(J, P, j, sm, ell_start);
        double outer_delta = -1.0;
        if (J.status[ST_NCKPT] > 0 && res.status == NKS_OK)
            outer_delta = weighted_change<T>(J, cc, j, J.ckpt, J.status[ST_KCKPT], sm);
        if (outer_delta >= 0.0 && outer_delta <= J.tol / 4) write_result<T>(J, cc, j, res, outer_delta, true, true);
        else store_checkpoint<T>(J, cc, j, outer_delta);
        return;
    }

    // NEST_FINAL
    const int kk = J.status[ST_KUSED];
    if (kk == 0) return;                              // zero source; lift writes zeros
    if (J.status[ST_CKPT_DONE]) return;               // a checkpoint already accepted H_kk
    NestResult res = nested_coeffs<T>(J, P, kk, sm, ell_start);
    double outer_delta = -1.0;
    if (kpol && J.status[ST_NCKPT] > 0 && res.status == NKS_OK)
        outer_delta = weighted_change<T>(J, cc, kk, J.ckpt, J.status[ST_KCKPT], sm);
    write_result<T>(J, cc, kk, res, outer_delta, false, kpol);
}

__global__ __launch_bounds__(NT) void nested_kernel(JobDesc* jobs, int mode, int j) {
    __shared__ double2 red[NT / 64];
    __shared__ double redd[NT / 64];
    __shared__ int redi[NT / 64];
    __shared__ Aff2<double2> scan_lds[NT];
    __shared__ double2 panel_lds[GJ_PANEL_BYTES / sizeof(double2)];
    __shared__ double2 hot_lds[HOT_BYTES / sizeof(double2)];
    __shared__ float net_out[2];
    Smem sm;
    sm.red = red;
    sm.redd = redd;
    sm.redi = redi;
    sm.scan = scan_lds;
    sm.panel = panel_lds;
    sm.hot = hot_lds;
    const JobDesc& J = jobs[blockIdx.x];
    if (J.two_sided) nested_job<double2>(J, mode, j, sm, net_out);
    else nested_job<double>(J, mode, j, sm, net_out);
}

// Label run, one workgroup per (job, k_i): c(k_i) with the ell doubling traced,
// and its weighted error against c_ref.  Each k_i has its own nested scratch.
template <typename T>
__device__ void label_point(const JobDesc& J, int i, const Smem& sm) {
    const int tid = threadIdx.x;
    const int kused = J.status[ST_KUSED];
    const int ki = LABEL_DK * (i + 1);
    if (!J.label || kused < LEARN_K0 + LABEL_DK || ki > kused) return;
    NestPtrs P = nest_ptrs(J.nest + (size_t)(i + 1) * J.nest_cap, J.k, J.lcap);
    const T* cc = (const T*)P.cc;
    __shared__ double trace[LABEL_NELL];
    if (tid < LABEL_NELL) trace[tid] = nan("");
    __syncthreads();
    nested_coeffs<T>(J, P, ki, sm, 0, LABEL_TOL, true, trace, LABEL_NELL);
    const double2* VN = J.sc + SC_VN * J.scstride;
    double dn = 0.0, rn = 0.0;
    for (int q = tid; q < kused; q += NT) {
        const double w2 = cabs2(VN[q + 1]);
        const double2 c = (q < ki) ? s_d2(cc[q]) : mk(0.0, 0.0);
        dn += cabs2(csub(c, J.ckpt[q])) * w2;
        rn += cabs2(J.ckpt[q]) * w2;
    }
    const double2 r = block_sum<NT>(mk(dn, rn), sm.red);
    if (tid == 0) {
        double* L = J.label;
        L[NFEAT + i] = sqrt(r.x) / sqrt(r.y);
        for (int e = 0; e < LABEL_NELL; ++e) L[NFEAT + LABEL_NK + i * LABEL_NELL + e] = trace[e];
    }
}

__global__ __launch_bounds__(NT) void label_kernel(JobDesc* jobs) {
    __shared__ double2 red[NT / 64];
    __shared__ double redd[NT / 64];
    __shared__ int redi[NT / 64];
    __shared__ Aff2<double2> scan_lds[NT];
    __shared__ double2 panel_lds[GJ_PANEL_BYTES / sizeof(double2)];
    Smem sm;
    sm.red = red;
    sm.redd = redd;
    sm.redi = redi;
    sm.scan = scan_lds;
    sm.panel = panel_lds;
    sm.hot = nullptr;
    const JobDesc& J = jobs[blockIdx.x];
    if (J.two_sided) label_point<double2>(J, blockIdx.y, sm);
    else label_point<double>(J, blockIdx.y, sm);
}

// H(k,k) = alpha_k from the partial sums of the last stencil pass (the
// recurrence pass of iteration k is not needed: App. A/B stop after it).
__global__ __launch_bounds__(NT) void finalize_kernel(JobDesc* jobs) {
    const JobDesc& J = jobs[blockIdx.x];
    const int kused = J.status[ST_KUSED];
    if (kused == 0 || J.status[ST_DONE]) return;
    const size_t st = J.scstride;
    // the last stencil pass's partials, or their total in the slot's last entry (collapsed)
    if (threadIdx.x >= 64) return;
    const double2* ps = J.part + (size_t)PS_S * J.pstride;
    const bool col = J.nblocks > J.collapse;
    const double2 s = wave_sum(col ? ps + J.pstride - 1 : ps, col ? 1 : J.nblocks);
    const double2 a = J.two_sided ? cmul(cconj(J.sc[SC_SW * st + kused]), s)
                                  : mk(J.sc[SC_SV * st + kused].x * s.x, 0.0);
    if (threadIdx.x == 0) J.sc[SC_ALPHA * st + kused] = a;
}

}  // namespace

size_t nest_words(int k, int ell, int levels, const int* ell_deep) {
    const int L = ell >= k ? k : ell;
    return nest_words_impl(k, L) + (ell < k ? deep_words_impl(L, levels, ell_deep) : 0);
}

void launch_finalize(JobDesc* jobs, int njobs, hipStream_t s) {
    hipLaunchKernelGGL(finalize_kernel, dim3(njobs), dim3(NT), 0, s, jobs);
}

void launch_nested(JobDesc* jobs, int njobs, hipStream_t s, LaunchEvents ev) {
    if (ev.a)
        hipExtLaunchKernelGGL(nested_kernel, dim3(njobs), dim3(NT), 0, s, ev.a, ev.b, 0, jobs, (int)NEST_FINAL, 0);
    else
        hipLaunchKernelGGL(nested_kernel, dim3(njobs), dim3(NT), 0, s, jobs, (int)NEST_FINAL, 0);
}

void launch_checkpoint(JobDesc* jobs, int njobs, int j, hipStream_t s) {
    hipLaunchKernelGGL(nested_kernel, dim3(njobs), dim3(NT), 0, s, jobs, (int)NEST_CHECKPOINT, j);
}

void launch_predict(JobDesc* jobs, int njobs, int j, hipStream_t s) {
    hipLaunchKernelGGL(nested_kernel, dim3(njobs), dim3(NT), 0, s, jobs, (int)NEST_PREDICT, j);
}

void launch_label(JobDesc* jobs, int njobs, hipStream_t s) {
    hipLaunchKernelGGL(nested_kernel, dim3(njobs), dim3(NT), 0, s, jobs, (int)NEST_LABEL, 0);
    hipLaunchKernelGGL(label_kernel, dim3(njobs, LABEL_NK), dim3(NT), 0, s, jobs);
}

}  // namespace nks
