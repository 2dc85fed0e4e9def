// Stand-alone application of A = gamma5 D_w(mu) (or A^dagger = A(-mu)) to a
// boundary-layout vector: gather to structure-of-arrays, stencil, scatter.
#include "wilson.h"

namespace nks {

constexpr int APPLY_NT = 128;

template <typename R>
__global__ __launch_bounds__(256) void aos_to_soa(const double2* __restrict__ in, cx_t<R>* __restrict__ out,
                                                 int V) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;   // e = comp * V + site
    if (e >= 12 * V) return;
    const int c = e / V, s = e - c * V;
    out[e] = from_d2<R>(in[(size_t)12 * s + c]);
}

template <typename R>
__global__ __launch_bounds__(256) void soa_to_aos(const cx_t<R>* __restrict__ in, double2* __restrict__ out,
                                                 int V) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 12 * V) return;
    const int c = e / V, s = e - c * V;
    out[(size_t)12 * s + c] = to_d2<R>(in[e]);
}

template <typename R>
__global__ __launch_bounds__(APPLY_NT) void apply_kernel(Geom g, const cx_t<R>* __restrict__ links,
                                                        const cx_t<R>* __restrict__ in,
                                                        cx_t<R>* __restrict__ out, double kappa, double mu) {
    const int site = blockIdx.x * APPLY_NT + threadIdx.x;
    if (site >= g.V) return;
    R cf[1][4], cb[1][4];
    hop_coefs<R>(kappa, mu, cf[0], cb[0]);
    const cx_t<R>* const fields[1] = {in};
    cx_t<R> acc[1][12];
    wilson_site<R, 1>(g, links, fields, cf, cb, site, acc);
#pragma unroll
    for (int c = 0; c < 12; ++c) out[(size_t)c * g.V + site] = acc[0][c];
}

template <typename R>
void launch_apply(const Geom& g, const cx_t<R>* links, double kappa, double mu, const double2* in,
                  double2* out, cx_t<R>* tmp_in, cx_t<R>* tmp_out, hipStream_t s) {
    const int n = 12 * g.V;
    hipLaunchKernelGGL(aos_to_soa<R>, dim3((n + 255) / 256), dim3(256), 0, s, in, tmp_in, g.V);
    hipLaunchKernelGGL(apply_kernel<R>, dim3((g.V + APPLY_NT - 1) / APPLY_NT), dim3(APPLY_NT), 0, s, g, links,
                       tmp_in, tmp_out, kappa, mu);
    hipLaunchKernelGGL(soa_to_aos<R>, dim3((n + 255) / 256), dim3(256), 0, s, tmp_out, out, g.V);
}

template void launch_apply<double>(const Geom&, const double2*, double, double, const double2*, double2*,
                                   double2*, double2*, hipStream_t);
template void launch_apply<float>(const Geom&, const float2*, double, double, const double2*, double2*,
                                  float2*, float2*, hipStream_t);

}  // namespace nks
