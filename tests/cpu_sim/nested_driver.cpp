// Runs the nested-step kernels of libnks (nested.hip, compiled for the host
// with the emulated HIP runtime of hip/hip_runtime.h in this directory) on
// one job whose outer Ritz matrix H_k is read from a file, so that tests can
// check the device code's arithmetic and, under AddressSanitizer, every
// memory access it makes, without a GPU.
//
// Every buffer of the job gets its own allocation, sized exactly as the
// library's workspace planner sizes it; in label mode the nested scratch
// areas that a launch must not touch are poisoned, so that an access outside
// the area of the running block is reported.
//
// usage: nested_sim <input> <output>
//   input  (little endian): int32[16] header, float64[8] parameters,
//          int32[8] ell_deep, float64[8] p_deep,
//          complex128[SC_COUNT * (k + 2)] scalars (the job's SC_* slots),
//          in label mode without the head launch: complex128[k] reference c
//   output: int32[ST_COUNT] status, float64[RP_COUNT] report,
//           complex128[k] omega, float64[LABEL_WORDS] label words (label mode)
#include "../../paper_0912_4457_amd/csrc/nested.hip"

#include <sanitizer/asan_interface.h>

#include <cstdio>
#include <cstring>
#include <vector>

namespace {

enum Hdr { H_K, H_ELL, H_TWO_SIDED, H_KUSED, H_MAX_RHI, H_MODE, H_I_LO, H_I_HI, H_V, H_KPOL, H_ELLPOL, H_LEVELS,
           H_NO_HEAD, H_FILL, H_COUNT = 16 };
enum Par { P_P, P_TOL, P_RHI_TOL, P_MU, P_BNORM, P_COUNT = 8 };

template <typename T>
T* alloc(size_t n) {
    T* p = static_cast<T*>(calloc(n ? n : 1, sizeof(T)));
    if (!p) { fprintf(stderr, "out of memory\n"); exit(2); }
    return p;
}

bool read_all(FILE* f, void* p, size_t n) { return fread(p, 1, n, f) == n; }

}  // namespace

int main(int argc, char** argv) {
    using namespace nks;
    if (argc != 3) { fprintf(stderr, "usage: %s <input> <output>\n", argv[0]); return 2; }
    FILE* f = fopen(argv[1], "rb");
    if (!f) { perror(argv[1]); return 2; }
    int32_t h[H_COUNT];
    double par[P_COUNT];
    int32_t ell_deep[8];
    double p_deep[8];
    if (!read_all(f, h, sizeof(h)) || !read_all(f, par, sizeof(par)) || !read_all(f, ell_deep, sizeof(ell_deep)) ||
        !read_all(f, p_deep, sizeof(p_deep))) {
        fprintf(stderr, "short header\n");
        return 2;
    }
    const int k = h[H_K], ell = h[H_ELL], mode = h[H_MODE];
    const bool label = mode == NEST_LABEL;
    const size_t scn = (size_t)SC_COUNT * (k + 2);
    double2* sc = alloc<double2>(scn);
    if (!read_all(f, sc, sizeof(double2) * scn)) { fprintf(stderr, "short scalars\n"); return 2; }
    std::vector<double2> cref;
    if (label && h[H_NO_HEAD]) {
        cref.resize(k);
        if (!read_all(f, cref.data(), sizeof(double2) * k)) { fprintf(stderr, "short reference\n"); return 2; }
    }
    fclose(f);

    JobDesc d{};
    d.k = k;
    d.ell = ell;
    d.p = par[P_P];
    d.max_rhi = h[H_MAX_RHI];
    d.rhi_tol = par[P_RHI_TOL];
    d.two_sided = h[H_TWO_SIDED];
    d.lcap = ell >= k ? k : ell;
    d.scstride = k + 2;
    d.nblocks = 1;
    d.precision = NKS_FP64;
    d.k_policy = h[H_KPOL];
    d.ell_policy = h[H_ELLPOL];
    d.tol = par[P_TOL];
    d.mu = par[P_MU];
    d.V = h[H_V];
    d.levels = h[H_LEVELS] > 0 ? h[H_LEVELS] : 1;
    for (int i = 0; i + 1 < NKS_MAX_LEVELS; ++i) {
        d.ell_deep[i] = i + 1 < d.levels ? ell_deep[i] : 0;
        d.p_deep[i] = i + 1 < d.levels ? p_deep[i] : 0.0;
    }
    d.sc = sc;
    d.status = alloc<int>(ST_COUNT);
    d.report = alloc<double>(RP_COUNT);
    d.omega = alloc<double2>(k);
    d.part = alloc<double2>(PS_COUNT);
    d.group = alloc<int>(GROUP_WORDS);
    const bool ck = d.k_policy != NKS_POLICY_FIXED || label;
    d.ckpt = ck ? alloc<double2>(k) : nullptr;
    for (size_t i = 0; i < cref.size(); ++i) d.ckpt[i] = cref[i];
    d.label = label ? alloc<double>(LABEL_WORDS) : nullptr;
    const size_t nw = nest_words(k, ell, d.levels, d.ell_deep);
    d.nest_cap = (int)nw;
    const int nareas = label ? 1 + LABEL_NK : 1;
    d.nest = alloc<double2>(nw * nareas);
    d.status[ST_KUSED] = h[H_KUSED];
    d.report[RP_BNORM] = par[P_BNORM];
    // device workspace is not cleared by the library: fill what the kernels
    // must write before reading with a byte pattern (H_FILL != 0), so that a
    // read of unwritten memory gives garbage here too rather than zeros
    if (h[H_FILL]) {
        const int fb = h[H_FILL] & 0xFF;
        memset(d.nest, fb, sizeof(double2) * nw * nareas);
        memset(d.omega, fb, sizeof(double2) * k);
        memset(d.part, fb, sizeof(double2) * PS_COUNT);
        if (d.label) memset(d.label, fb, sizeof(double) * LABEL_WORDS);
        if (d.ckpt && cref.empty()) memset(d.ckpt, fb, sizeof(double2) * k);
    }
    JobDesc* table = alloc<JobDesc>(1);
    table[0] = d;

    auto poison_all_but = [&](int area) {
        for (int a = 0; a < nareas; ++a) {
            void* base = d.nest + nw * a;
            if (a == area) ASAN_UNPOISON_MEMORY_REGION(base, sizeof(double2) * nw);
            else ASAN_POISON_MEMORY_REGION(base, sizeof(double2) * nw);
        }
    };

    if (!label) {
        if (mode == NEST_FINAL) launch_nested(table, 1, nullptr);
        else { fprintf(stderr, "mode %d is not run by this driver\n", mode); return 2; }
    } else {
        poison_all_but(0);
        // the head launch (features and the reference c) unless only label points are asked for
        if (!h[H_NO_HEAD]) hipLaunchKernelGGL(nested_kernel, dim3(1), dim3(NT), 0, nullptr, table, (int)NEST_LABEL, 0);
        for (int i = h[H_I_LO]; i < h[H_I_HI] && i < LABEL_NK; ++i) {
            poison_all_but(i + 1);
            fprintf(stderr, "label point %d (k_i = %d)\n", i, LABEL_DK * (i + 1));
            ::hipsim::g_only_y = i;
            hipLaunchKernelGGL(label_kernel, dim3(1, LABEL_NK), dim3(NT), 0, nullptr, table);
            ::hipsim::g_only_y = -1;
        }
        poison_all_but(-1);
    }

    FILE* o = fopen(argv[2], "wb");
    if (!o) { perror(argv[2]); return 2; }
    fwrite(d.status, sizeof(int), ST_COUNT, o);
    fwrite(d.report, sizeof(double), RP_COUNT, o);
    fwrite(d.omega, sizeof(double2), k, o);
    if (label) fwrite(d.label, sizeof(double), LABEL_WORDS, o);
    fclose(o);
    return 0;
}
