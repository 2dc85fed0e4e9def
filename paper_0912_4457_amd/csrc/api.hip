// C ABI of libnks: contexts, lattices, workspace planning and the launch
// sequence of a (batched) sign application.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "nks_internal.h"

namespace {
constexpr int EIG_DEGREE = 40;                    // Chebyshev filter degree of the eigensolver
constexpr unsigned long long EIG_SEED = 20091224;  // its start block

// Workspace of nks_sign_apply_noalloc, for callers that cannot allocate: one
// array of NKS_NOALLOC_BYTES on every GPU the library runs on, held from when
// the library's code object is loaded until the process ends.  In host code
// the name `scratch` is only a stand-in: its device address on each GPU is
// taken once, by nks_create with that GPU current, into g_scratch[device].
static __device__ __align__(256) char scratch[NKS_NOALLOC_BYTES];
constexpr int MAX_DEVICES = 64;
void* g_scratch[MAX_DEVICES] = {};
std::mutex g_scratch_mu;

// Device address of the calling GPU's scratch array; the GPU must be current.
int scratch_address(int device, void** out) {
    if (device < 0 || device >= MAX_DEVICES) return NKS_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return NKS_E_HIP;
        g_scratch[device] = p;
    }
    *out = g_scratch[device];
    return NKS_OK;
}
}  // namespace

using namespace nks;

struct ProfRecord {
    int cls;
    hipEvent_t a, b;
    double bytes;
};

struct nks_ctx {
    int device = 0;
    std::string last_error;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    // host copy of the last job table, kept alive while its upload may be in flight
    std::vector<JobDesc> descs;
    // sampled kernel timing (nks_profile_enable)
    bool prof = false;
    std::vector<hipEvent_t> pool;
    std::vector<ProfRecord> pending;
    long long prof_count[NKS_K_COUNT] = {0, 0, 0, 0};
    Tuning tune;
    PolicyNet* net = nullptr;     // device copy of the learned-policy network (nks_policy_load)
    // graph mode: captured launch sequences keyed by the job table they were captured for
    int graph = 1;
    hipStream_t cap = nullptr;    // private stream the sequences are captured on
    // side streams and fork/join events for lattice groups run concurrently
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr;
    hipEvent_t lead = nullptr;    // staggered groups: the lead group reached its start point
    struct Graph {
        std::vector<char> key;
        hipGraphExec_t exec = nullptr;
        unsigned long long used = 0;
        hipEvent_t done = nullptr;   // recorded after every launch of exec, on the launching stream
    };
    std::vector<Graph> graphs;
    unsigned long long graph_clock = 0;
    long long graph_captures = 0, graph_replays = 0;
};

struct nks_lattice {
    nks_ctx* ctx = nullptr;
    Geom g{};
    double m0 = 1.6, mu = 0.0, kappa = 1.0 / 4.8;
    double2* links64 = nullptr;   // SoA [nu][row][col][site]
    float2* links32 = nullptr;
    double2* tmp = nullptr;       // 2 * 12V complex128 scratch for nks_apply_op
    // deflation: m eigenpairs, SoA [i][comp][site]
    int defl_m = 0, defl_cap = 0;
    double2* defl_r = nullptr;
    double2* defl_l = nullptr;    // null: left = right (Hermitian)
    double* defl_sgn = nullptr;
};

namespace {

int fail(nks_ctx* ctx, int code, const std::string& msg) {
    if (ctx) ctx->last_error = msg;
    return code;
}

#define HIP_TRY(ctx, call)                                                                     \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail((ctx), NKS_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }
constexpr int NONNESTED_MAX = RHI_MAX;   // dense k x k RHi limit of the non-nested mode

// caller layout [i][12*site + comp] -> [i][comp][site]
__global__ void vecs_to_soa(const double2* __restrict__ in, double2* __restrict__ out, int V, int m) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;   // e = (i * 12 + comp) * V + site
    const long long n = 12LL * V;
    if (e >= n * m) return;
    const long long i = e / n, r = e - i * n;
    const int c = (int)(r / V), s = (int)(r - (long long)c * V);
    out[e] = in[i * n + 12LL * s + c];
}

// [i][comp][site] -> caller layout [i][12*site + comp]
__global__ void vecs_from_soa(const double2* __restrict__ in, double2* __restrict__ out, int V, int m) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;   // e = (i * 12 + comp) * V + site
    const long long n = 12LL * V;
    if (e >= n * m) return;
    const long long i = e / n, r = e - i * n;
    const int c = (int)(r / V), s = (int)(r - (long long)c * V);
    out[i * n + 12LL * s + c] = in[e];
}

__global__ void links_to_soa(const double2* __restrict__ in, double2* __restrict__ o64, float2* __restrict__ o32,
                             int V) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;   // e = q * V + site, q = nu*9 + row*3 + col
    if (e >= 36 * V) return;
    const int q = e / V, s = e - q * V;
    const double2 u = in[(size_t)s * 36 + q];
    o64[e] = u;
    o32[e] = make_float2((float)u.x, (float)u.y);
}

int even_up(int k) { return k + (k & 1); }

struct JobPlan {
    int idx;            // index in the caller's job array
    nks_lattice* lat;
    int k, ell, precision, two_sided;
    double p;
    int max_rhi;
    double rhi_tol;
    int nblocks, lcap;
    int k_policy, ell_policy;
    double tol;
    bool label;         // label run (nks_policy_label): checkpoint buffer + label words
    int group;          // index of its (lattice, precision) group
    int overlap;        // NKS_FLAG_OVERLAP
    int dm;             // deflated eigenpairs (NKS_FLAG_DEFLATE)
    int ring;           // NKS_FLAG_DOUBLE_PASS: two-column store, second pass
    int levels;         // nested levels (multi-level nesting)
    int ell_deep[NKS_MAX_LEVELS - 1];
    double p_deep[NKS_MAX_LEVELS - 1];
    size_t off_dcoef, off_dpart;
    size_t off_vstore, off_yacc, off_lring, off_part, off_sc, off_status, off_report, off_omega, off_ckpt, off_label, off_nest,
        end;
    bool learned() const { return k_policy == NKS_POLICY_LEARNED || ell_policy == NKS_POLICY_LEARNED; }
};

struct Plan {
    std::vector<JobPlan> jobs;     // ordered by group
    std::vector<std::pair<int, int>> groups;   // [start, count) per (lattice, precision)
    size_t table_bytes = 0;
    size_t group_off = 0;     // GROUP_WORDS ints per group, after the job table
    size_t total = 0;
};

// Levels of a validated nks_opts: sizes rounded up to even, unused entries 0.
void set_levels(int& levels, int* ell_deep, double* p_deep, const nks_opts* o) {
    levels = o->levels;
    for (int i = 0; i + 1 < NKS_MAX_LEVELS; ++i) {
        const bool used = i + 1 < levels;
        ell_deep[i] = used ? even_up(o->ell_deep[i]) : 0;
        p_deep[i] = used ? o->p_deep[i] : 0.0;
    }
}

void fill_level_stats(nks_stats& o, const int* st, const double* rp) {
    o.levels_used = st[ST_LEVELS];
    for (int i = 0; i + 1 < NKS_MAX_LEVELS; ++i) {
        const bool ran = i + 1 < o.levels_used;
        o.ell_deep_used[i] = ran ? st[ST_ELL_DEEP + i] : 0;
        o.p_deep_used[i] = ran ? rp[RP_P_DEEP + i] : 0.0;
    }
}

int validate_opts(nks_ctx* ctx, const nks_opts* o) {
    if (!o) return fail(ctx, NKS_E_INVALID, "opts is NULL");
    if (o->size != sizeof(nks_opts)) return fail(ctx, NKS_E_INVALID, "opts->size mismatch (ABI version)");
    if (o->k < 1) return fail(ctx, NKS_E_INVALID, "k must be >= 1");
    if (o->ell < 1) return fail(ctx, NKS_E_INVALID, "ell must be >= 1");
    if (o->precision != NKS_FP64 && o->precision != NKS_MIXED)
        return fail(ctx, NKS_E_INVALID, "unknown precision");
    if (o->max_rhi_iter < 1) return fail(ctx, NKS_E_INVALID, "max_rhi_iter must be >= 1");
    if (!(o->rhi_tol > 0.0)) return fail(ctx, NKS_E_INVALID, "rhi_tol must be > 0");
    if (o->k_policy < NKS_POLICY_FIXED || o->k_policy > NKS_POLICY_LEARNED ||
        o->ell_policy < NKS_POLICY_FIXED || o->ell_policy > NKS_POLICY_LEARNED)
        return fail(ctx, NKS_E_INVALID, "unknown policy");
    if ((o->k_policy == NKS_POLICY_LEARNED || o->ell_policy == NKS_POLICY_LEARNED) && !(ctx && ctx->net))
        return fail(ctx, NKS_E_UNSUPPORTED, "learned policy needs a network (nks_policy_load)");
    if (o->flags & ~(unsigned)(NKS_FLAG_OVERLAP | NKS_FLAG_DEFLATE | NKS_FLAG_DOUBLE_PASS))
        return fail(ctx, NKS_E_INVALID, "unknown flag bits");
    if ((o->k_policy != NKS_POLICY_FIXED || o->ell_policy != NKS_POLICY_FIXED) && !(o->tol > 0.0 && o->tol < 1.0))
        return fail(ctx, NKS_E_INVALID, "policies need 0 < tol < 1");
    if (o->levels < 1 || o->levels > NKS_MAX_LEVELS) return fail(ctx, NKS_E_INVALID, "levels must be in 1..NKS_MAX_LEVELS");
    for (int i = 0; i + 1 < o->levels; ++i) {
        if (o->ell_deep[i] < 1) return fail(ctx, NKS_E_INVALID, "ell_deep[i] must be >= 1 for i < levels - 1");
        if (!std::isfinite(o->p_deep[i])) return fail(ctx, NKS_E_INVALID, "p_deep[i] must be finite");
    }
    if (o->levels > 1 && (o->ell_policy != NKS_POLICY_FIXED || o->k_policy == NKS_POLICY_LEARNED))
        return fail(ctx, NKS_E_UNSUPPORTED, "levels > 1 needs the FIXED ell policy and a FIXED or DOUBLING k policy");
    return NKS_OK;
}

int make_plan(nks_ctx* ctx, int njobs, const nks_job* jobs, Plan& P, bool label = false) {
    if (njobs < 1 || !jobs) return fail(ctx, NKS_E_INVALID, "no jobs");
    std::vector<JobPlan> tmp;
    for (int i = 0; i < njobs; ++i) {
        const nks_job& J = jobs[i];
        if (!J.lat) return fail(ctx, NKS_E_INVALID, "job lattice is NULL");
        int rc = validate_opts(ctx, J.opts);
        if (rc) return rc;
        JobPlan jp{};
        jp.idx = i;
        jp.lat = J.lat;
        jp.k = even_up(J.opts->k);
        jp.ell = even_up(J.opts->ell);
        jp.precision = J.opts->precision;
        jp.two_sided = J.lat->mu != 0.0;
        jp.p = J.opts->p;
        jp.max_rhi = J.opts->max_rhi_iter;
        jp.rhi_tol = J.opts->rhi_tol;
        jp.k_policy = J.opts->k_policy;
        jp.ell_policy = J.opts->ell_policy;
        jp.tol = J.opts->tol;
        jp.label = label;
        jp.overlap = (J.opts->flags & NKS_FLAG_OVERLAP) ? 1 : 0;
        jp.ring = (J.opts->flags & NKS_FLAG_DOUBLE_PASS) ? 1 : 0;
        set_levels(jp.levels, jp.ell_deep, jp.p_deep, J.opts);
        jp.dm = 0;
        if (J.opts->flags & NKS_FLAG_DEFLATE) {
            if (J.lat->defl_m == 0)
                return fail(ctx, NKS_E_INVALID, "NKS_FLAG_DEFLATE on a lattice without deflation (nks_lattice_set_deflation)");
            jp.dm = J.lat->defl_m;
        }
        jp.lcap = jp.ell >= jp.k ? jp.k : jp.ell;
        if (jp.ell >= jp.k && jp.k > NONNESTED_MAX)
            return fail(ctx, NKS_E_UNSUPPORTED, "non-nested mode (ell >= k) is limited to k <= 1024");
        if (jp.lcap > RHI_MAX) return fail(ctx, NKS_E_UNSUPPORTED, "ell is limited to 1024");
        jp.nblocks = (J.lat->g.V + OUTER_NT - 1) / OUTER_NT;
        tmp.push_back(jp);
    }
    // group by (lattice, precision), keeping first-appearance order
    std::vector<int> order;
    std::vector<bool> used(tmp.size(), false);
    for (size_t i = 0; i < tmp.size(); ++i) {
        if (used[i]) continue;
        const int start = (int)P.jobs.size();
        for (size_t j = i; j < tmp.size(); ++j)
            if (!used[j] && tmp[j].lat == tmp[i].lat && tmp[j].precision == tmp[i].precision) {
                used[j] = true;
                P.jobs.push_back(tmp[j]);
            }
        P.groups.push_back({start, (int)P.jobs.size() - start});
    }
    size_t off = align_up(sizeof(JobDesc) * P.jobs.size());
    P.group_off = off;
    off = align_up(off + sizeof(int) * GROUP_WORDS * P.groups.size());
    for (size_t gi = 0; gi < P.groups.size(); ++gi)
        for (int i = P.groups[gi].first; i < P.groups[gi].first + P.groups[gi].second; ++i) P.jobs[i].group = (int)gi;
    P.table_bytes = off;
    for (auto& jp : P.jobs) {
        const size_t n = (size_t)12 * jp.lat->g.V;
        const size_t es = jp.precision == NKS_FP64 ? sizeof(double2) : sizeof(float2);
        jp.off_vstore = off; off = align_up(off + (size_t)(jp.ring ? 2 : jp.k) * n * es);
        jp.off_yacc = off; off = align_up(off + (jp.ring ? 2 * n * sizeof(double2) : 0));
        jp.off_lring = off; off = align_up(off + (jp.two_sided ? 2 * n * es : 0));
        jp.off_part = off; off = align_up(off + sizeof(double2) * PS_COUNT * (jp.nblocks + 1));
        jp.off_sc = off; off = align_up(off + sizeof(double2) * SC_COUNT * (jp.k + 2));
        jp.off_status = off; off = align_up(off + sizeof(int) * ST_COUNT);
        jp.off_report = off; off = align_up(off + sizeof(double) * RP_COUNT);
        jp.off_omega = off; off = align_up(off + sizeof(double2) * jp.k);
        const bool ck = jp.k_policy != NKS_POLICY_FIXED || jp.label;
        jp.off_ckpt = off; off = align_up(off + (ck ? sizeof(double2) * jp.k : 0));
        jp.off_label = off; off = align_up(off + (jp.label ? sizeof(double) * LABEL_WORDS : 0));
        jp.off_dcoef = off; off = align_up(off + sizeof(double2) * jp.dm);
        jp.off_dpart = off; off = align_up(off + sizeof(double2) * (size_t)jp.dm * jp.nblocks);
        jp.off_nest = off;
        off = align_up(off + sizeof(double2) * nest_words(jp.k, jp.ell, jp.levels, jp.ell_deep) * (jp.label ? 1 + LABEL_NK : 1));
        jp.end = off;
    }
    P.total = off;
    return NKS_OK;
}

JobDesc make_desc(const nks_ctx* ctx, const Plan& P, const JobPlan& jp, char* ws, const void* b, void* x) {
    JobDesc d{};
    d.b = static_cast<const double2*>(b);
    d.x = static_cast<double2*>(x);
    d.vstore = ws + jp.off_vstore;
    d.ring = jp.ring;
    d.yacc = jp.ring ? reinterpret_cast<double2*>(ws + jp.off_yacc) : nullptr;
    d.lring = jp.two_sided ? ws + jp.off_lring : nullptr;
    d.part = reinterpret_cast<double2*>(ws + jp.off_part);
    d.sc = reinterpret_cast<double2*>(ws + jp.off_sc);
    d.status = reinterpret_cast<int*>(ws + jp.off_status);
    d.report = reinterpret_cast<double*>(ws + jp.off_report);
    d.omega = reinterpret_cast<double2*>(ws + jp.off_omega);
    d.nest = reinterpret_cast<double2*>(ws + jp.off_nest);
    d.k = jp.k;
    d.ell = jp.ell;
    d.p = jp.p;
    d.max_rhi = jp.max_rhi;
    d.rhi_tol = jp.rhi_tol;
    d.two_sided = jp.two_sided;
    d.nest_cap = (int)nest_words(jp.k, jp.ell, jp.levels, jp.ell_deep);
    d.lcap = jp.lcap;
    d.scstride = jp.k + 2;
    d.nblocks = jp.nblocks;
    d.pstride = jp.nblocks + 1;   // + the collapsed total
    d.collapse = ctx->tune.collapse;
    d.precision = jp.precision;
    d.k_policy = jp.k_policy;
    d.ell_policy = jp.ell_policy;
    d.tol = jp.tol;
    d.ckpt = (jp.k_policy != NKS_POLICY_FIXED || jp.label) ? reinterpret_cast<double2*>(ws + jp.off_ckpt) : nullptr;
    d.label = jp.label ? reinterpret_cast<double*>(ws + jp.off_label) : nullptr;
    d.mu = jp.lat->mu;
    d.zcap = norm_bound(jp.lat->kappa, jp.lat->mu);
    d.V = jp.lat->g.V;
    d.net = jp.learned() ? ctx->net : nullptr;
    d.group = reinterpret_cast<int*>(ws + P.group_off) + (size_t)GROUP_WORDS * jp.group;
    d.overlap = jp.overlap;
    d.levels = jp.levels;
    for (int i = 0; i + 1 < NKS_MAX_LEVELS; ++i) {
        d.ell_deep[i] = jp.ell_deep[i];
        d.p_deep[i] = jp.p_deep[i];
    }
    d.dm = jp.dm;
    if (jp.dm > 0) {
        d.dr = jp.lat->defl_r;
        d.dl = jp.lat->defl_l ? jp.lat->defl_l : jp.lat->defl_r;
        d.dsgn = jp.lat->defl_sgn;
        d.dcoef = reinterpret_cast<double2*>(ws + jp.off_dcoef);
        d.dpart = reinterpret_cast<double2*>(ws + jp.off_dpart);
    }
    return d;
}

OuterLaunch group_launch(const nks_ctx* ctx, const Plan& P, int gi, JobDesc* table) {
    const auto [start, count] = P.groups[gi];
    const JobPlan& jp = P.jobs[start];
    OuterLaunch L{};
    L.g = jp.lat->g;
    L.links = jp.precision == NKS_FP64 ? (const void*)jp.lat->links64 : (const void*)jp.lat->links32;
    L.kappa = jp.lat->kappa;
    L.mu = jp.lat->mu;
    L.jobs = table + start;
    L.njobs = count;
    L.kmax = 0;
    L.deflate = 0;
    L.ring = 0;
    L.pass2 = 0;
    for (int i = start; i < start + count; ++i) {
        L.kmax = std::max(L.kmax, P.jobs[i].k);
        if (P.jobs[i].dm > 0) L.deflate = 1;
        if (P.jobs[i].ring) L.ring = 1;
    }
    L.nblocks = jp.nblocks;
    L.precision = jp.precision;
    L.two_sided = jp.two_sided;
    L.tune = ctx->tune;
    return L;
}

constexpr int PROF_EVERY = 8;     // time one launch in eight of each class
constexpr size_t PROF_POOL = 4096;

// Pick one launch in PROF_EVERY of class cls for timing; its events go to the
// dispatch of that launch (LaunchEvents), which stamps the kernel's own start
// and end.  Returns null events for launches that are not timed.
LaunchEvents prof_take(nks_ctx* ctx, int cls, double bytes) {
    if (!ctx->prof) return {};
    if (ctx->prof_count[cls]++ % PROF_EVERY != 0) return {};
    if (ctx->pool.size() < 2) return {};
    ProfRecord r{cls, ctx->pool.back(), nullptr, bytes};
    ctx->pool.pop_back();
    r.b = ctx->pool.back();
    ctx->pool.pop_back();
    ctx->pending.push_back(r);
    return {r.a, r.b};
}

// The nested step and the lift are timed at every launch.
LaunchEvents prof_take_always(nks_ctx* ctx, int cls, double bytes) {
    const long long c = ctx->prof_count[cls];
    ctx->prof_count[cls] = 0;
    LaunchEvents ev = prof_take(ctx, cls, bytes);
    ctx->prof_count[cls] = c + 1;
    return ev;
}

// Algorithmic bytes of one launch: every input read once, every output written once.
double bytes_S(const OuterLaunch& L, const Plan& P, int start, int j) {
    const double cs = L.precision == NKS_FP64 ? 16.0 : 8.0;
    const double sp = 12.0 * cs, lk = 36.0 * cs;
    double per_site = lk;
    for (int i = start; i < start + L.njobs; ++i) {
        const int k = P.jobs[i].k;
        if (j > k) continue;
        const double f = L.two_sided ? 2.0 : 1.0;          // A v and A^dagger w
        per_site += f * sp * (1.0 + (j >= 2 ? 1.0 : 0.0) + (j < k ? 1.0 : 0.0));
    }
    return per_site * L.g.V;
}
double bytes_R(const OuterLaunch& L, const Plan& P, int start, int j) {
    const double cs = L.precision == NKS_FP64 ? 16.0 : 8.0;
    const double sp = 12.0 * cs;
    double per_site = 0.0;
    for (int i = start; i < start + L.njobs; ++i)
        if (j < P.jobs[i].k) per_site += (L.two_sided ? 6.0 : 3.0) * sp;
    return per_site * L.g.V;
}
double bytes_lift(const OuterLaunch& L, const Plan& P, int start) {
    const double cs = L.precision == NKS_FP64 ? 16.0 : 8.0;
    double per_site = 0.0;
    for (int i = start; i < start + L.njobs; ++i)
        per_site += (P.jobs[i].ring ? 2.0 * 12.0 * 16.0 : 12.0 * cs * P.jobs[i].k) + 12.0 * 16.0;
    return per_site * L.g.V;
}

// Double-pass jobs of a group: pack again and regenerate the basis, summing
// omega_j u_j on the way (Sec. 4.4).  The nested step must have run.
void enqueue_second_pass(OuterLaunch L, hipStream_t s) {
    if (!L.ring) return;
    L.pass2 = 1;
    launch_pack(L, s);
    for (int j = 1; j <= L.kmax; ++j) {
        launch_outer_S(L, j, s);
        if (j < L.kmax) launch_outer_R(L, j, s);
    }
}

enum Phase { PH_ALL = 0, PH_OUTER_ONLY = 1, PH_LABEL = 2 };

// Enqueue the whole method for all jobs; the job table must already be on the
// device at the start of ws.  Events (when timed) mark phase ends.
// Streams for the lattice groups: group 0 on the call's stream, the others
// on side streams that fork from it and join it again (all at the default
// priority).  With concurrency off every group uses the call's stream.
int ensure_side_streams(nks_ctx* ctx, size_t ngroups) {
    if (!ctx->fork) HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
    if (!ctx->lead) HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->lead, hipEventDisableTiming));
    while (ctx->side.size() + 1 < ngroups) {
        hipStream_t st;
        HIP_TRY(ctx, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        ctx->side.push_back(st);
        hipEvent_t e;
        HIP_TRY(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->join.push_back(e);
    }
    return NKS_OK;
}

int fork_groups(nks_ctx* ctx, size_t ngroups, hipStream_t s) {
    if (!ctx->tune.concurrent || ngroups < 2) return NKS_OK;
    int rc = ensure_side_streams(ctx, ngroups);
    if (rc) return rc;
    HIP_TRY(ctx, hipEventRecord(ctx->fork, s));
    for (size_t g = 1; g < ngroups; ++g) HIP_TRY(ctx, hipStreamWaitEvent(ctx->side[g - 1], ctx->fork, 0));
    return NKS_OK;
}

int join_groups(nks_ctx* ctx, size_t ngroups, hipStream_t s) {
    if (!ctx->tune.concurrent || ngroups < 2) return NKS_OK;
    for (size_t g = 1; g < ngroups; ++g) {
        HIP_TRY(ctx, hipEventRecord(ctx->join[g - 1], ctx->side[g - 1]));
        HIP_TRY(ctx, hipStreamWaitEvent(s, ctx->join[g - 1], 0));
    }
    return NKS_OK;
}

hipStream_t group_stream(const nks_ctx* ctx, size_t gi, size_t ngroups, hipStream_t s) {
    return (ctx->tune.concurrent && ngroups >= 2 && gi > 0) ? ctx->side[gi - 1] : s;
}

int enqueue_kernels(nks_ctx* ctx, const Plan& P, const std::vector<JobDesc>& descs, char* ws, hipStream_t s0,
                    bool timed, int phase) {
    JobDesc* table = reinterpret_cast<JobDesc*>(ws);
    const size_t ng = P.groups.size();
    // With concurrent groups (and no per-phase timing) each group also runs its
    // own nested step and lift right after its outer loop, so they overlap the
    // outer loops of slower groups.
    const bool pipe = !timed && phase == PH_ALL && ctx->tune.concurrent && ctx->tune.pipeline && ng >= 2;
    // Staggered start (pipelined groups): the group with the costliest nested
    // step (two-sided first, then the largest k) is enqueued first and the
    // others wait until it has done stagger % of its outer loop, so that their
    // outer passes still run while its nested step leaves most CUs idle.
    size_t lead = 0;
    int lead_j = 0;
    if (pipe && ctx->tune.stagger > 0) {
        auto cost = [&](size_t g) {
            const JobPlan& jp = P.jobs[P.groups[g].first];
            int kmax = 0;
            for (int i = P.groups[g].first; i < P.groups[g].first + P.groups[g].second; ++i)
                kmax = std::max(kmax, P.jobs[i].k);
            return (jp.two_sided ? 2.0 : 1.0) * kmax;
        };
        for (size_t g = 1; g < ng; ++g)
            if (cost(g) > cost(lead)) lead = g;
        int kl = 0;
        for (int i = P.groups[lead].first; i < P.groups[lead].first + P.groups[lead].second; ++i)
            kl = std::max(kl, P.jobs[i].k);
        lead_j = std::max(1, kl * ctx->tune.stagger / 100);
    }
    if (timed) HIP_TRY(ctx, hipEventRecord(ctx->ev[0], s0));
    int frc = fork_groups(ctx, ng, s0);
    if (frc) return frc;
    for (size_t oi = 0; oi < ng; ++oi) {
        const size_t gi = lead_j ? (oi == 0 ? lead : (oi <= lead ? oi - 1 : oi)) : oi;
        hipStream_t s = group_stream(ctx, gi, ng, s0);
        OuterLaunch L = group_launch(ctx, P, (int)gi, table);
        const int start = P.groups[gi].first;
        if (lead_j && gi != lead) HIP_TRY(ctx, hipStreamWaitEvent(s, ctx->lead, 0));
        bool kpol = false, learned = false, klearned = false;
        for (int i = start; i < start + L.njobs; ++i) {
            kpol = kpol || P.jobs[i].k_policy != NKS_POLICY_FIXED;
            learned = learned || P.jobs[i].learned();
            klearned = klearned || P.jobs[i].k_policy == NKS_POLICY_LEARNED;
        }
        launch_pack(L, s);
        for (int j = 1; j <= L.kmax; ++j) {
            L.ev = prof_take(ctx, NKS_K_STENCIL, ctx->prof ? bytes_S(L, P, start, j) : 0.0);
            launch_outer_S(L, j, s);
            L.ev = {};
            if (j < L.kmax) {
                L.ev = prof_take(ctx, NKS_K_RECUR, ctx->prof ? bytes_R(L, P, start, j) : 0.0);
                launch_outer_R(L, j, s);
                L.ev = {};
                if (learned && j == LEARN_K0) launch_predict(L.jobs, L.njobs, j, s);
                // plain checkpoints every CKPT_DK; a learned k target is a multiple of LEARN_DK
                if (kpol && (j % CKPT_DK == 0 || (klearned && j > LEARN_K0 && j % LEARN_DK == 0)))
                    launch_checkpoint(L.jobs, L.njobs, j, s);
            }
            if (lead_j && gi == lead && j == std::min(lead_j, L.kmax)) HIP_TRY(ctx, hipEventRecord(ctx->lead, s));
        }
        if (pipe) {
            launch_finalize(L.jobs, L.njobs, s);
            launch_nested(L.jobs, L.njobs, s, prof_take_always(ctx, NKS_K_NESTED, 0.0));
            enqueue_second_pass(L, s);
            L.ev = prof_take_always(ctx, NKS_K_LIFT, ctx->prof ? bytes_lift(L, P, start) : 0.0);
            launch_lift(L, s);
            L.ev = {};
        }
    }
    frc = join_groups(ctx, ng, s0);
    if (frc) return frc;
    HIP_TRY(ctx, hipGetLastError());
    if (pipe) return NKS_OK;
    hipStream_t s = s0;
    launch_finalize(table, (int)descs.size(), s);
    HIP_TRY(ctx, hipGetLastError());
    if (timed) HIP_TRY(ctx, hipEventRecord(ctx->ev[1], s));
    if (phase == PH_OUTER_ONLY) return NKS_OK;
    if (phase == PH_LABEL) {
        launch_label(table, (int)descs.size(), s);
        HIP_TRY(ctx, hipGetLastError());
        return NKS_OK;
    }
    launch_nested(table, (int)descs.size(), s, prof_take_always(ctx, NKS_K_NESTED, 0.0));
    HIP_TRY(ctx, hipGetLastError());
    if (timed) HIP_TRY(ctx, hipEventRecord(ctx->ev[2], s));
    frc = fork_groups(ctx, ng, s0);
    if (frc) return frc;
    for (size_t gi = 0; gi < ng; ++gi) {
        hipStream_t sl = group_stream(ctx, gi, ng, s0);
        OuterLaunch L = group_launch(ctx, P, (int)gi, table);
        enqueue_second_pass(L, sl);
        L.ev = prof_take_always(ctx, NKS_K_LIFT, ctx->prof ? bytes_lift(L, P, P.groups[gi].first) : 0.0);
        launch_lift(L, sl);
    }
    frc = join_groups(ctx, ng, s0);
    if (frc) return frc;
    HIP_TRY(ctx, hipGetLastError());
    if (timed) HIP_TRY(ctx, hipEventRecord(ctx->ev[3], s));
    return NKS_OK;
}

int enqueue(nks_ctx* ctx, const Plan& P, const std::vector<JobDesc>& descs, char* ws, hipStream_t s, bool timed,
            int phase) {
    HIP_TRY(ctx, hipMemcpyAsync(ws, descs.data(), sizeof(JobDesc) * descs.size(), hipMemcpyHostToDevice, s));
    return enqueue_kernels(ctx, P, descs, ws, s, timed, phase);
}

constexpr size_t GRAPH_CACHE = 4;

// Graph mode: the kernel sequence of a batch is captured once (on a private
// stream) and replayed; the job table is uploaded before every replay.  The
// key is the table itself (every pointer, size and option of every job)
// except each job's b and x: the kernels read those from the uploaded table
// only, so new source and output buffers replay the same graph.
int enqueue_graph(nks_ctx* ctx, const Plan& P, const std::vector<JobDesc>& descs, char* ws, hipStream_t s) {
    std::vector<JobDesc> kd(descs);
    for (auto& d : kd) { d.b = nullptr; d.x = nullptr; }
    std::vector<char> key(sizeof(JobDesc) * kd.size());
    std::memcpy(key.data(), kd.data(), key.size());
    auto put = [&key](const void* p, size_t n) {
        key.insert(key.end(), static_cast<const char*>(p), static_cast<const char*>(p) + n);
    };
    const size_t wsaddr = reinterpret_cast<size_t>(ws);
    put(&wsaddr, sizeof(wsaddr));
    put(&ctx->tune, sizeof(ctx->tune));
    for (const auto& gr : P.groups) {
        // launch arguments taken by value at capture: operator parameters and link fields
        const nks_lattice* lat = P.jobs[gr.first].lat;
        put(&lat->kappa, sizeof(lat->kappa));
        put(&lat->mu, sizeof(lat->mu));
        put(&lat->links64, sizeof(lat->links64));
        put(&lat->links32, sizeof(lat->links32));
        put(&lat->g, sizeof(lat->g));
    }
    nks_ctx::Graph* hit = nullptr;
    for (auto& g : ctx->graphs)
        if (g.key == key) hit = &g;
    if (!hit) {
        if (!ctx->cap) HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
        HIP_TRY(ctx, hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue_kernels(ctx, P, descs, ws, ctx->cap, false, PH_ALL);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(ctx->cap, &graph);
        if (rc) { if (graph) (void)hipGraphDestroy(graph); return rc; }
        if (e != hipSuccess) return fail(ctx, NKS_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        hipGraphExec_t exec = nullptr;
        const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e2 != hipSuccess) return fail(ctx, NKS_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
        if (ctx->graphs.size() >= GRAPH_CACHE) {
            auto old = std::min_element(ctx->graphs.begin(), ctx->graphs.end(),
                                        [](const nks_ctx::Graph& a, const nks_ctx::Graph& b) { return a.used < b.used; });
            // the evicted graph may still run on the stream of its last launch
            if (old->done) {
                HIP_TRY(ctx, hipEventSynchronize(old->done));
                (void)hipEventDestroy(old->done);
            }
            (void)hipGraphExecDestroy(old->exec);
            ctx->graphs.erase(old);
        }
        hipEvent_t done = nullptr;
        const hipError_t e3 = hipEventCreateWithFlags(&done, hipEventDisableTiming);
        if (e3 != hipSuccess) {
            (void)hipGraphExecDestroy(exec);
            return fail(ctx, NKS_E_HIP, std::string("hipEventCreate: ") + hipGetErrorString(e3));
        }
        ctx->graphs.push_back({key, exec, 0, done});
        hit = &ctx->graphs.back();
        ++ctx->graph_captures;
    } else {
        ++ctx->graph_replays;
    }
    hit->used = ++ctx->graph_clock;
    HIP_TRY(ctx, hipMemcpyAsync(ws, descs.data(), sizeof(JobDesc) * descs.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipGraphLaunch(hit->exec, s));
    HIP_TRY(ctx, hipEventRecord(hit->done, s));
    return NKS_OK;
}

int read_stats(nks_ctx* ctx, const Plan& P, char* ws, bool timed, nks_stats* out_by_caller_index) {
    float t01 = 0, t12 = 0, t23 = 0;
    if (timed) {
        (void)hipEventElapsedTime(&t01, ctx->ev[0], ctx->ev[1]);
        (void)hipEventElapsedTime(&t12, ctx->ev[1], ctx->ev[2]);
        (void)hipEventElapsedTime(&t23, ctx->ev[2], ctx->ev[3]);
    }
    for (const auto& jp : P.jobs) {
        int st[ST_COUNT];
        double rp[RP_COUNT];
        HIP_TRY(ctx, hipMemcpy(st, ws + jp.off_status, sizeof(st), hipMemcpyDeviceToHost));
        HIP_TRY(ctx, hipMemcpy(rp, ws + jp.off_report, sizeof(rp), hipMemcpyDeviceToHost));
        nks_stats& o = out_by_caller_index[jp.idx];
        std::memset(&o, 0, sizeof(o));
        o.status = st[ST_STATUS];
        o.k_used = st[ST_KUSED];
        o.ell_used = st[ST_ELL];
        o.rhi_iters = st[ST_RHI];
        o.breakdown_iter = st[ST_BDITER];
        o.p_used = rp[RP_P];
        o.z_min = rp[RP_ZMIN];
        o.z_max = rp[RP_ZMAX];
        o.b_norm = rp[RP_BNORM];
        o.inner_delta = rp[RP_INNER_DELTA];
        o.outer_delta = rp[RP_OUTER_DELTA];
        o.ms_outer = t01;
        o.ms_nested = t12;
        o.ms_lift = t23;
        fill_level_stats(o, st, rp);
    }
    return NKS_OK;
}

}  // namespace

extern "C" {

void nks_opts_default(nks_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->size = sizeof(nks_opts);
    o->k = 200;
    o->ell = 50;
    o->tol = 1e-8;
    o->precision = NKS_FP64;
    o->p = 0.0;
    o->k_policy = NKS_POLICY_FIXED;
    o->ell_policy = NKS_POLICY_FIXED;
    o->max_rhi_iter = 50;
    o->rhi_tol = 1e-14;
    o->flags = 0;
    o->levels = 1;
}

int nks_create(int device, nks_ctx** out) {
    if (!out) return NKS_E_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return NKS_E_INVALID;
    if (hipSetDevice(device) != hipSuccess) return NKS_E_HIP;
    void* scr = nullptr;
    if (const int rc = scratch_address(device, &scr)) return rc;
    auto* c = new nks_ctx();
    c->device = device;
    if (const char* e = getenv("NKS_XCD_MAP")) c->tune.xcd_map = std::min(3, std::max(0, atoi(e)));
    if (const char* e = getenv("NKS_GRAPH")) c->graph = atoi(e) != 0;
    for (auto& e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) { delete c; return NKS_E_HIP; }
    *out = c;
    return NKS_OK;
}

void nks_destroy(nks_ctx* ctx) {
    if (!ctx) return;
    for (auto& e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& r : ctx->pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto& e : ctx->pool) (void)hipEventDestroy(e);
    if (ctx->net) (void)hipFree(ctx->net);
    for (auto& g : ctx->graphs) {
        if (g.done) {
            (void)hipEventSynchronize(g.done);
            (void)hipEventDestroy(g.done);
        }
        (void)hipGraphExecDestroy(g.exec);
    }
    for (auto& st : ctx->side) (void)hipStreamDestroy(st);
    for (auto& e : ctx->join) (void)hipEventDestroy(e);
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    if (ctx->lead) (void)hipEventDestroy(ctx->lead);
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    delete ctx;
}

const char* nks_last_error(nks_ctx* ctx) { return ctx ? ctx->last_error.c_str() : "no context"; }

const char* nks_status_str(int s) {
    switch (s) {
        case NKS_OK: return "ok";
        case NKS_E_INVALID: return "invalid argument";
        case NKS_E_NOMEM: return "workspace too small or out of memory";
        case NKS_E_HIP: return "HIP error";
        case NKS_E_UNSUPPORTED: return "unsupported";
        case NKS_E_BREAKDOWN: return "serious two-sided Lanczos breakdown";
        case NKS_E_NOCONV: return "no convergence";
        default: return "unknown status";
    }
}

int nks_lattice_create(nks_ctx* ctx, const int32_t dims[4], const void* links_dev, nks_lattice** out) {
    if (!ctx || !dims || !links_dev || !out) return fail(ctx, NKS_E_INVALID, "NULL argument");
    *out = nullptr;
    long long V = 1;
    for (int i = 0; i < 4; ++i) {
        if (dims[i] < 2) return fail(ctx, NKS_E_INVALID, "every lattice extent must be >= 2");
        V *= dims[i];
    }
    if (V * 36 > (1LL << 31) - 1) return fail(ctx, NKS_E_UNSUPPORTED, "lattice too large for 32-bit indexing");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    auto lat = std::make_unique<nks_lattice>();
    lat->ctx = ctx;
    lat->g = Geom{dims[0], dims[1], dims[2], dims[3], (int)V};
    HIP_TRY(ctx, hipMalloc(&lat->links64, sizeof(double2) * 36 * V));
    HIP_TRY(ctx, hipMalloc(&lat->links32, sizeof(float2) * 36 * V));
    HIP_TRY(ctx, hipMalloc(&lat->tmp, sizeof(double2) * 24 * V));
    const int n = (int)(36 * V);
    hipLaunchKernelGGL(links_to_soa, dim3((n + 255) / 256), dim3(256), 0, nullptr,
                       static_cast<const double2*>(links_dev), lat->links64, lat->links32, (int)V);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipDeviceSynchronize());
    *out = lat.release();
    return NKS_OK;
}

int nks_lattice_set_params(nks_lattice* lat, double m0, double mu) {
    if (!lat) return NKS_E_INVALID;
    const double mw = -m0;
    if (!(mw > -2.0 && mw < 0.0)) return fail(lat->ctx, NKS_E_INVALID, "m_w = -m0 must lie in (-2, 0)");
    if (!(mu == mu) || mu > 50.0 || mu < -50.0) return fail(lat->ctx, NKS_E_INVALID, "mu must be finite");
    lat->m0 = m0;
    lat->mu = mu;
    lat->kappa = 1.0 / (8.0 + 2.0 * mw);
    return NKS_OK;
}

void nks_lattice_destroy(nks_lattice* lat) {
    if (!lat) return;
    (void)hipFree(lat->defl_r);
    (void)hipFree(lat->defl_l);
    (void)hipFree(lat->defl_sgn);
    (void)hipFree(lat->links64);
    (void)hipFree(lat->links32);
    (void)hipFree(lat->tmp);
    delete lat;
}

int nks_lattice_set_deflation(nks_lattice* lat, int m, const void* r_dev, const void* l_dev,
                              const double* lambda_host) {
    if (!lat) return NKS_E_INVALID;
    nks_ctx* ctx = lat->ctx;
    if (m < 0 || m > DEFL_MAX) return fail(ctx, NKS_E_INVALID, "deflation takes 0 <= m <= 64 eigenpairs");
    if (m > 0 && (!r_dev || !lambda_host)) return fail(ctx, NKS_E_INVALID, "NULL eigenvectors or eigenvalues");
    std::vector<double> sg(m);
    for (int i = 0; i < m; ++i) {
        const double re = lambda_host[2 * i];
        if (!(re == re) || re == 0.0) return fail(ctx, NKS_E_INVALID, "sgn is undefined for Re(lambda) = 0 or NaN");
        sg[i] = re > 0.0 ? 1.0 : -1.0;
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipDeviceSynchronize());     // no call in flight may read the old eigenpairs
    const size_t n = (size_t)12 * lat->g.V;
    if (m > lat->defl_cap) {
        (void)hipFree(lat->defl_r);
        (void)hipFree(lat->defl_l);
        (void)hipFree(lat->defl_sgn);
        lat->defl_r = lat->defl_l = nullptr;
        lat->defl_sgn = nullptr;
        lat->defl_cap = lat->defl_m = 0;
        HIP_TRY(ctx, hipMalloc(&lat->defl_r, sizeof(double2) * n * m));
        HIP_TRY(ctx, hipMalloc(&lat->defl_l, sizeof(double2) * n * m));
        HIP_TRY(ctx, hipMalloc(&lat->defl_sgn, sizeof(double) * m));
        lat->defl_cap = m;
    }
    if (m > 0) {
        const long long tot = (long long)n * m;
        const int nb = (int)((tot + 255) / 256);
        hipLaunchKernelGGL(vecs_to_soa, dim3(nb), dim3(256), 0, nullptr, static_cast<const double2*>(r_dev),
                           lat->defl_r, lat->g.V, m);
        hipLaunchKernelGGL(vecs_to_soa, dim3(nb), dim3(256), 0, nullptr,
                           static_cast<const double2*>(l_dev ? l_dev : r_dev), lat->defl_l, lat->g.V, m);
        HIP_TRY(ctx, hipGetLastError());
        HIP_TRY(ctx, hipMemcpy(lat->defl_sgn, sg.data(), sizeof(double) * m, hipMemcpyHostToDevice));
        HIP_TRY(ctx, hipDeviceSynchronize());
    }
    lat->defl_m = m;
    return NKS_OK;
}

int nks_lattice_eigensolve(nks_lattice* lat, int m, int max_iter, double tol, double* lambda_host,
                           double* resid_host, int* iters) {
    if (!lat) return NKS_E_INVALID;
    nks_ctx* ctx = lat->ctx;
    if (m < 1 || m > DEFL_MAX) return fail(ctx, NKS_E_INVALID, "the eigensolver takes 1 <= m <= 64 eigenpairs");
    if (max_iter < 1 || !(tol > 0.0)) return fail(ctx, NKS_E_INVALID, "max_iter must be >= 1 and tol > 0");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipDeviceSynchronize());     // no call in flight may read the old eigenpairs
    const size_t n = (size_t)12 * lat->g.V;
    if (m > lat->defl_cap) {
        (void)hipFree(lat->defl_r);
        (void)hipFree(lat->defl_l);
        (void)hipFree(lat->defl_sgn);
        lat->defl_r = lat->defl_l = nullptr;
        lat->defl_sgn = nullptr;
        lat->defl_cap = lat->defl_m = 0;
        HIP_TRY(ctx, hipMalloc(&lat->defl_r, sizeof(double2) * n * m));
        HIP_TRY(ctx, hipMalloc(&lat->defl_l, sizeof(double2) * n * m));
        HIP_TRY(ctx, hipMalloc(&lat->defl_sgn, sizeof(double) * m));
        lat->defl_cap = m;
    }
    lat->defl_m = 0;
    const int p = m + std::max(8, m);
    std::vector<double> lam(2 * m), res(m);
    int it = 0;
    std::string err;
    const int rc = eig_chfsi(lat->g, lat->links64, lat->kappa, lat->mu, m, p, EIG_DEGREE, max_iter, tol, EIG_SEED,
                             lat->defl_r, lat->defl_l, lam.data(), res.data(), &it, err);
    if (iters) *iters = it;
    for (int i = 0; i < m; ++i) {
        if (lambda_host) {
            lambda_host[2 * i] = lam[2 * i];
            lambda_host[2 * i + 1] = lam[2 * i + 1];
        }
        if (resid_host) resid_host[i] = res[i];
    }
    if (rc != NKS_OK) return fail(ctx, rc, err);
    std::vector<double> sg(m);
    for (int i = 0; i < m; ++i) {   // sgn(lambda) = sgn(Re lambda)
        const double re = lam[2 * i];
        if (!(re != 0.0)) return fail(ctx, NKS_E_NOCONV, "eigensolver: an eigenvalue with Re(lambda) = 0 has no sign");
        sg[i] = re > 0.0 ? 1.0 : -1.0;
    }
    HIP_TRY(ctx, hipMemcpy(lat->defl_sgn, sg.data(), sizeof(double) * m, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipDeviceSynchronize());
    lat->defl_m = m;
    return NKS_OK;
}

int nks_lattice_get_deflation(nks_lattice* lat, int* m_out, void* r_dev, void* l_dev) {
    if (!lat || !m_out) return NKS_E_INVALID;
    nks_ctx* ctx = lat->ctx;
    *m_out = lat->defl_m;
    const int m = lat->defl_m;
    if (m == 0 || (!r_dev && !l_dev)) return NKS_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const long long tot = 12LL * lat->g.V * m;
    const int nb = (int)((tot + 255) / 256);
    if (r_dev) hipLaunchKernelGGL(vecs_from_soa, dim3(nb), dim3(256), 0, nullptr, lat->defl_r, static_cast<double2*>(r_dev), lat->g.V, m);
    if (l_dev) hipLaunchKernelGGL(vecs_from_soa, dim3(nb), dim3(256), 0, nullptr, lat->defl_l, static_cast<double2*>(l_dev), lat->g.V, m);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipDeviceSynchronize());
    return NKS_OK;
}

int nks_apply_op(nks_lattice* lat, const void* in, void* out, int dagger, int precision, void* stream) {
    if (!lat || !in || !out) return fail(lat ? lat->ctx : nullptr, NKS_E_INVALID, "NULL argument");
    if (in == out) return fail(lat->ctx, NKS_E_INVALID, "in and out must not alias");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double mu = dagger ? -lat->mu : lat->mu;
    const size_t n = (size_t)12 * lat->g.V;
    if (precision == NKS_FP64) {
        launch_apply<double>(lat->g, lat->links64, lat->kappa, mu, static_cast<const double2*>(in),
                             static_cast<double2*>(out), lat->tmp, lat->tmp + n, s);
    } else if (precision == NKS_MIXED) {
        auto* t = reinterpret_cast<float2*>(lat->tmp);
        launch_apply<float>(lat->g, lat->links32, lat->kappa, mu, static_cast<const double2*>(in),
                            static_cast<double2*>(out), t, t + n, s);
    } else {
        return fail(lat->ctx, NKS_E_INVALID, "unknown precision");
    }
    HIP_TRY(lat->ctx, hipGetLastError());
    return NKS_OK;
}

int nks_workspace_size(nks_ctx* ctx, int njobs, const nks_job* jobs, size_t* bytes) {
    if (!ctx || !bytes) return NKS_E_INVALID;
    Plan P;
    int rc = make_plan(ctx, njobs, jobs, P);
    if (rc) return rc;
    *bytes = P.total;
    return NKS_OK;
}

int nks_sign_apply_batch(nks_ctx* ctx, int njobs, const nks_job* jobs, void* ws, size_t ws_bytes, void* stream,
                         nks_stats* stats) {
    if (!ctx) return NKS_E_INVALID;
    Plan P;
    int rc = make_plan(ctx, njobs, jobs, P);
    if (rc) return rc;
    if (!ws || ws_bytes < P.total)
        return fail(ctx, NKS_E_NOMEM, "workspace smaller than nks_workspace_size (" + std::to_string(P.total) + " bytes)");
    for (int i = 0; i < njobs; ++i)
        if (!jobs[i].b || !jobs[i].x) return fail(ctx, NKS_E_INVALID, "job b or x is NULL");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    char* w = static_cast<char*>(ws);
    std::vector<JobDesc>& descs = ctx->descs;
    descs.clear();
    for (const auto& jp : P.jobs) descs.push_back(make_desc(ctx, P, jp, w, jobs[jp.idx].b, jobs[jp.idx].x));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool timed = stats != nullptr;
    if (ctx->graph && !timed && !ctx->prof) rc = enqueue_graph(ctx, P, descs, w, s);
    else rc = enqueue(ctx, P, descs, w, s, timed, PH_ALL);
    if (rc) return rc;
    if (stats) {
        HIP_TRY(ctx, hipStreamSynchronize(s));
        rc = read_stats(ctx, P, w, timed, stats);
        if (rc) return rc;
    }
    return NKS_OK;
}

int nks_sign_apply(nks_ctx* ctx, nks_lattice* lat, const void* b, void* x, const nks_opts* opts, void* ws,
                   size_t ws_bytes, void* stream, nks_stats* stats) {
    nks_job j{lat, b, x, opts};
    return nks_sign_apply_batch(ctx, 1, &j, ws, ws_bytes, stream, stats);
}

int nks_sign_apply_noalloc(nks_ctx* ctx, nks_lattice* lat, const void* b, void* x, const nks_opts* opts, void* stream,
                           nks_stats* stats) {
    if (!ctx || !lat || !b || !x) return fail(ctx, NKS_E_INVALID, "NULL argument");
    nks_job j{lat, b, x, opts};
    Plan P;
    int rc = make_plan(ctx, 1, &j, P);
    if (rc) return rc;
    if (P.total > (size_t)NKS_NOALLOC_BYTES)
        return fail(ctx, NKS_E_NOMEM,
                    "nks_sign_apply_noalloc: this job needs " + std::to_string(P.total) +
                        " bytes of workspace, more than the NKS_NOALLOC_BYTES (" + std::to_string(NKS_NOALLOC_BYTES) +
                        ") the library holds per GPU; use NKS_FLAG_DOUBLE_PASS (O(n) memory) or nks_sign_apply "
                        "with a workspace of nks_workspace_size bytes");
    void* ws = nullptr;
    if (scratch_address(ctx->device, &ws)) return fail(ctx, NKS_E_HIP, "no scratch address for this GPU");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    char* w = static_cast<char*>(ws);
    std::vector<JobDesc>& descs = ctx->descs;
    descs.clear();
    descs.push_back(make_desc(ctx, P, P.jobs[0], w, b, x));
    hipStream_t s = static_cast<hipStream_t>(stream);
    // eager launches on the caller's stream only: one job is one lattice group,
    // so no side stream, no graph and nothing else is created or allocated
    rc = enqueue(ctx, P, descs, w, s, stats != nullptr, PH_ALL);
    if (rc) return rc;
    if (stats) {
        HIP_TRY(ctx, hipStreamSynchronize(s));
        rc = read_stats(ctx, P, w, true, stats);
        if (rc) return rc;
    }
    return NKS_OK;
}

int nks_outer_basis(nks_ctx* ctx, nks_lattice* lat, const void* b, const nks_opts* opts, void* ws, size_t ws_bytes,
                    void* stream, double* alpha_host, double* beta_host, double* gamma_host, nks_stats* stats) {
    if (!ctx || !lat || !b || !alpha_host || !beta_host || !gamma_host) return fail(ctx, NKS_E_INVALID, "NULL argument");
    nks_job j{lat, b, nullptr, opts};
    Plan P;
    int rc = make_plan(ctx, 1, &j, P);
    if (rc) return rc;
    if (!ws || ws_bytes < P.total) return fail(ctx, NKS_E_NOMEM, "workspace too small");
    char* w = static_cast<char*>(ws);
    std::vector<JobDesc> descs{make_desc(ctx, P, P.jobs[0], w, b, nullptr)};
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = enqueue(ctx, P, descs, w, s, false, PH_OUTER_ONLY);
    if (rc) return rc;
    HIP_TRY(ctx, hipStreamSynchronize(s));
    const JobPlan& jp = P.jobs[0];
    int st[ST_COUNT];
    HIP_TRY(ctx, hipMemcpy(st, w + jp.off_status, sizeof(st), hipMemcpyDeviceToHost));
    const int k = st[ST_KUSED];
    std::vector<double2> sc((size_t)SC_COUNT * (jp.k + 2));
    HIP_TRY(ctx, hipMemcpy(sc.data(), w + jp.off_sc, sizeof(double2) * sc.size(), hipMemcpyDeviceToHost));
    const size_t stride = jp.k + 2;
    for (int i = 0; i < jp.k; ++i) {
        double2 a = i < k ? sc[SC_ALPHA * stride + i + 1] : mk(0, 0);
        alpha_host[2 * i] = a.x;
        alpha_host[2 * i + 1] = a.y;
        if (i + 1 < jp.k) {
            double2 bb = i + 1 < k ? sc[SC_BETA * stride + i + 1] : mk(0, 0);
            double2 gg = i + 1 < k ? sc[SC_GAMMA * stride + i + 1] : mk(0, 0);
            beta_host[2 * i] = bb.x;
            beta_host[2 * i + 1] = bb.y;
            gamma_host[2 * i] = gg.x;
            gamma_host[2 * i + 1] = gg.y;
        }
    }
    if (stats) {
        nks_stats tmp[1];
        rc = read_stats(ctx, P, w, false, tmp);
        if (rc) return rc;
        *stats = tmp[0];
    }
    return NKS_OK;
}

int nks_nested_step(nks_ctx* ctx, int k, const double* alpha_host, const double* beta_host, const double* gamma_host,
                    int hermitian, const nks_opts* opts, double* c_host, nks_stats* stats) {
    if (!ctx || !alpha_host || !c_host || (k > 1 && (!beta_host || !gamma_host)))
        return fail(ctx, NKS_E_INVALID, "NULL argument");
    if (k < 1) return fail(ctx, NKS_E_INVALID, "k must be >= 1");
    int rc = validate_opts(ctx, opts);
    if (rc) return rc;
    if (opts->ell_policy == NKS_POLICY_LEARNED || opts->k_policy != NKS_POLICY_FIXED)
        return fail(ctx, NKS_E_UNSUPPORTED, "nks_nested_step takes FIXED k and a FIXED or DOUBLING ell policy");
    const int ell = even_up(opts->ell);
    if (ell >= k && k > NONNESTED_MAX) return fail(ctx, NKS_E_UNSUPPORTED, "non-nested mode limited to k <= 1024");
    if (ell < k && ell > RHI_MAX) return fail(ctx, NKS_E_UNSUPPORTED, "ell is limited to 1024");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    // a one-job layout: descriptor, scalars, status, report, omega, nest
    const size_t stride = (size_t)k + 2;
    const int lcap = ell >= k ? k : ell;
    size_t off = align_up(sizeof(JobDesc));
    const size_t off_sc = off; off = align_up(off + sizeof(double2) * SC_COUNT * stride);
    const size_t off_st = off; off = align_up(off + sizeof(int) * ST_COUNT);
    const size_t off_rp = off; off = align_up(off + sizeof(double) * RP_COUNT);
    const size_t off_om = off; off = align_up(off + sizeof(double2) * k);
    int levels, ell_deep[NKS_MAX_LEVELS - 1];
    double p_deep[NKS_MAX_LEVELS - 1];
    set_levels(levels, ell_deep, p_deep, opts);
    const size_t nwords = nest_words(k, ell, levels, ell_deep);
    const size_t off_ne = off; off = align_up(off + sizeof(double2) * nwords);
    char* w = nullptr;
    HIP_TRY(ctx, hipMalloc(&w, off));
    std::unique_ptr<char, decltype(&hipFree)> guard(w, &hipFree);
    std::vector<double2> sc(SC_COUNT * stride, mk(0, 0));
    for (int i = 0; i < k; ++i) {
        sc[SC_ALPHA * stride + i + 1] = mk(alpha_host[2 * i], hermitian ? 0.0 : alpha_host[2 * i + 1]);
        if (i + 1 < k) {
            sc[SC_BETA * stride + i + 1] = mk(beta_host[2 * i], hermitian ? 0.0 : beta_host[2 * i + 1]);
            sc[SC_GAMMA * stride + i + 1] =
                hermitian ? sc[SC_BETA * stride + i + 1] : mk(gamma_host[2 * i], gamma_host[2 * i + 1]);
        }
        sc[SC_SV * stride + i + 1] = mk(1.0, 0.0);
        sc[SC_SW * stride + i + 1] = mk(1.0, 0.0);
    }
    int st[ST_COUNT] = {0};
    st[ST_DONE] = 1;
    st[ST_KUSED] = k;
    double rp[RP_COUNT] = {0};
    rp[RP_BNORM] = 1.0;
    JobDesc d{};
    d.sc = reinterpret_cast<double2*>(w + off_sc);
    d.status = reinterpret_cast<int*>(w + off_st);
    d.report = reinterpret_cast<double*>(w + off_rp);
    d.omega = reinterpret_cast<double2*>(w + off_om);
    d.nest = reinterpret_cast<double2*>(w + off_ne);
    d.k = k;
    d.ell = ell;
    d.p = opts->p;
    d.max_rhi = opts->max_rhi_iter;
    d.rhi_tol = opts->rhi_tol;
    d.two_sided = !hermitian;
    d.nest_cap = (int)nwords;
    d.lcap = lcap;
    d.levels = levels;
    for (int i = 0; i + 1 < NKS_MAX_LEVELS; ++i) {
        d.ell_deep[i] = ell_deep[i];
        d.p_deep[i] = p_deep[i];
    }
    d.scstride = (int)stride;
    d.precision = NKS_FP64;
    d.k_policy = NKS_POLICY_FIXED;
    d.ell_policy = opts->ell_policy;
    d.tol = opts->tol;
    HIP_TRY(ctx, hipMemcpy(w, &d, sizeof(d), hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(w + off_sc, sc.data(), sizeof(double2) * sc.size(), hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(w + off_st, st, sizeof(st), hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(w + off_rp, rp, sizeof(rp), hipMemcpyHostToDevice));
    launch_nested(reinterpret_cast<JobDesc*>(w), 1, nullptr);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipDeviceSynchronize());
    HIP_TRY(ctx, hipMemcpy(c_host, w + off_om, sizeof(double2) * k, hipMemcpyDeviceToHost));
    if (stats) {
        HIP_TRY(ctx, hipMemcpy(st, w + off_st, sizeof(st), hipMemcpyDeviceToHost));
        HIP_TRY(ctx, hipMemcpy(rp, w + off_rp, sizeof(rp), hipMemcpyDeviceToHost));
        std::memset(stats, 0, sizeof(*stats));
        stats->status = st[ST_STATUS];
        stats->k_used = k;
        stats->ell_used = st[ST_ELL];
        stats->rhi_iters = st[ST_RHI];
        stats->p_used = rp[RP_P];
        stats->z_min = rp[RP_ZMIN];
        stats->z_max = rp[RP_ZMAX];
        stats->b_norm = 1.0;
        stats->inner_delta = rp[RP_INNER_DELTA];
        fill_level_stats(*stats, st, rp);
    }
    return NKS_OK;
}

int nks_mlp_forward(nks_ctx* ctx, const float* params, const float* x, int batch, float* y, void* stream) {
    if (!ctx || !params || !x || !y || batch < 1) return fail(ctx, NKS_E_INVALID, "bad nks_mlp_forward arguments");
    launch_mlp_forward(params, x, batch, y, static_cast<hipStream_t>(stream));
    HIP_TRY(ctx, hipGetLastError());
    return NKS_OK;
}

int nks_mlp_backward(nks_ctx* ctx, const float* params, const float* x, const float* t, int batch, float* grad,
                     float* loss, void* stream) {
    if (!ctx || !params || !x || !t || !grad || !loss || batch < 1)
        return fail(ctx, NKS_E_INVALID, "bad nks_mlp_backward arguments");
    launch_mlp_backward(params, x, t, batch, grad, loss, static_cast<hipStream_t>(stream));
    HIP_TRY(ctx, hipGetLastError());
    return NKS_OK;
}

int nks_mlp_adam_step(nks_ctx* ctx, float* params, const float* grad, float* m, float* v, int step, float lr,
                      void* stream) {
    if (!ctx || !params || !grad || !m || !v || step < 1) return fail(ctx, NKS_E_INVALID, "bad nks_mlp_adam_step arguments");
    launch_mlp_adam(params, grad, m, v, step, lr, static_cast<hipStream_t>(stream));
    HIP_TRY(ctx, hipGetLastError());
    return NKS_OK;
}

int nks_policy_load(nks_ctx* ctx, const float* blob, int nfloats) {
    if (!ctx || !blob) return fail(ctx, NKS_E_INVALID, "NULL argument");
    if (nfloats != NKS_POLICY_NFLOATS || sizeof(PolicyNet) != sizeof(float) * NKS_POLICY_NFLOATS)
        return fail(ctx, NKS_E_INVALID, "policy blob must hold NKS_POLICY_NFLOATS floats");
    for (int i = 0; i < nfloats; ++i)
        if (!(blob[i] == blob[i]) || blob[i] > 1e30f || blob[i] < -1e30f)
            return fail(ctx, NKS_E_INVALID, "policy blob holds a non-finite value");
    PolicyNet h;
    std::memcpy(&h, blob, sizeof(h));
    for (int i = 0; i < NFEAT; ++i)
        if (!(h.fstd[i] > 0.f)) return fail(ctx, NKS_E_INVALID, "feature scales must be > 0");
    for (int i = 0; i < 2; ++i)
        if (!(h.tstd[i] > 0.f)) return fail(ctx, NKS_E_INVALID, "target scales must be > 0");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (!ctx->net) HIP_TRY(ctx, hipMalloc(&ctx->net, sizeof(PolicyNet)));
    HIP_TRY(ctx, hipDeviceSynchronize());   // no call in flight may read the old network
    HIP_TRY(ctx, hipMemcpy(ctx->net, &h, sizeof(h), hipMemcpyHostToDevice));
    return NKS_OK;
}

int nks_policy_label(nks_ctx* ctx, int njobs, const nks_job* jobs, double* labels_host) {
    if (!ctx || !labels_host) return fail(ctx, NKS_E_INVALID, "NULL argument");
    if (njobs < 1 || !jobs) return fail(ctx, NKS_E_INVALID, "no jobs");
    for (int i = 0; i < njobs; ++i) {
        if (!jobs[i].b || !jobs[i].opts) return fail(ctx, NKS_E_INVALID, "job b or opts is NULL");
        if (jobs[i].opts->k_policy != NKS_POLICY_FIXED || jobs[i].opts->ell_policy != NKS_POLICY_FIXED)
            return fail(ctx, NKS_E_INVALID, "label runs take FIXED policies (the outer loop runs to opts.k)");
        // Two-sided label runs are switched off: one of them (4^4, mu = 0.3,
        // k = 400) faulted the GPU in the parallel label kernel and the cause is
        // not found yet.  Hermitian label runs are unaffected.
        if (jobs[i].lat && jobs[i].lat->mu != 0.0)
            return fail(ctx, NKS_E_UNSUPPORTED, "label runs at mu != 0 are switched off (unresolved GPU fault)");
    }
    Plan P;
    int rc = make_plan(ctx, njobs, jobs, P, true);
    if (rc) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    char* w = nullptr;
    HIP_TRY(ctx, hipMalloc(&w, P.total));
    std::unique_ptr<char, decltype(&hipFree)> guard(w, &hipFree);
    std::vector<JobDesc> descs;
    for (const auto& jp : P.jobs) descs.push_back(make_desc(ctx, P, jp, w, jobs[jp.idx].b, nullptr));
    rc = enqueue(ctx, P, descs, w, nullptr, false, PH_LABEL);
    if (rc) return rc;
    HIP_TRY(ctx, hipDeviceSynchronize());
    for (const auto& jp : P.jobs)
        HIP_TRY(ctx, hipMemcpy(labels_host + (size_t)jp.idx * LABEL_WORDS, w + jp.off_label,
                               sizeof(double) * LABEL_WORDS, hipMemcpyDeviceToHost));
    return NKS_OK;
}

int nks_tune_set(nks_ctx* ctx, const char* key, int value) {
    if (!ctx || !key) return NKS_E_INVALID;
    const std::string k(key);
    if (k == "xcd_map") {
        if (value < 0 || value > 3) return fail(ctx, NKS_E_INVALID, "xcd_map takes 0, 1, 2 or 3");
        ctx->tune.xcd_map = value;
    } else if (k == "split_dual") ctx->tune.split_dual = value != 0;
    else if (k == "min_waves") {
        if (value != 1 && value != 3 && value != 4) return fail(ctx, NKS_E_INVALID, "min_waves takes 1, 3 or 4");
        ctx->tune.min_waves = value;
    } else if (k == "collapse") {
        if (value < 1) return fail(ctx, NKS_E_INVALID, "collapse takes a block count >= 1");
        ctx->tune.collapse = value;
    } else if (k == "concurrent_groups") ctx->tune.concurrent = value != 0;
    else if (k == "pipeline_groups") ctx->tune.pipeline = value != 0;
    else if (k == "stagger_groups") {
        if (value < 0 || value > 100) return fail(ctx, NKS_E_INVALID, "stagger_groups takes 0..100 (percent)");
        ctx->tune.stagger = value;
    }
    else if (k == "graph") ctx->graph = value != 0;
    else return fail(ctx, NKS_E_INVALID, "unknown tuning key " + k);
    return NKS_OK;
}

int nks_tune_get(nks_ctx* ctx, const char* key, int* value) {
    if (!ctx || !key || !value) return NKS_E_INVALID;
    const std::string k(key);
    if (k == "xcd_map") *value = ctx->tune.xcd_map;
    else if (k == "split_dual") *value = ctx->tune.split_dual;
    else if (k == "min_waves") *value = ctx->tune.min_waves;
    else if (k == "collapse") *value = ctx->tune.collapse;
    else if (k == "concurrent_groups") *value = ctx->tune.concurrent;
    else if (k == "pipeline_groups") *value = ctx->tune.pipeline;
    else if (k == "stagger_groups") *value = ctx->tune.stagger;
    else if (k == "graph") *value = ctx->graph;
    else if (k == "graph_captures") *value = (int)ctx->graph_captures;
    else if (k == "graph_replays") *value = (int)ctx->graph_replays;
    else return fail(ctx, NKS_E_INVALID, "unknown tuning key " + k);
    return NKS_OK;
}

int nks_profile_enable(nks_ctx* ctx, int enable) {
    if (!ctx) return NKS_E_INVALID;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (enable && ctx->pool.empty() && ctx->pending.empty()) {
        for (size_t i = 0; i < PROF_POOL; ++i) {
            hipEvent_t e;
            HIP_TRY(ctx, hipEventCreate(&e));
            ctx->pool.push_back(e);
        }
    }
    ctx->prof = enable != 0;
    for (auto& c : ctx->prof_count) c = 0;
    return NKS_OK;
}

int nks_profile_read(nks_ctx* ctx, int kernel_class, int* launches, double* total_ms, double* alg_bytes) {
    if (!ctx || kernel_class < 0 || kernel_class >= NKS_K_COUNT || !launches || !total_ms || !alg_bytes)
        return fail(ctx, NKS_E_INVALID, "bad nks_profile_read arguments");
    int n = 0;
    double ms = 0.0, bytes = 0.0;
    std::vector<ProfRecord> keep;
    for (auto& r : ctx->pending) {
        if (r.cls != kernel_class) { keep.push_back(r); continue; }
        HIP_TRY(ctx, hipEventSynchronize(r.b));
        float t = 0.f;
        HIP_TRY(ctx, hipEventElapsedTime(&t, r.a, r.b));
        ++n;
        ms += t;
        bytes += r.bytes;
        ctx->pool.push_back(r.a);
        ctx->pool.push_back(r.b);
    }
    ctx->pending.swap(keep);
    *launches = n;
    *total_ms = ms;
    *alg_bytes = bytes;
    return NKS_OK;
}

}  // extern "C"
