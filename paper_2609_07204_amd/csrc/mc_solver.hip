// Host driver and C ABI of the minimum-cut library.
//
// mc_mincut runs Algorithm 2 of the paper on the device:
//   normalise the input (contraction by the identity), lambda-hat <- minimum
//   degree (Section 2 "Basic Concepts"), connectivity check (lambda = 0),
//   then rounds of { reduction tests 1-2, parallel CAPFOREST passes,
//   sequential CAPFOREST if nothing was marked, union-find relabel,
//   contraction, collapsed degrees as bounds } until at most two vertices
//   remain. The host only launches kernels and reads back a few scalars per
//   round; every step of the path runs in the kernels of this library.
//
// The side of the cut is tracked without keeping old graphs (paper,
// Section 4, session 1 item 2): map0 sends every input vertex to its
// current vertex, and whenever lambda-hat strictly drops the side is
// snapshot from the vertex or scanned prefix that produced the new bound.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mc_internal.h"
#include "mincut_steps.h"

namespace {

inline int grid_for(int64_t count, int threads, int cap = 8192) {
    int64_t b = (count + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

__global__ void k_set_lam(DevScalars* sc, int64_t lam) { sc->lam = lam; }
__global__ void k_reset_round(DevScalars* sc) {
    sc->marks_pr = 0;
    sc->marks_cf = 0;
    sc->marks_tri = 0;
    sc->err = 0;
    sc->best_pass = -1;
    sc->best_alpha = INT64_MAX;
}
__global__ void k_uf_pairs(const int32_t* a, const int32_t* b, int64_t np, int32_t* par) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x)
        uf_union(par, a[i], b[i]);
}

uint64_t splitmix_host(uint64_t x) {
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}

mc_status fail(mc_status code, const std::string& msg) { return mc_fail(code, msg); }

}  // namespace

bool mc_hip_ok(hipError_t e, const char* what) {
    if (e == hipSuccess) return true;
    mc_error_slot() = std::string(what) + ": " + hipGetErrorString(e);
    return false;
}

// ------------------------------------------------------------ profiling
namespace {
struct Prof {
    bool on = false;
    unsigned long long* dbytes = nullptr;   // device counters [PK_COUNT]
    double hbytes[PK_COUNT] = {};
    int64_t launches[PK_COUNT] = {};
    double ms[PK_COUNT] = {};
    hipEvent_t open[PK_COUNT] = {};      // start event of the launch in flight
    hipEvent_t close[PK_COUNT] = {};     // its end event, taken before the launch
    std::vector<hipEvent_t> pool;
    struct Pending { int k; hipEvent_t a, b; };
    std::vector<Pending> pending;
    struct Round { int32_t kind, n_in, n_out; int64_t m_in, m_out; hipEvent_t a, b; };
    std::vector<Round> rounds;   // of the last solve
    bool round_open = false;

    hipEvent_t take() {
        hipEvent_t e = nullptr;
        if (!pool.empty()) { e = pool.back(); pool.pop_back(); return e; }
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    // fold finished event pairs into the totals (the stream has been synchronised)
    void resolve() {
        for (const Pending& p : pending) {
            float t = 0.f;
            if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&t, p.a, p.b) == hipSuccess)
                ms[p.k] += t;
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pending.clear();
    }
    // a new solve: the last solve's round events go back to the pool
    void clear_rounds() {
        for (const Round& r : rounds) {
            if (r.a) pool.push_back(r.a);
            if (r.b) pool.push_back(r.b);
        }
        rounds.clear();
        round_open = false;
    }
    ~Prof() {
        clear_rounds();
        for (const Pending& p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        if (dbytes) (void)hipFree(dbytes);
    }
};
thread_local Prof* g_prof = nullptr;   // the profiler of the solve running on this thread
constexpr size_t kProfCounterBytes = sizeof(unsigned long long) * PK_COUNT * PROF_LANES * PROF_STRIDE;

const char* const kProfNames[PK_COUNT] = {"k_cfs_edges",    "k_merge_small", "k_big_insert", "k_group_count",
                                          "k_group_scatter", "k_pr12",       "k_uf_link_rest", "k_lp_flat",
                                          "k_lp_first",     "k_mid_merge",   "k_pr1_first",  "k_pr1_rest"};

// sets g_prof for the duration of one call and resolves its events at the end
struct ProfScope {
    explicit ProfScope(Prof* p) { g_prof = p && p->on ? p : nullptr; }
    ~ProfScope() {
        if (g_prof) g_prof->resolve();
        g_prof = nullptr;
    }
};
}  // namespace

// Both events of a launch are taken before it is issued, so nothing slow
// (an event creation) sits between the kernel and its end event.
void prof_begin(int k, hipStream_t s) {
    Prof* p = g_prof;
    if (!p) return;
    hipEvent_t a = p->take(), b = p->take();
    if (!a || !b || hipEventRecord(a, s) != hipSuccess) {
        if (a) p->pool.push_back(a);
        if (b) p->pool.push_back(b);
        a = b = nullptr;
    }
    p->open[k] = a;
    p->close[k] = b;
}

void prof_end(int k, hipStream_t s) {
    Prof* p = g_prof;
    if (!p || !p->open[k]) return;
    if (hipEventRecord(p->close[k], s) != hipSuccess) {
        p->pool.push_back(p->open[k]);
        p->pool.push_back(p->close[k]);
    } else {
        p->pending.push_back({k, p->open[k], p->close[k]});
        p->launches[k]++;
    }
    p->open[k] = p->close[k] = nullptr;
}

unsigned long long* prof_dev_bytes(int k) {
    return g_prof ? g_prof->dbytes + (size_t)k * PROF_LANES * PROF_STRIDE : nullptr;
}

void prof_host_bytes(int k, double bytes) {
    if (g_prof) g_prof->hbytes[k] += bytes;
}

// round records: a round left open (no contraction followed) closes with
// its input sizes when the next one begins
void prof_round_end(int32_t n_out, int64_t m_out, hipStream_t s) {
    Prof* p = g_prof;
    if (!p || !p->round_open) return;
    Prof::Round& r = p->rounds.back();
    r.b = p->take();
    if (r.b) (void)hipEventRecord(r.b, s);
    r.n_out = n_out;
    r.m_out = m_out;
    p->round_open = false;
}

void prof_round_begin(int32_t kind, int32_t n, int64_t m, hipStream_t s) {
    Prof* p = g_prof;
    if (!p) return;
    if (p->round_open) prof_round_end(p->rounds.back().n_in, p->rounds.back().m_in, s);
    Prof::Round r{kind, n, n, m, m, p->take(), nullptr};
    if (r.a) (void)hipEventRecord(r.a, s);
    p->rounds.push_back(r);
    p->round_open = true;
}


// ------------------------------------------ static scratch (no allocation)
// Workspace of mc_mincut_static: a file-scope device array, one copy on each
// GPU the library runs on, held until the process ends. In host code its
// name is only a host-side stand-in, never a device address: the address
// comes from hipGetSymbolAddress, taken once per device (with that device
// current) when the first context on the device is created, and only that
// address is handed to kernels and copies.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the device address of this device's copy (device current); nullptr and
// the error set on failure
void* scratch_address(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) {
        fail(MC_E_DEVICE, "static scratch: device index out of range");
        return nullptr;
    }
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            fail(MC_E_DEVICE, std::string("hipGetSymbolAddress of the static scratch failed: ") + hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[device] = p;
    }
    return g_scratch_ptr[device];
}
}  // namespace

extern "C" mc_status mc_ctx_create(int device, void* hip_stream, const mc_options* opt, mc_ctx** out) {
    if (!out) return fail(MC_E_INVALID_ARG, "mc_ctx_create: out is NULL");
    if (opt && mc_options_check(opt) != MC_OK) return MC_E_INVALID_ARG;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return fail(MC_E_DEVICE, "mc_ctx_create: no such HIP device");
    mc_ctx* c = new (std::nothrow) mc_ctx();
    if (!c) return fail(MC_E_OOM, "mc_ctx_create: out of host memory");
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (opt) c->opt = *opt; else mc_default_options(&c->opt);
    if (hipSetDevice(device) != hipSuccess) { delete c; return fail(MC_E_DEVICE, "hipSetDevice failed"); }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->cus = prop.multiProcessorCount;
    c->scratch = scratch_address(device);
    if (!c->scratch) { delete c; return MC_E_DEVICE; }
    if (hipHostMalloc((void**)&c->hsc, sizeof(DevScalars), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return fail(MC_E_DEVICE, "hipHostMalloc failed");
    }
    *out = c;
    return MC_OK;
}

extern "C" mc_status mc_ctx_destroy(mc_ctx* c) {
    if (!c) return MC_OK;
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->hsc) (void)hipHostFree(c->hsc);
    delete static_cast<Prof*>(c->prof);
    delete c;
    return MC_OK;
}

extern "C" mc_status mc_profile(mc_ctx* c, int32_t on) {
    if (!c) return fail(MC_E_INVALID_ARG, "mc_profile: ctx is NULL");
    if (hipSetDevice(c->device) != hipSuccess) return fail(MC_E_DEVICE, "hipSetDevice failed");
    if (!on) {
        if (c->prof) static_cast<Prof*>(c->prof)->on = false;
        return MC_OK;
    }
    if (!c->prof) {
        Prof* np = new (std::nothrow) Prof();
        if (!np) return fail(MC_E_OOM, "mc_profile: out of host memory");
        if (hipMalloc((void**)&np->dbytes, kProfCounterBytes) != hipSuccess) {
            delete np;
            return fail(MC_E_DEVICE, "mc_profile: hipMalloc of the byte counters failed");
        }
        c->prof = np;
    }
    Prof* p = static_cast<Prof*>(c->prof);
    if (hipMemsetAsync(p->dbytes, 0, kProfCounterBytes, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(MC_E_DEVICE, "mc_profile: clearing the byte counters failed");
    for (int k = 0; k < PK_COUNT; k++) { p->hbytes[k] = 0; p->launches[k] = 0; p->ms[k] = 0; }
    // events for a few solves up front: creating one inside a timed solve
    // would delay the host between launches
    while (p->pool.size() < 512) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return fail(MC_E_DEVICE, "mc_profile: hipEventCreate failed");
        p->pool.push_back(e);
    }
    p->on = true;
    return MC_OK;
}

extern "C" mc_status mc_profile_read(mc_ctx* c, int32_t kernel, mc_kernel_time* out) {
    if (!c || !out) return fail(MC_E_INVALID_ARG, "mc_profile_read: NULL argument");
    if (kernel < 0 || kernel >= PK_COUNT) return fail(MC_E_INVALID_ARG, "mc_profile_read: no such kernel");
    std::memset(out, 0, sizeof(*out));
    std::snprintf(out->name, sizeof(out->name), "%s", kProfNames[kernel]);
    if (!c->prof) return MC_OK;
    Prof* p = static_cast<Prof*>(c->prof);
    std::vector<unsigned long long> db(kProfCounterBytes / sizeof(unsigned long long));
    if (hipSetDevice(c->device) != hipSuccess ||
        hipMemcpy(db.data(), p->dbytes, kProfCounterBytes, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(MC_E_DEVICE, "mc_profile_read: reading the byte counters failed");
    double dev_bytes = 0;
    for (int i = 0; i < PROF_LANES; i++) dev_bytes += (double)db[((size_t)kernel * PROF_LANES + i) * PROF_STRIDE];
    out->launches = p->launches[kernel];
    out->ms = p->ms[kernel];
    out->bytes = dev_bytes + p->hbytes[kernel];
    return MC_OK;
}

extern "C" mc_status mc_profile_round(mc_ctx* c, int32_t i, mc_round_time* out, int32_t* count) {
    if (!c || !count) return fail(MC_E_INVALID_ARG, "mc_profile_round: NULL argument");
    *count = 0;
    if (!c->prof) return MC_OK;
    Prof* p = static_cast<Prof*>(c->prof);
    *count = (int32_t)p->rounds.size();
    if (i < 0 || i >= *count || !out) return MC_OK;
    const Prof::Round& r = p->rounds[(size_t)i];
    std::memset(out, 0, sizeof(*out));
    out->kind = r.kind;
    out->n_in = r.n_in;
    out->m_in = r.m_in;
    out->n_out = r.n_out;
    out->m_out = r.m_out;
    float t = 0.f;
    if (hipSetDevice(c->device) != hipSuccess) return fail(MC_E_DEVICE, "hipSetDevice failed");
    if (r.a && r.b && hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess)
        out->ms = t;
    return MC_OK;
}

extern "C" mc_status mc_ctx_set_options(mc_ctx* c, const mc_options* opt) {
    if (!c || !opt) return fail(MC_E_INVALID_ARG, "mc_ctx_set_options: NULL argument");
    if (mc_options_check(opt) != MC_OK) return MC_E_INVALID_ARG;
    c->opt = *opt;
    return MC_OK;
}

namespace {

// All device buffers of one solve, carved from the caller's workspace.
struct SolveWS {
    int32_t* in_rp = nullptr;
    int32_t* in_col = nullptr;
    int64_t* in_w = nullptr;
    DGraph g[3];
    int32_t* L = nullptr;
    int32_t* parent = nullptr;
    int32_t* flag = nullptr;
    uint8_t* flag8 = nullptr;
    int32_t* claim = nullptr;
    int32_t* map0 = nullptr;
    uint8_t* side = nullptr;
    ContractWS cw;
    int32_t passes = 0;
    int32_t* order = nullptr;
    int32_t* nscan = nullptr;
    int64_t* alpha = nullptr;
    int32_t* alen = nullptr;
    int64_t* lamout = nullptr;
    int32_t* cst = nullptr;
    int64_t* cr = nullptr;
    int64_t* cl1 = nullptr;
    int32_t* corder = nullptr;
    int32_t* cnscan = nullptr;
    int64_t* calpha = nullptr;
    int32_t* calen = nullptr;
    int64_t* clamout = nullptr;
    Pr12WS prw{};
    Pr34WS tw{};                  // reduction tests 3 and 4
    LpWS lw{};                    // label propagation of the heuristic
    int32_t* lab2 = nullptr;      // second label array of the synchronous rounds
    PrivateArgs pv{};             // per-pass arrays of the private passes
    StepArgs sa{};                // control of the level-synchronous form
    int32_t* psteps = nullptr;
    DevScalars* sc = nullptr;
    unsigned long long* vpart = nullptr;
    int32_t* vpart_i32() { return reinterpret_cast<int32_t*>(vpart); }
    int64_t* fin64 = nullptr;     // [2] finisher: bound in, bound out
    int32_t* fin32 = nullptr;     // [4] finisher: dropped, rounds, error, work-queue ticket
    int32_t* fx_col[2] = {nullptr, nullptr};   // finisher scratch graphs
    int64_t* fx_w[2] = {nullptr, nullptr};
};

void carve_graph(Arena& a, int32_t n, int64_t cap, DGraph& g) {
    g.n = n;
    g.cap = cap;
    g.off = a.take<int32_t>((size_t)n + 1);
    g.len = a.take<int32_t>((size_t)n + 1);
    g.deg = a.take<int64_t>((size_t)n + 1);
    g.col = a.take<int32_t>((size_t)cap + 1);
    g.w = a.take<int64_t>((size_t)cap + 1);
}

void carve_steps(Arena& a, int32_t n, int64_t cap, int32_t passes, int32_t len_cap, StepArgs& sa) {
    sa.ctl = a.take<StepCtl>((size_t)passes);
    sa.bcap = len_cap > 0 && len_cap < n ? len_cap : n;
    const size_t per = (size_t)sa.bcap + 1;
    const size_t total = std::max((size_t)passes * per, (size_t)n + 1);
    sa.bpre = a.take<int32_t>(total);
    sa.single = a.take<int32_t>((size_t)passes);
    sa.ptile = a.take<int32_t>((size_t)passes + 1);
    sa.running = a.take<int32_t>(1);
    sa.popk = a.take<int64_t>((size_t)passes * 512);
    sa.popv = a.take<int32_t>((size_t)passes * 512);
    sa.spread = a.take<unsigned long long>((size_t)passes * SPREAD * SPREAD_STRIDE);
    sa.hid = a.take<int32_t>((size_t)n);
    sa.max_hubs = (int32_t)std::min<int64_t>(n, cap / HUB_LEN + 1);
    sa.hv = a.take<int32_t>((size_t)sa.max_hubs);
    sa.nhub = a.take<int32_t>(1);
    sa.hacc = a.take<unsigned long long>((size_t)passes * sa.max_hubs * HUB_SLOTS * 2);
    // a step's batches hold at most every row once per pass: entries <= cap
    // per pass, in 1024-entry tiles
    sa.max_tiles = (int64_t)passes * (cap / 1024 + 2);
    sa.tinfo = a.take<int32_t>((size_t)(2 * sa.max_tiles));
    sa.max_singles = 0;
}

// Per-pass state of the private passes: `passes` passes over graphs of at
// most n vertices, and (small > passes) up to `small` passes over graphs of
// at most small_n vertices. A launch sets the stride to its current graph's
// n, so the same region holds few passes over a large graph or many over a
// small one.
void carve_private(Arena& a, int32_t n, int32_t passes, PrivateArgs& pv, int32_t*& psteps, int32_t small = 0,
                   int32_t small_n = 0) {
    const int32_t pmax = std::max(passes, small);
    pv.passes = pmax;
    pv.stride = n;
    pv.region = std::max((int64_t)passes * n, (int64_t)small * small_n);
    pv.stride1 = (int64_t)n / 64 + 2;
    pv.region1 = std::max((int64_t)passes * pv.stride1, (int64_t)small * ((int64_t)small_n / 64 + 2));
    const size_t cnt = (size_t)pv.region;
    pv.st = a.take<int32_t>(cnt);
    pv.r = a.take<int64_t>(cnt);
    pv.fifo = a.take<int32_t>(cnt);
    pv.touched = a.take<int32_t>(cnt);
    pv.order = a.take<int32_t>(cnt);
    pv.l1 = a.take<int64_t>((size_t)pv.region1);
    pv.dlist = a.take<int32_t>((size_t)pv.region1);
    pv.dbits = a.take<uint32_t>((size_t)(pv.region1 / 32 + pmax + 1));
    pv.nscan = a.take<int32_t>((size_t)pmax);
    pv.alpha = a.take<int64_t>((size_t)pmax);
    pv.alpha_len = a.take<int32_t>((size_t)pmax);
    pv.lam_out = a.take<int64_t>((size_t)pmax);
    psteps = a.take<int32_t>((size_t)pmax);
    pv.diag = a.take<int64_t>((size_t)pmax * 8);
}

void carve(Arena& a, int32_t n, int64_t cap, int32_t passes, int32_t ppasses, int32_t len_cap, bool host_input,
           int ngraphs, SolveWS& w, int32_t small = 0, int32_t small_n = 0, bool sort = false) {
    w.sc = a.take<DevScalars>(1);
    if (host_input) {
        w.in_rp = a.take<int32_t>((size_t)n + 1);
        w.in_col = a.take<int32_t>((size_t)cap + 1);
        w.in_w = a.take<int64_t>((size_t)cap + 1);
    }
    for (int k = 0; k < ngraphs; k++) carve_graph(a, n, cap, w.g[k]);
    w.L = a.take<int32_t>((size_t)n + 1);
    w.parent = a.take<int32_t>((size_t)n + 1);
    w.flag = a.take<int32_t>((size_t)n + 2);
    w.flag8 = a.take<uint8_t>((size_t)n + 1);
    w.claim = a.take<int32_t>((size_t)n + 1);
    w.map0 = a.take<int32_t>((size_t)n + 1);
    w.side = a.take<uint8_t>((size_t)n + 1);
    contract_ws_carve(a, n, cap, w.cw, sort);
    pr12_ws_carve(a, n, cap, w.prw);
    w.passes = passes;
    w.order = a.take<int32_t>((size_t)passes * CF_HC);
    w.nscan = a.take<int32_t>((size_t)passes);
    w.alpha = a.take<int64_t>((size_t)passes);
    w.alen = a.take<int32_t>((size_t)passes);
    w.lamout = a.take<int64_t>((size_t)passes);
    w.cst = a.take<int32_t>((size_t)n + 1);
    w.cr = a.take<int64_t>((size_t)n + 1);
    w.cl1 = a.take<int64_t>((size_t)n / 64 + 2);
    w.corder = a.take<int32_t>((size_t)n + 1);
    w.cnscan = a.take<int32_t>(1);
    w.calpha = a.take<int64_t>(1);
    w.calen = a.take<int32_t>(1);
    w.clamout = a.take<int64_t>(1);
    w.vpart = a.take<unsigned long long>(1024);
    w.fin64 = a.take<int64_t>(2);
    w.fin32 = a.take<int32_t>(4);
    // a simple graph of at most FIN_N vertices has at most FIN_N (FIN_N - 1)
    // entries, and never more than the input
    const int64_t fx = std::min<int64_t>(cap, (int64_t)FIN_N * (FIN_N - 1)) + 1;
    for (int q = 0; q < 2; q++) {
        w.fx_col[q] = a.take<int32_t>((size_t)fx);
        w.fx_w[q] = a.take<int64_t>((size_t)fx);
    }
    lp_ws_carve(a, n, cap, w.lw);
    pr34_ws_carve(a, n, w.tw);
    w.lab2 = a.take<int32_t>((size_t)n + 1);
    carve_private(a, n, ppasses, w.pv, w.psteps, small, small_n);
    carve_steps(a, n, cap, ppasses, len_cap, w.sa);
}

// passes of the shared-visited-array form (one wavefront each)
int32_t pass_count(const mc_ctx* c) {
    if (c->opt.capforest_mode == MC_CF_PRIVATE || c->opt.deterministic) return 1;
    int32_t p = c->opt.capforest_passes;
    if (p <= 0) p = 4 * c->cus;
    return p;
}

// passes of the private form. Graphs large enough for the whole-GPU step
// form run one long pass (measured fastest on power-law graphs: every pass
// repeats the traversal of the dense core); smaller graphs run one
// workgroup per pass, so several passes keep several compute units busy.
int32_t levels_min_n(const mc_ctx* c) { return c->opt.levels_min_n > 0 ? c->opt.levels_min_n : (1 << 16); }

// passes used on a current graph with n vertices (the first round of the
// small-graph regime; see small_pass_max)
int32_t private_pass_count(const mc_ctx* c, int32_t n) {
    if (c->opt.capforest_mode == MC_CF_SHARED || c->opt.deterministic) return 1;
    if (c->opt.capforest_passes > 0) return c->opt.capforest_passes;
    return n >= levels_min_n(c) ? 1 : 32;
}

// passes the workspace holds at the stride of the input (rounds on graphs
// of at least levels_min_n vertices, and the complete fallback pass)
int32_t large_pass_count(const mc_ctx* c) { return private_pass_count(c, levels_min_n(c)); }

// Small-graph rounds start with 32 passes; a round that removes fewer than
// one vertex in ten raises the count to one pass per compute unit for the
// rest of the solve. On graphs that resist contraction each pass marks a
// few edges and the passes run side by side on idle compute units, so more
// passes mean proportionally fewer rounds (20,000-vertex 6-regular graphs
// with three hubs: 152 rounds and 17.7 s with 32 passes, 37 rounds and
// 3.5 s with 256).
int32_t small_pass_max(const mc_ctx* c) {
    if (c->opt.capforest_mode == MC_CF_SHARED || c->opt.deterministic || c->opt.capforest_passes > 0)
        return private_pass_count(c, 2);
    return std::max(32, c->cus);
}
int32_t small_pass_n(const mc_ctx* c, int32_t n) { return std::min(n, levels_min_n(c) - 1); }

int32_t private_len_cap(const mc_ctx* c) {
    if (c->opt.pass_len_cap < 0) return 0;
    if (c->opt.pass_len_cap > 0) return c->opt.pass_len_cap;
    return 32768;
}

// CAPFOREST form a round ran (whose pass orders hold its best prefix)
enum { CF_RUN_NONE = 0, CF_RUN_SEQ, CF_RUN_SHARED, CF_RUN_PRIVATE };

struct Solver {
    mc_ctx* c;
    hipStream_t s;
    SolveWS w;
    int cf_choice[2] = {CF_RUN_NONE, CF_RUN_NONE};   // automatic mode: kept form per size regime
    int32_t n0 = 0;
    int64_t lam = 0;
    bool debug = false;
    bool tri_on = false;          // reduction tests 3 and 4 still pay off
    bool in_heuristic = false;    // exact rounds on the heuristic's coarse graph
    bool conn_pending = false;    // connectivity not decided yet (the heuristic's coarse graph decides it)
    bool lp1_ready = false;       // the input pass left the first LP round of the input in lab2
    bool disconnected = false;    // lambda = 0; the side is set
    bool pv_clean = false;        // private pass state cleared (once per solve, before the first private pass)
    int32_t small_max = 32;       // passes of small rounds the workspace holds
    int32_t small_passes = 0;     // passes of small rounds now (0: the first round's count)
    int64_t pv_stride = 0;        // stride of the last private launch (its pass orders)
    int64_t cur_m = 0;            // entries of the current graph
    int32_t last_cf_steps = 0;    // whole-GPU steps of the round's last CAPFOREST launch
    int64_t last_cf_scans = 0;    // and the vertices it scanned
    mc_stats stats{};

    // Reduction tests of one round on g into parent (reset beforehand):
    // tests 1 and 2, then tests 3 and 4 while they keep finding at least
    // one contraction per 100 vertices (as repeated linear sweeps stop once
    // they stop shrinking the graph, App. A).
    bool reduction_tests(const DGraph& g) {
        const bool tri = tri_on && c->opt.pr_tri_deg_cap > 0;
        if (!pr12(g, &w.sc->lam, w.parent, &w.sc->marks_pr, nullptr, tri ? w.tw.ptr2 : nullptr, w.prw, s))
            return false;
        if (!tri) return true;
        if (!pr34(g, &w.sc->lam, c->opt.pr_tri_deg_cap, w.parent, &w.sc->marks_tri, w.tw.ptr2, w.tw, nullptr,
                  nullptr, s))
            return false;
        return true;
    }
    // after the round's readback: fold the test-3/4 marks into the PR count
    void tri_account(int32_t n) {
        if (!tri_on || c->opt.pr_tri_deg_cap <= 0) return;
        const unsigned long long t = c->hsc->marks_tri;
        stats.marks_tri += (int64_t)t;
        if (t * 100 < (unsigned long long)n) tri_on = false;
    }

    // passes of the private form on an n-vertex round
    int32_t passes_for(int32_t n) const {
        const int32_t base = private_pass_count(c, n);
        if (n >= levels_min_n(c) || c->opt.capforest_passes > 0 || base == 1 || small_passes <= 0) return base;
        return std::min(small_passes, small_max);
    }

    bool readback() {
        MC_HIP(hipMemcpyAsync(c->hsc, w.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
        MC_HIP(hipStreamSynchronize(s));
        return true;
    }
    // After a readback: the best proper-prefix alpha of the form that ran
    // last, if below the bound, becomes the bound and its prefix the side.
    bool apply_alpha(int used, int32_t n) {
        const DevScalars& h = *c->hsc;
        if (used == CF_RUN_NONE || h.best_pass < 0 || h.best_alpha >= lam) return true;
        const int32_t* pref = used == CF_RUN_SEQ      ? w.corder
                              : used == CF_RUN_SHARED ? w.order + (int64_t)h.best_pass * CF_HC
                                                      : w.pv.order + (int64_t)h.best_pass * pv_stride;
        if (!side_from_prefix(w.side, w.map0, n0, w.flag8, n, pref, &w.sc->best_len, s)) return false;
        return set_lam(h.best_alpha);
    }
    bool set_lam(int64_t v) {
        lam = v;
        k_set_lam<<<1, 1, 0, s>>>(w.sc, v);
        MC_LAUNCHED("k_set_lam");
        return true;
    }
};

}  // namespace

// bytes of a solve's workspace with room for `small` passes of small rounds
static size_t workspace_bytes(const mc_ctx* c, int32_t n, int32_t nnz, int32_t small) {
    Arena a;
    SolveWS w;
    carve(a, n, nnz, pass_count(c), large_pass_count(c), private_len_cap(c), true, 3, w, small,
          small_pass_n(c, n), c->opt.contract_mode == 1);
    return a.used + 256;
}

size_t workspace_min_bytes(const mc_ctx* c, int32_t n, int32_t nnz) {
    return workspace_bytes(c, n, nnz, private_pass_count(c, 2));
}

extern "C" mc_status mc_workspace_size(const mc_ctx* c, int32_t n, int32_t nnz, size_t* bytes) {
    if (!c || !bytes) return fail(MC_E_INVALID_ARG, "mc_workspace_size: NULL argument");
    if (n < 2 || nnz < 0) return fail(MC_E_INVALID_ARG, "mc_workspace_size: need n >= 2 and nnz >= 0");
    *bytes = workspace_bytes(c, n, nnz, small_pass_max(c));
    return MC_OK;
}

// MC_DEBUG=1: one line per round on stderr (sizes, marks, pass counters).
static void debug_round(Solver& S, const DGraph& g, int32_t round, int32_t passes) {
    DevScalars h = *S.c->hsc;
    std::vector<int64_t> d((size_t)std::max(passes, 1) * 8, 0);
    std::vector<int32_t> len((size_t)g.n);
    if (passes > 0) (void)hipMemcpy(d.data(), S.w.pv.diag, d.size() * sizeof(int64_t), hipMemcpyDeviceToHost);
    (void)hipMemcpy(len.data(), g.len, len.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
    int64_t nnz = 0;
    for (int32_t v : len) nnz += v;
    int64_t mx[8] = {0}, sum[8] = {0};
    for (int32_t p = 0; p < passes; p++)
        for (int k = 0; k < 8; k++) { mx[k] = std::max(mx[k], d[p * 8 + k]); sum[k] += d[p * 8 + k]; }
    int clk = 100000;
    (void)hipDeviceGetAttribute(&clk, hipDeviceAttributeWallClockRate, S.c->device);
    fprintf(stderr,
            "[mc] round %d n=%d nnz=%lld lam=%lld marks_pr=%llu marks_cf=%llu | passes=%d steps max %lld singles max %lld "
            "touched max %lld entries sum %lld max %lld | pop ms max %.3f batch ms max %.3f | scans max %lld maxbatch %lld\n",
            round, g.n, (long long)nnz, (long long)S.lam, h.marks_pr, h.marks_cf, passes, (long long)mx[0],
            (long long)mx[1], (long long)mx[2], (long long)sum[3], (long long)mx[3], mx[4] / (double)clk,
            mx[5] / (double)clk, (long long)mx[6], (long long)mx[7]);
}

// The shared-visited-array passes of Algorithm 1 as printed: many passes,
// one wavefront each, that blacklist vertices another pass scanned. A probe
// runs kProbePasses passes per compute unit of at most kProbeScans pops
// (scans or blacklistings) each, 32 K pops on 256 compute units. The passes
// run side by side while the pops of a pass are a chain, so four short
// passes per unit take about a quarter of the time of one pass four times as
// long (Chung-Lu 2^22: 256 passes of 128 pops took 0.69 ms).
constexpr int32_t kProbeScans = 32;
constexpr int32_t kProbePasses = 4;
constexpr int32_t kProbePrivate = 4096;   // scans per private pass in a probe round
static bool shared_passes(Solver& S, const DGraph& g, bool probe) {
    SolveWS& w = S.w;
    CapforestArgs ca{};
    ca.g = g;
    ca.lam = &w.sc->lam;
    ca.parent = w.parent;
    ca.claim = w.claim;
    ca.tag = ++S.c->tag;
    ca.shared = 1;
    ca.passes = probe ? std::min(w.passes, kProbePasses * S.c->cus) : w.passes;
    ca.len_cap = S.c->opt.pass_len_cap > 0 ? S.c->opt.pass_len_cap : 0;
    if (probe && (ca.len_cap <= 0 || ca.len_cap > kProbeScans)) ca.len_cap = kProbeScans;
    ca.pop_cap = probe ? kProbeScans : 0;
    ca.seed = S.c->opt.seed;
    ca.start = -1;
    ca.order = w.order;
    ca.nscan = w.nscan;
    ca.alpha = w.alpha;
    ca.alpha_len = w.alen;
    ca.lam_out = w.lamout;
    ca.marks = &w.sc->marks_cf;
    return capforest_passes(ca, S.s) && capforest_reduce(ca, w.sc, S.s);
}

// One sequential single-pop pass over g (deterministic), results in sc.
static bool sequential_pass(Solver& S, const DGraph& g, int32_t round) {
    SolveWS& w = S.w;
    CompleteArgs cp{};
    cp.g = g;
    cp.lam = &w.sc->lam;
    cp.parent = w.parent;
    cp.start = (int32_t)(splitmix_host(S.c->opt.seed ^ (uint64_t)round) % (uint64_t)g.n);
    cp.tag = ++S.c->tag;
    cp.st = w.cst;
    cp.r = w.cr;
    cp.l1 = w.cl1;
    cp.order = w.corder;
    cp.nscan = w.cnscan;
    cp.alpha = w.calpha;
    cp.alpha_len = w.calen;
    cp.lam_out = w.clamout;
    cp.marks = &w.sc->marks_cf;
    if (!capforest_complete(cp, S.s)) return false;
    CapforestArgs ra{};
    ra.alpha = w.calpha;
    ra.alpha_len = w.calen;
    ra.passes = 1;
    return capforest_reduce(ra, w.sc, S.s);
}

// `passes` private batched passes over g (len_cap 0: complete), results in sc.
// the context's private stream for graph capture (null: capture off, or the
// stream could not be made)
static hipStream_t capture_stream(mc_ctx* c) {
    if (c->graphs_off) return nullptr;
    if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        c->cap_stream = nullptr;
        c->graphs_off = true;
        (void)hipGetLastError();
    }
    return c->cap_stream;
}

static bool private_passes(Solver& S, const DGraph& g, int32_t round, int32_t passes, int32_t len_cap) {
    SolveWS& w = S.w;
    // every pass leaves its state cleared, so one clear per solve suffices,
    // and a solve whose rounds never run a private pass needs none
    if (!S.pv_clean) {
        if (!capforest_private_reset(w.pv, S.s)) return false;
        S.pv_clean = true;
    }
    if (len_cap > 0) S.last_cf_steps = 0, S.last_cf_scans = 0;
    PrivateArgs pa = w.pv;
    pa.g = g;
    pa.lam = &w.sc->lam;
    pa.parent = w.parent;
    // the per-pass arrays at the current graph's stride, as many passes as
    // the region holds
    pa.stride = std::max<int64_t>(g.n, 1);
    pa.stride1 = (int64_t)g.n / 64 + 2;
    passes = (int32_t)std::min<int64_t>({(int64_t)passes, (int64_t)w.pv.passes, w.pv.region / pa.stride,
                                         w.pv.region1 / pa.stride1});
    if (passes < 1) return mc_hip_ok(hipErrorInvalidValue, "private passes: no room for one pass");
    S.pv_stride = pa.stride;
    pa.passes = passes;
    pa.len_cap = len_cap;
    pa.seed = S.c->opt.seed;
    pa.round = round;
    pa.start = -1;
    pa.marks = &w.sc->marks_cf;
    pa.steps = w.psteps;
    // A complete pass (len_cap 0, the fallback of Algorithm 2) of a graph
    // whose truncated passes were mostly single pops (many whole-GPU steps
    // of fewer than 8 vertices on average: heavy weights, a bound far above
    // most edge weights) runs in one workgroup of 512 threads (the best of
    // 64..1024 measured), which selects a single pop from its two-level
    // index and scans it in a few microseconds, where a whole-GPU step costs
    // about seven launches per pop.
    // Below 4x the level threshold it always does; above, a complete pass
    // of large batches stays on the whole GPU.
    const int64_t lmin = levels_min_n(S.c);
    const bool singles_heavy = len_cap <= 0 && S.last_cf_steps > 200 && S.last_cf_scans < 8 * (int64_t)S.last_cf_steps;
    if (len_cap <= 0 && (singles_heavy || g.n < 4 * lmin)) pa.threads = 512;
    if (g.n >= lmin && (len_cap > 0 || (g.n >= 4 * lmin && !singles_heavy))) {
        StepArgs sa = w.sa;
        sa.pv = pa;
        int32_t running = 0;
        if (len_cap <= 0 || len_cap > sa.bcap) sa.bcap = g.n;   // unlimited pass: one pass, n+1 prefix slots
        // a truncated pass with no capped vertex queued continues one vertex
        // per whole-GPU step; bound such runs (the complete fallback pass is
        // never bounded)
        sa.max_singles = len_cap > 0 ? 256 : 0;
        if (!capforest_steps(sa, &running, S.s, capture_stream(S.c))) return false;
        S.last_cf_steps = sa.steps_run;
        S.last_cf_scans = sa.scans_run;
    } else if (!capforest_private(pa, S.s)) {
        return false;
    }
    CapforestArgs ra{};
    ra.alpha = pa.alpha;
    ra.alpha_len = pa.alpha_len;
    ra.passes = passes;
    return capforest_reduce(ra, w.sc, S.s);
}

// vertices at or below which the remaining rounds run in the finisher
static int32_t finish_max_n(const mc_ctx* c) {
    if (c->opt.finish_max_n < 0) return 0;
    return c->opt.finish_max_n > 0 ? std::min(c->opt.finish_max_n, FIN_N) : FIN_N;
}

// All remaining rounds of a small current graph in one launch (one
// workgroup): the bound and, if it dropped, the side come back at once.
static mc_status finish(Solver& S, DGraph* cur, int32_t round) {
    SolveWS& w = S.w;
    hipStream_t s = S.s;
    FinishArgs fa{};
    fa.g = *cur;
    fa.gvoff = nullptr;
    fa.glist = nullptr;
    fa.lam_in = &w.sc->lam;
    fa.lam_out = w.fin64;
    fa.dropped = w.fin32;
    fa.rounds = w.fin32 + 1;
    fa.err = w.fin32 + 2;
    fa.qnext = w.fin32 + 3;
    fa.fside = w.flag8;
    for (int q = 0; q < 2; q++) {
        fa.xcol[q] = w.fx_col[q];
        fa.xw[q] = w.fx_w[q];
    }
    fa.xwindow = 0;
    fa.seed = S.c->opt.seed ^ ((uint64_t)(uint32_t)round << 20);
    fa.qmode = S.c->opt.deterministic ? 2 : S.c->opt.queue;
    if (!fill_i32(w.fin32, 0, 4, s) || !finish_graphs(fa, 1, S.c->cus, s)) return MC_E_DEVICE;
    int64_t lam_out = 0;
    int32_t r32[4] = {0, 0, 0, 0};
    if (hipMemcpyAsync(&lam_out, w.fin64, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(r32, w.fin32, sizeof(r32), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(MC_E_DEVICE, "finisher: readback failed");
    if (r32[2] != 0) return fail(MC_E_DEVICE, "finisher: a graph could not finish (code " + std::to_string(r32[2]) + ")");
    if (r32[0] && lam_out < S.lam) {
        if (!side_from_flag(w.side, w.map0, S.n0, w.flag8, s)) return MC_E_DEVICE;
        if (!S.set_lam(lam_out)) return MC_E_DEVICE;
    }
    S.stats.rounds += r32[1];
    S.stats.finish_rounds += r32[1];
    return MC_OK;
}

// Exact rounds of Algorithm 2 on w.g[src] until at most two vertices remain.
static mc_status exact_rounds(Solver& S, int src) {
    SolveWS& w = S.w;
    hipStream_t s = S.s;
    DGraph* cur = &w.g[src];
    int nxt_idx = src == 1 ? 2 : 1;
    int32_t round = 0;
    while (cur->n > 2) {
        if (cur->n <= finish_max_n(S.c)) {
            // a small graph finishes every remaining round in one launch
            mc_status r = finish(S, cur, round);
            if (r != MC_OK) return r;
            break;
        }
        DGraph* nxt = &w.g[nxt_idx];
        const int32_t n = cur->n;
        prof_round_begin(S.in_heuristic ? 2 : 0, n, S.cur_m, s);
        k_reset_round<<<1, 1, 0, s>>>(w.sc);
        if (!uf_init(w.parent, n, s)) return MC_E_DEVICE;
        if (!S.reduction_tests(*cur)) return MC_E_DEVICE;
        const bool det = S.c->opt.deterministic != 0;
        // when the reduction tests alone at least halve the graph, contract
        // now and leave CAPFOREST to the smaller graph of the next round
        // (any set of contractible edges is a valid round)
        if (!S.readback()) return MC_E_DEVICE;
        S.tri_account(n);
        const bool skip_cf = 2 * (int64_t)(S.c->hsc->marks_pr + S.c->hsc->marks_tri) >= n;
        int used = CF_RUN_NONE;   // the CAPFOREST form whose results the round keeps last
        if (skip_cf) {
            S.stats.rounds_pr_only++;
        } else if (det) {
            if (!sequential_pass(S, *cur, round)) return MC_E_DEVICE;
            used = CF_RUN_SEQ;
        } else {
            // visited-array policy (Section 4, parallel session (1)): shared
            // or private visited state, fixed by the options or, in the
            // automatic mode, chosen on the first round of each size regime
            // that runs CAPFOREST. A short probe of shared passes (four per
            // compute unit, 32 pops each) runs first: if it contracts fewer
            // than one vertex in 1024, private passes are kept; otherwise a
            // private run of at most kProbePrivate scans per pass follows in
            // the same round, and the form with more marks per millisecond
            // is kept. Every mark of both runs is contracted.
            const int reg = n >= levels_min_n(S.c) ? 0 : 1;
            int form = S.c->opt.capforest_mode == MC_CF_SHARED ? CF_RUN_SHARED
                       : S.c->opt.capforest_mode == MC_CF_PRIVATE ? CF_RUN_PRIVATE : S.cf_choice[reg];
            const int32_t npriv = std::min(w.pv.passes, S.passes_for(n));
            bool private_done = false;
            if (form == CF_RUN_NONE) {
                using clk = std::chrono::steady_clock;
                const auto t0 = clk::now();
                if (!shared_passes(S, *cur, true) || !S.readback()) return MC_E_DEVICE;
                const double ms_s = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
                const unsigned long long marks_s = S.c->hsc->marks_cf;
                if (!S.apply_alpha(CF_RUN_SHARED, n)) return MC_E_DEVICE;
                used = CF_RUN_SHARED;
                form = CF_RUN_PRIVATE;
                double ms_p = 0;
                unsigned long long marks_p = 0;
                if (marks_s * 1024 >= (unsigned long long)n) {
                    const int32_t cap = private_len_cap(S.c);
                    const auto t1 = clk::now();
                    if (!private_passes(S, *cur, round, npriv, cap > 0 && cap < kProbePrivate ? cap : kProbePrivate) ||
                        !S.readback())
                        return MC_E_DEVICE;
                    ms_p = std::chrono::duration<double, std::milli>(clk::now() - t1).count();
                    marks_p = S.c->hsc->marks_cf - marks_s;
                    used = CF_RUN_PRIVATE;
                    private_done = true;
                    if ((double)marks_s * ms_p > (double)marks_p * ms_s) form = CF_RUN_SHARED;
                }
                S.cf_choice[reg] = form;
                if (S.debug)
                    fprintf(stderr,
                            "[mc] round %d visited-array probe: shared %llu marks in %.3f ms, private %llu in %.3f ms, "
                            "n=%d -> %s\n",
                            round, marks_s, ms_s, marks_p, ms_p, n, form == CF_RUN_SHARED ? "shared" : "private");
            } else if (form == CF_RUN_SHARED) {
                if (!shared_passes(S, *cur, false)) return MC_E_DEVICE;
                used = CF_RUN_SHARED;
            }
            if (form == CF_RUN_PRIVATE && !private_done) {
                if (!private_passes(S, *cur, round, npriv, private_len_cap(S.c))) return MC_E_DEVICE;
                used = CF_RUN_PRIVATE;
            }
        }
        if (!S.readback()) return MC_E_DEVICE;
        if (S.debug) debug_round(S, *cur, round, used == CF_RUN_PRIVATE ? std::min(w.pv.passes, S.passes_for(n)) : 0);
        if (!S.apply_alpha(used, n)) return MC_E_DEVICE;
        if (!S.readback()) return MC_E_DEVICE;
        DevScalars h = *S.c->hsc;
        S.stats.marks_pr += (int64_t)(h.marks_pr + h.marks_tri);
        S.stats.marks_capforest += (int64_t)h.marks_cf;
        const unsigned long long marks0 = h.marks_pr + h.marks_tri + h.marks_cf;
        // Algorithm 2: no contractible edge found, run CAPFOREST over the
        // whole graph without a length limit; with a fixed bound it marks at
        // least one edge, otherwise it lowered the bound. The same complete
        // pass also follows truncated passes that found fewer than one
        // contraction per 1024 vertices (on heavily weighted graphs a pass
        // reaches capped vertices only after many single pops, and a
        // truncated one stops first), so such graphs are not contracted a
        // handful of edges per round.
        const bool truncated = used == CF_RUN_PRIVATE && private_len_cap(S.c) > 0;
        if (marks0 == 0 || (truncated && marks0 * 1024 < (unsigned long long)n)) {
            const int64_t lam_before = S.lam;
            if (S.debug)
                fprintf(stderr, "[mc] round %d complete pass: n=%d marks so far %llu, last truncated launch %d steps %lld scans\n",
                        round, n, marks0, S.last_cf_steps, (long long)S.last_cf_scans);
            if (det) {
                if (!sequential_pass(S, *cur, round + 7777)) return MC_E_DEVICE;
            } else {
                if (!private_passes(S, *cur, round + 7777, 1, 0)) return MC_E_DEVICE;
            }
            if (!S.readback()) return MC_E_DEVICE;
            const unsigned long long cf0 = h.marks_cf;
            h = *S.c->hsc;
            S.stats.fallback_passes++;
            S.stats.marks_capforest += (int64_t)(h.marks_cf - cf0);
            if (h.best_pass >= 0 && h.best_alpha < S.lam) {
                const int32_t* pref_order = det ? w.corder : w.pv.order;
                if (!side_from_prefix(w.side, w.map0, S.n0, w.flag8, n, pref_order, &w.sc->best_len, s))
                    return MC_E_DEVICE;
                if (!S.set_lam(h.best_alpha)) return MC_E_DEVICE;
            }
            if (marks0 == 0 && h.marks_cf == 0) {
                if (S.lam < lam_before) { round++; continue; }
                return fail(MC_E_DEVICE, "sequential CAPFOREST marked no edge at a fixed bound");
            }
        }
        if (!uf_labels(w.parent, n, w.L, w.flag, w.cw.scan_tmp, w.sc, s)) return MC_E_DEVICE;
        if (!S.readback()) return MC_E_DEVICE;
        const int32_t n2 = S.c->hsc->n2;
        if (n2 == 1) {
            // everything joins one vertex: the solve ends with this round
            // and no later bound needs the contracted graph or the map
            prof_round_end(1, 0, s);
            S.cur_m = 0;
            round++;
            cur->n = 1;
            break;
        }
        if (!contract(entries_view(*cur, S.cur_m), w.L, n2, *nxt, w.cw, w.sc, s)) return MC_E_DEVICE;
        if (!map_update(w.map0, w.L, S.n0, s)) return MC_E_DEVICE;
        if (!S.readback()) return MC_E_DEVICE;
        h = *S.c->hsc;
        S.cur_m = h.m2;
        // a small round that removed fewer than one vertex in ten: more
        // passes from now on (small_pass_max)
        if (used == CF_RUN_PRIVATE && n < levels_min_n(S.c) && (int64_t)n2 * 10 > (int64_t)n * 9)
            S.small_passes = S.small_max;
        if (n2 >= 2 && h.dmin < S.lam) {
            if (!side_from_vertex(w.side, w.map0, S.n0, &w.sc->dmin_arg, s)) return MC_E_DEVICE;
            if (!S.set_lam(h.dmin)) return MC_E_DEVICE;
        }
        prof_round_end(n2, S.cur_m, s);
        nxt_idx = (nxt_idx == 1) ? 2 : 1;
        cur = nxt;
        round++;
    }
    if (cur->n > 1) prof_round_end(cur->n, S.cur_m, s);   // a round that ended without contraction
    S.stats.rounds += round;
    return MC_OK;
}

// Contract cur by labels L (n2 groups) into g[*nxt_idx]; the collapsed
// degrees of the result bound lambda (Section 2.1 "Overall algorithm"; only
// while at least two vertices remain). Returns the new current graph.
// lambda = 0 iff the input is disconnected. g is the input or a contraction
// of it that merged vertices of one component only (map0 takes input
// vertices to g's vertices): such a contraction keeps every component
// connected and joins no two, so g has exactly the input's components. On a
// disconnected input the side becomes the complement of vertex 0's
// component.
static bool check_connected(Solver& S, const DGraph& g) {
    SolveWS& w = S.w;
    hipStream_t s = S.s;
    if (!uf_init(w.parent, g.n, s) || !uf_connectivity(g, w.parent, w.vpart_i32(), w.flag8, w.L, s) ||
        !uf_labels(w.parent, g.n, w.L, w.flag, w.cw.scan_tmp, w.sc, s) || !S.readback())
        return false;
    S.conn_pending = false;
    if (S.c->hsc->n2 > 1) {
        S.disconnected = true;
        if (!side_from_components(w.side, w.parent, &g == &w.g[0] ? nullptr : w.map0, S.n0, s)) return false;
    }
    return true;
}

static DGraph* contract_and_bound(Solver& S, DGraph* cur, int32_t n2, int* nxt_idx, mc_status* err) {
    SolveWS& w = S.w;
    hipStream_t s = S.s;
    DGraph* nxt = &w.g[*nxt_idx];
    *err = MC_E_DEVICE;
    if (!contract(entries_view(*cur, S.cur_m), w.L, n2, *nxt, w.cw, w.sc, s) || !map_update(w.map0, w.L, S.n0, s) ||
        !S.readback())
        return nullptr;
    const DevScalars h = *S.c->hsc;
    S.cur_m = h.m2;
    if (n2 >= 2 && h.dmin < S.lam) {
        if (!side_from_vertex(w.side, w.map0, S.n0, &w.sc->dmin_arg, s) || !S.set_lam(h.dmin)) return nullptr;
    }
    *nxt_idx = *nxt_idx == 1 ? 2 : 1;
    *err = MC_OK;
    return nxt;
}

// The inexact heuristic that lowers the bound before the exact rounds
// (Section 2.1 "Lowering the upper bound"; Algorithm 2's first step). While
// the graph has more than heuristic_min_n vertices: lp_iters synchronous
// label-propagation rounds from singleton labels, contraction of every
// cluster, then the reduction tests 1 and 2 against the bound and their
// contraction. The coarse graph that remains is solved exactly by the same
// rounds. Every bound found is a cut of the input (clusters are unions of
// input vertices), so the side snapshots stay valid. Coarsening stops when a
// level removes fewer than 5 percent of the vertices.
static mc_status heuristic(Solver& S) {
    SolveWS& w = S.w;
    hipStream_t s = S.s;
    const int32_t nh = S.c->opt.heuristic_min_n;
    const int iters = S.c->opt.lp_iters > 0 ? S.c->opt.lp_iters : 2;
    DGraph* cur = &w.g[0];
    int nxt_idx = 1;
    mc_status err = MC_OK;
    while (cur->n > nh && cur->n > 2) {
        const int32_t n = cur->n;
        prof_round_begin(1, n, S.cur_m, s);
        int32_t* a = w.parent;   // labels ping-pong between parent[] and lab2[]
        int32_t* b = w.lab2;
        // the first round starts from singleton labels on a normal graph
        // (on the input, the input pass took it already); the last readback
        // holds cur's maximum degree (its last min_degree)
        const bool narrow = S.c->hsc->dmax < ((int64_t)1 << 32);
        if (S.lp1_ready && cur == &w.g[0]) S.lp1_ready = false;
        else if (!lp_first(*cur, b, w.lw, w.cw, s)) return MC_E_DEVICE;
        std::swap(a, b);
        for (int it = 1; it < iters; it++) {
            if (!lp_round(entries_view(*cur, S.cur_m), a, b, w.lw, w.cw, s, narrow)) return MC_E_DEVICE;
            std::swap(a, b);
        }
        if (!lp_relabel(a, n, w.L, w.flag, w.cw.scan_tmp, w.sc, s) || !S.readback()) return MC_E_DEVICE;
        const int32_t n2 = S.c->hsc->n2;
        if (S.debug) fprintf(stderr, "[mc] heuristic level %d: n=%d clusters=%d lam=%lld\n", S.stats.heuristic_levels, n, n2,
                             (long long)S.lam);
        if ((int64_t)n2 * 20 > (int64_t)n * 19) break;
        cur = contract_and_bound(S, cur, n2, &nxt_idx, &err);
        if (!cur) return err;
        S.stats.heuristic_levels++;
        // reduction tests 1 and 2 on the clustered graph (tests 3 and 4 are
        // off in a solve that runs the heuristic)
        k_reset_round<<<1, 1, 0, s>>>(w.sc);
        if (!uf_init(w.parent, cur->n, s) || !S.reduction_tests(*cur) ||
            !uf_labels(w.parent, cur->n, w.L, w.flag, w.cw.scan_tmp, w.sc, s) || !S.readback())
            return MC_E_DEVICE;
        S.tri_account(cur->n);
        const int32_t n3 = S.c->hsc->n2;
        if (S.debug) fprintf(stderr, "[mc]   after cluster contraction n=%d lam=%lld, tests 1-2 leave %d\n", cur->n,
                             (long long)S.lam, n3);
        if (n3 < cur->n) {
            S.stats.marks_pr += (int64_t)(S.c->hsc->marks_pr + S.c->hsc->marks_tri);
            cur = contract_and_bound(S, cur, n3, &nxt_idx, &err);
            if (!cur) return err;
        }
        prof_round_end(cur->n, S.cur_m, s);
    }
    prof_round_end(cur->n, S.cur_m, s);   // a level that stopped before contracting
    // Every contraction above merged vertices inside a label cluster or
    // along an edge. A label is the id of a vertex joined to its holder by a
    // path (labels only move along edges), so a cluster lies inside one
    // component: the coarse graph has the input's components, and deciding
    // connectivity there costs next to nothing.
    if (S.conn_pending) {
        if (!check_connected(S, *cur)) return MC_E_DEVICE;
        if (S.disconnected) return MC_OK;
    }
    if (cur == &w.g[0]) return MC_OK;   // nothing coarsened: the exact rounds start from the min degree
    if (cur->n > 2) {
        S.in_heuristic = true;
        mc_status r = exact_rounds(S, nxt_idx == 1 ? 2 : 1);
        S.in_heuristic = false;
        if (r != MC_OK) return r;
    }
    S.stats.lambda_heuristic = S.lam;
    return MC_OK;
}

extern "C" mc_status mc_mincut(mc_ctx* c, const mc_csr* g, void* dev_ws, size_t ws_bytes, int64_t* lambda,
                               uint8_t* side_out, mc_stats* st) {
    auto t0 = std::chrono::steady_clock::now();
    if (!c || !g || !lambda) return fail(MC_E_INVALID_ARG, "mc_mincut: NULL argument");
    if (g->n < 2) return fail(MC_E_INVALID_ARG, "mc_mincut: need n >= 2");
    if (g->nnz < 0 || !g->row_ptr || (g->nnz > 0 && (!g->col || !g->w)))
        return fail(MC_E_INVALID_ARG, "mc_mincut: bad CSR pointers");
    if (g->location != MC_HOST && g->location != MC_DEVICE) return fail(MC_E_INVALID_ARG, "mc_mincut: bad location");
    if (!dev_ws) return fail(MC_E_INVALID_ARG, "mc_mincut: workspace is NULL");
    const bool host_input = g->location == MC_HOST;
    if (host_input) {
        mc_status v = check_host_csr(g, c->opt.validate != 0);
        if (v != MC_OK) return v;
    }
    if (hipSetDevice(c->device) != hipSuccess) return fail(MC_E_DEVICE, "hipSetDevice failed");

    ProfScope prof_scope(static_cast<Prof*>(c->prof));
    if (g_prof) g_prof->clear_rounds();
    Solver S;
    S.c = c;
    S.s = c->stream;
    S.debug = getenv("MC_DEBUG") != nullptr;
    S.tri_on = c->opt.pr_tri_deg_cap > 0;
    const int32_t n = g->n;
    const int64_t nnz = g->nnz;
    Arena a;
    a.base = (char*)dev_ws;
    a.size = ws_bytes;
    // the most passes of small rounds that the workspace holds: one per
    // compute unit, else the first round's count (the least a solve needs)
    S.small_max = small_pass_max(c);
    carve(a, n, nnz, pass_count(c), large_pass_count(c), private_len_cap(c), host_input, 3, S.w, S.small_max,
          small_pass_n(c, n), c->opt.contract_mode == 1);
    if (a.used > ws_bytes) {
        S.small_max = private_pass_count(c, 2);
        a = Arena{};
        a.base = (char*)dev_ws;
        a.size = ws_bytes;
        S.w = SolveWS{};
        carve(a, n, nnz, pass_count(c), large_pass_count(c), private_len_cap(c), host_input, 3, S.w,
              S.small_max, small_pass_n(c, n), c->opt.contract_mode == 1);
    }
    if (a.used > ws_bytes) return fail(MC_E_INVALID_ARG, "mc_mincut: workspace too small");
    SolveWS& w = S.w;
    hipStream_t s = S.s;
    S.n0 = n;
    S.stats.lambda_heuristic = -1;

    const int32_t* rp = g->row_ptr;
    const int32_t* col = g->col;
    const int64_t* wt = g->w;
    if (host_input) {
        if (hipMemcpyAsync(w.in_rp, g->row_ptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice, s) != hipSuccess ||
            (nnz > 0 && hipMemcpyAsync(w.in_col, g->col, sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice, s) != hipSuccess) ||
            (nnz > 0 && hipMemcpyAsync(w.in_w, g->w, sizeof(int64_t) * (size_t)nnz, hipMemcpyHostToDevice, s) != hipSuccess))
            return fail(MC_E_DEVICE, "copy of the input graph failed");
        rp = w.in_rp;
        col = w.in_col;
        wt = w.in_w;
    }
    k_reset_round<<<1, 1, 0, s>>>(w.sc);
    // normalise. An input already in normal form (rows strictly increasing,
    // no loops, positive weights) is used in place as the first graph: no
    // kernel writes the current graph's off/col/w. Otherwise contraction by
    // the identity folds loops, parallel entries and zero weights; the
    // padded view of the input reuses g[1]'s arrays. A device input is
    // checked in the same pass (host inputs were checked on the host), and
    // nothing else reads it before the check's result is known. The minimum
    // degree of a normal input is taken before that readback: it reads only
    // the lengths and degrees the pass wrote, so one readback serves both.
    w.g[0].n = n;
    // a solve that runs the heuristic takes its first label-propagation
    // round from this pass when the input is normal
    const bool run_heuristic = c->opt.heuristic_min_n > 0 && n >= c->opt.heuristic_min_n;
    if (!canon_check(rp, col, wt, n, (int32_t)nnz, w.g[0].len, w.g[0].deg, &w.sc->noncanon,
                     host_input ? nullptr : w.sc, w.vpart, run_heuristic ? w.lab2 : nullptr, s) ||
        !min_degree(w.g[0], w.cw, w.sc, s) || !S.readback())
        return MC_E_DEVICE;
    if (c->hsc->err != 0)
        return fail((mc_status)c->hsc->err, c->hsc->err == MC_E_OVERFLOW ? "total weight must be below 2^62"
                                                                          : "malformed CSR (row_ptr, col or w)");
    const bool input_normal = c->hsc->noncanon == 0;
    if (input_normal) {
        w.g[0].cap = nnz;
        w.g[0].off = const_cast<int32_t*>(rp);
        w.g[0].col = const_cast<int32_t*>(col);
        w.g[0].w = const_cast<int64_t*>(wt);
    } else {
        DGraph user = w.g[1];
        user.n = n;
        user.cap = nnz;
        user.col = const_cast<int32_t*>(col);
        user.w = const_cast<int64_t*>(wt);
        if (!csr_to_padded(rp, n, user.off, user.len, s)) return MC_E_DEVICE;
        if (!contract(user, nullptr, n, w.g[0], w.cw, w.sc, s)) return MC_E_DEVICE;
    }
    S.stats.input_normal = input_normal;
    if (!iota_i32(w.map0, n, s) || !fill_i32(w.claim, 0, n, s)) return MC_E_DEVICE;
    // connectivity: lambda = 0 iff the positive-weight graph is disconnected.
    // When the heuristic runs, its coarse graph has the same components and
    // decides it at a fraction of the cost (a vertex of degree 0 decides it
    // here).
    S.lp1_ready = run_heuristic && input_normal;
    // Tests 3 and 4 run only in solves without the heuristic. With it they
    // cost more than they save, on the clusters and in the exact rounds
    // after it (hyperbolic 2^23: 7.12 ms per solve with them, 6.83 without;
    // Chung-Lu 2^22: 14.54 and 14.42 ms).
    if (run_heuristic) S.tri_on = false;
    if (!input_normal && !S.readback()) return MC_E_DEVICE;   // the normalisation's minimum degree
    if (run_heuristic && c->hsc->dmin > 0) {
        S.conn_pending = true;
    } else if (!check_connected(S, w.g[0])) {
        return MC_E_DEVICE;
    }
    DevScalars h = *c->hsc;
    S.stats.n_input = n;
    const int64_t m_input = h.m2;   // entries of the normalised input (read by min_degree)
    S.cur_m = m_input;
    int64_t result = 0;
    if (S.disconnected) {
        result = 0;   // check_connected set the side
    } else {
        // minimum degree is the first bound; its vertex is the first side
        if (!side_from_vertex(w.side, w.map0, n, &w.sc->dmin_arg, s)) return MC_E_DEVICE;
        if (!S.set_lam(h.dmin)) return MC_E_DEVICE;
        S.stats.lambda_min_degree = h.dmin;
        mc_status r = MC_OK;
        if (run_heuristic) {
            if ((r = heuristic(S)) != MC_OK) return r;
            // the exact rounds start again from the normalised input
            if (!iota_i32(w.map0, n, s)) return MC_E_DEVICE;
            S.cur_m = m_input;
        }
        if (S.disconnected) {
            result = 0;
        } else {
            if ((r = exact_rounds(S, 0)) != MC_OK) return r;
            result = S.lam;
        }
    }
    if (side_out) {
        if (hipMemcpyAsync(side_out, w.side, (size_t)n, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(MC_E_DEVICE, "copy of the side failed");
        if (side_out[0])
            for (int32_t v = 0; v < n; v++) side_out[v] ^= 1;
    } else if (hipStreamSynchronize(s) != hipSuccess) {
        return fail(MC_E_DEVICE, "stream synchronisation failed");
    }
    *lambda = result;
    if (st) {
        S.stats.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        *st = S.stats;
    }
    return MC_OK;
}

extern "C" mc_status mc_mincut_static(mc_ctx* c, const mc_csr* g, int64_t* lambda, uint8_t* side_out, mc_stats* st) {
    if (!c || !g || !lambda) return fail(MC_E_INVALID_ARG, "mc_mincut_static: NULL argument");
    if (!c->scratch) return fail(MC_E_DEVICE, "mc_mincut_static: no static scratch on this device");
    if (g->n < 2 || g->nnz < 0) return fail(MC_E_INVALID_ARG, "mc_mincut_static: need n >= 2 and nnz >= 0");
    // the least a solve needs (small rounds with their first pass count);
    // mc_mincut takes more passes where the scratch holds them
    const size_t need = workspace_min_bytes(c, g->n, g->nnz);
    mc_status r = MC_OK;
    if (need > kStaticScratchBytes)
        return fail(MC_E_INVALID_ARG, "mc_mincut_static: the graph needs " + std::to_string(need) +
                                          " bytes of scratch, more than the static " +
                                          std::to_string(kStaticScratchBytes) + " (use mc_mincut with a workspace)");
    // kernel timing and graph capture are suspended for the call: the event
    // pool and graph instantiation could allocate
    void* prof = c->prof;
    const bool graphs_off = c->graphs_off;
    c->prof = nullptr;
    c->graphs_off = true;
    r = mc_mincut(c, g, c->scratch, kStaticScratchBytes, lambda, side_out, st);
    c->prof = prof;
    c->graphs_off = graphs_off;
    return r;
}

// ------------------------------------------------------------ step ABI
namespace {
DGraph to_dgraph(const mc_dgraph* g) {
    DGraph d;
    d.n = g->n;
    d.cap = g->cap;
    d.off = g->off;
    d.len = g->len;
    d.col = g->col;
    d.w = g->w;
    d.deg = g->deg;
    return d;
}

struct StepWS {
    LpWS lw;
    Pr34WS tw;
    DevScalars* sc;
    int32_t* parent;
    int32_t* flag;
    int32_t* claim;
    ContractWS cw;
    int32_t* order;
    int32_t* nscan;
    int64_t* alpha;
    int32_t* alen;
    int64_t* lamout;
    int32_t* cst;
    int64_t* cr;
    int64_t* cl1;
    int64_t* lam;
    PrivateArgs pv;
    int32_t* psteps;
    Pr12WS prw;
    StepArgs sa;
};

void carve_step(Arena& a, int32_t n, int64_t cap, int32_t passes, StepWS& w) {
    w.sc = a.take<DevScalars>(1);
    lp_ws_carve(a, n, cap, w.lw);
    pr34_ws_carve(a, n, w.tw);
    w.lam = a.take<int64_t>(1);
    w.parent = a.take<int32_t>((size_t)n + 1);
    w.flag = a.take<int32_t>((size_t)n + 2);
    w.claim = a.take<int32_t>((size_t)n + 1);
    contract_ws_carve(a, n, cap, w.cw);
    pr12_ws_carve(a, n, cap, w.prw);
    if (passes < 1) passes = 1;
    w.order = a.take<int32_t>((size_t)passes * CF_HC);
    w.nscan = a.take<int32_t>((size_t)passes);
    w.alpha = a.take<int64_t>((size_t)passes);
    w.alen = a.take<int32_t>((size_t)passes);
    w.lamout = a.take<int64_t>((size_t)passes);
    w.cst = a.take<int32_t>((size_t)n + 1);
    w.cr = a.take<int64_t>((size_t)n + 1);
    w.cl1 = a.take<int64_t>((size_t)n / 64 + 2);
    carve_private(a, n, passes, w.pv, w.psteps);
    carve_steps(a, n, cap, passes, 0, w.sa);
    // the sort merge's workspace too, so that contract_mode can pick either
    sort_ws_carve(a, n, cap, w.cw.sw);
}

mc_status step_begin(mc_ctx* c, int32_t n, int64_t cap, int32_t passes, void* ws, size_t bytes, StepWS& w) {
    if (!c || !ws) return fail(MC_E_INVALID_ARG, "step: NULL context or workspace");
    if (hipSetDevice(c->device) != hipSuccess) return fail(MC_E_DEVICE, "hipSetDevice failed");
    Arena a;
    a.base = (char*)ws;
    a.size = bytes;
    carve_step(a, n, cap, passes, w);
    if (a.used > bytes) return fail(MC_E_INVALID_ARG, "step: workspace too small");
    w.cw.sorted = c->opt.contract_mode == 1;
    return MC_OK;
}

mc_status sync_read(mc_ctx* c, StepWS& w) {
    if (hipMemcpyAsync(c->hsc, w.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(MC_E_DEVICE, "step: readback failed");
    return MC_OK;
}
}  // namespace

extern "C" mc_status mc_step_ws_size(int32_t n, int64_t cap, int32_t passes, size_t* bytes) {
    if (!bytes || n < 1 || cap < 0) return fail(MC_E_INVALID_ARG, "mc_step_ws_size: bad arguments");
    Arena a;
    StepWS w;
    carve_step(a, n, cap, passes, w);
    *bytes = a.used + 256;
    return MC_OK;
}

extern "C" mc_status mc_step_contract(mc_ctx* c, const mc_dgraph* src, const int32_t* labels, int32_t n2,
                                      mc_dgraph* dst, void* ws, size_t bytes, int64_t* dmin, int32_t* dmin_arg) {
    if (!src || !dst) return fail(MC_E_INVALID_ARG, "mc_step_contract: NULL graph");
    StepWS w;
    mc_status r = step_begin(c, src->n, src->cap, 1, ws, bytes, w);
    if (r != MC_OK) return r;
    DGraph s = to_dgraph(src), d = to_dgraph(dst);
    if (!contract(s, labels, labels ? n2 : src->n, d, w.cw, w.sc, c->stream)) return MC_E_DEVICE;
    if ((r = sync_read(c, w)) != MC_OK) return r;
    if (dmin) *dmin = c->hsc->dmin;
    if (dmin_arg) *dmin_arg = c->hsc->dmin_arg;
    return MC_OK;
}

extern "C" mc_status mc_step_components(mc_ctx* c, int32_t n, int64_t np, const int32_t* a, const int32_t* b,
                                        int32_t* labels, int32_t* n2, void* ws, size_t bytes) {
    StepWS w;
    mc_status r = step_begin(c, n, 1, 1, ws, bytes, w);
    if (r != MC_OK) return r;
    hipStream_t s = c->stream;
    if (!uf_init(w.parent, n, s)) return MC_E_DEVICE;
    if (np > 0) {
        k_uf_pairs<<<grid_for(np, 256), 256, 0, s>>>(a, b, np, w.parent);
        if (!mc_hip_ok(hipGetLastError(), "k_uf_pairs")) return MC_E_DEVICE;
    }
    if (!uf_labels(w.parent, n, labels, w.flag, w.cw.scan_tmp, w.sc, s)) return MC_E_DEVICE;
    if ((r = sync_read(c, w)) != MC_OK) return r;
    if (n2) *n2 = c->hsc->n2;
    return MC_OK;
}

extern "C" mc_status mc_step_pr12(mc_ctx* c, const mc_dgraph* g, int64_t lam, uint8_t* flag1, int32_t* ptr2,
                                  int32_t* labels, int32_t* n2, void* ws, size_t bytes) {
    if (!g) return fail(MC_E_INVALID_ARG, "mc_step_pr12: NULL graph");
    StepWS w;
    mc_status r = step_begin(c, g->n, g->cap, 1, ws, bytes, w);
    if (r != MC_OK) return r;
    hipStream_t s = c->stream;
    k_set_lam<<<1, 1, 0, s>>>(w.sc, lam);
    k_reset_round<<<1, 1, 0, s>>>(w.sc);
    if (!uf_init(w.parent, g->n, s)) return MC_E_DEVICE;
    if (!pr12(to_dgraph(g), &w.sc->lam, w.parent, &w.sc->marks_pr, flag1, ptr2, w.prw, s)) return MC_E_DEVICE;
    if (!uf_labels(w.parent, g->n, labels, w.flag, w.cw.scan_tmp, w.sc, s)) return MC_E_DEVICE;
    if ((r = sync_read(c, w)) != MC_OK) return r;
    if (n2) *n2 = c->hsc->n2;
    return MC_OK;
}

extern "C" mc_status mc_step_pr34(mc_ctx* c, const mc_dgraph* g, int64_t lam, int32_t D, const int32_t* ptr2,
                                  uint8_t* flag4, int32_t* acc3, int32_t* labels, int32_t* n2, void* ws, size_t bytes) {
    if (!g || !ptr2) return fail(MC_E_INVALID_ARG, "mc_step_pr34: NULL graph or ptr2");
    if (D < 0 || D > 64) return fail(MC_E_INVALID_ARG, "mc_step_pr34: D must be in [0, 64]");
    StepWS w;
    mc_status r = step_begin(c, g->n, g->cap, 1, ws, bytes, w);
    if (r != MC_OK) return r;
    hipStream_t s = c->stream;
    k_set_lam<<<1, 1, 0, s>>>(w.sc, lam);
    k_reset_round<<<1, 1, 0, s>>>(w.sc);
    if (!uf_init(w.parent, g->n, s)) return MC_E_DEVICE;
    if (!pr34(to_dgraph(g), &w.sc->lam, D, w.parent, &w.sc->marks_tri, ptr2, w.tw, flag4, acc3, s)) return MC_E_DEVICE;
    if (!uf_labels(w.parent, g->n, labels, w.flag, w.cw.scan_tmp, w.sc, s)) return MC_E_DEVICE;
    if ((r = sync_read(c, w)) != MC_OK) return r;
    if (n2) *n2 = c->hsc->n2;
    return MC_OK;
}

extern "C" mc_status mc_step_lp(mc_ctx* c, const mc_dgraph* g, const int32_t* lab_in, int32_t* lab_out, void* ws,
                                size_t bytes) {
    if (!g || !lab_out) return fail(MC_E_INVALID_ARG, "mc_step_lp: NULL argument");
    if (lab_in == lab_out) return fail(MC_E_INVALID_ARG, "mc_step_lp: lab_in and lab_out must differ");
    StepWS w;
    mc_status r = step_begin(c, g->n, g->cap, 1, ws, bytes, w);
    if (r != MC_OK) return r;
    bool narrow = false;
    if (lab_in && !lp_narrow(to_dgraph(g), w.lw.counters + 3, &narrow, c->stream)) return MC_E_DEVICE;
    const bool ok = lab_in ? lp_round(to_dgraph(g), lab_in, lab_out, w.lw, w.cw, c->stream, narrow)
                           : lp_first(to_dgraph(g), lab_out, w.lw, w.cw, c->stream);
    if (!ok) return MC_E_DEVICE;
    return sync_read(c, w);
}

extern "C" mc_status mc_step_capforest(mc_ctx* c, const mc_dgraph* g, int64_t lam, int32_t start, int32_t mode,
                                       int32_t passes, int32_t shared, int32_t len_cap, int32_t* labels, int32_t* n2,
                                       int32_t* order, int32_t* nscan, int64_t* best_alpha, int32_t* best_len,
                                       int64_t* lam_out, void* ws, size_t bytes) {
    if (!g || !labels || !order) return fail(MC_E_INVALID_ARG, "mc_step_capforest: NULL argument");
    if (mode < MC_STEP_CF_SHARED || mode > MC_STEP_CF_HEAP) return fail(MC_E_INVALID_ARG, "mc_step_capforest: bad mode");
    if (mode == MC_STEP_CF_BUCKET || mode == MC_STEP_CF_HEAP) {
        // one pass of the finisher's CAPFOREST, queue in LDS
        if (g->n > FIN_N) return fail(MC_E_INVALID_ARG, "mc_step_capforest: the LDS-queue pass takes n <= 1024");
        if (start < 0 || start >= g->n) return fail(MC_E_INVALID_ARG, "mc_step_capforest: bad start");
        StepWS w;
        mc_status r = step_begin(c, g->n, g->cap, 1, ws, bytes, w);
        if (r != MC_OK) return r;
        hipStream_t s = c->stream;
        if (!fill_i64(w.lamout, lam, 1, s)) return MC_E_DEVICE;
        if (!finish_pass(to_dgraph(g), start, mode == MC_STEP_CF_HEAP ? 2 : 1, w.lamout, w.alpha, w.parent, order,
                         w.nscan, w.alen, s))
            return fail(MC_E_DEVICE, "mc_step_capforest: finisher pass launch failed");
        if (!uf_labels(w.parent, g->n, labels, w.flag, w.cw.scan_tmp, w.sc, s)) return MC_E_DEVICE;
        int64_t lo[2] = {0, 0};
        int32_t cnt[2] = {0, 0};
        if (hipMemcpyAsync(&lo[0], w.lamout, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&lo[1], w.alpha, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&cnt[0], w.nscan, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&cnt[1], w.alen, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
            return fail(MC_E_DEVICE, "step: readback failed");
        if ((r = sync_read(c, w)) != MC_OK) return r;
        if (n2) *n2 = c->hsc->n2;
        if (nscan) *nscan = cnt[0];
        if (best_alpha) *best_alpha = lo[1];
        if (best_len) *best_len = lo[1] == INT64_MAX ? 0 : cnt[1];
        if (lam_out) *lam_out = lo[0];
        return MC_OK;
    }
    if ((mode == MC_STEP_CF_SEQUENTIAL && start < 0) || start >= g->n)
        return fail(MC_E_INVALID_ARG, "mc_step_capforest: bad start");
    if (mode != MC_STEP_CF_SEQUENTIAL && passes < 1) return fail(MC_E_INVALID_ARG, "mc_step_capforest: passes must be >= 1");
    if (mode == MC_STEP_CF_SEQUENTIAL) passes = 1;
    StepWS w;
    mc_status r = step_begin(c, g->n, g->cap, passes, ws, bytes, w);
    if (r != MC_OK) return r;
    hipStream_t s = c->stream;
    k_set_lam<<<1, 1, 0, s>>>(w.sc, lam);
    k_reset_round<<<1, 1, 0, s>>>(w.sc);
    if (!uf_init(w.parent, g->n, s)) return MC_E_DEVICE;
    const int32_t* nscan_dev = w.nscan;
    const int64_t* lamout_dev = w.lamout;
    const int32_t* order_dev = w.order;
    int64_t order_len = CF_HC;
    CapforestArgs red{};
    if (mode == MC_STEP_CF_SEQUENTIAL) {
        CompleteArgs cp{};
        cp.g = to_dgraph(g);
        cp.lam = &w.sc->lam;
        cp.parent = w.parent;
        cp.start = start;
        cp.tag = ++c->tag;
        cp.st = w.cst;
        cp.r = w.cr;
        cp.l1 = w.cl1;
        cp.order = order;
        cp.nscan = w.nscan;
        cp.alpha = w.alpha;
        cp.alpha_len = w.alen;
        cp.lam_out = w.lamout;
        cp.marks = &w.sc->marks_cf;
        if (!capforest_complete(cp, s)) return MC_E_DEVICE;
        red.alpha = w.alpha;
        red.alpha_len = w.alen;
        red.passes = 1;
        order_dev = nullptr;
    } else if (mode == MC_STEP_CF_SHARED) {
        if (!fill_i32(w.claim, 0, g->n, s)) return MC_E_DEVICE;
        CapforestArgs ca{};
        ca.g = to_dgraph(g);
        ca.lam = &w.sc->lam;
        ca.parent = w.parent;
        ca.claim = w.claim;
        ca.tag = ++c->tag;
        ca.shared = shared;
        ca.passes = passes;
        ca.len_cap = len_cap;
        ca.seed = c->opt.seed;
        ca.start = start;
        ca.order = w.order;
        ca.nscan = w.nscan;
        ca.alpha = w.alpha;
        ca.alpha_len = w.alen;
        ca.lam_out = w.lamout;
        ca.marks = &w.sc->marks_cf;
        if (!capforest_passes(ca, s)) return MC_E_DEVICE;
        red = ca;
    } else {
        PrivateArgs pa = w.pv;
        pa.g = to_dgraph(g);
        pa.lam = &w.sc->lam;
        pa.parent = w.parent;
        pa.passes = passes;
        pa.len_cap = len_cap;
        pa.seed = c->opt.seed;
        pa.round = ++c->tag;
        pa.start = start;
        pa.marks = &w.sc->marks_cf;
        pa.steps = w.psteps;
        if (!capforest_private_reset(pa, s)) return MC_E_DEVICE;
        if (mode == MC_STEP_CF_LEVELS) {
            StepArgs sa = w.sa;
            sa.pv = pa;
            sa.bcap = g->n;
            int32_t running = 0;
            if (!capforest_steps(sa, &running, s)) return MC_E_DEVICE;
        } else if (!capforest_private(pa, s)) {
            return MC_E_DEVICE;
        }
        red.alpha = pa.alpha;
        red.alpha_len = pa.alpha_len;
        red.passes = passes;
        nscan_dev = pa.nscan;
        lamout_dev = pa.lam_out;
        order_dev = pa.order;
        order_len = g->n;
    }
    if (!capforest_reduce(red, w.sc, s)) return MC_E_DEVICE;
    if (!uf_labels(w.parent, g->n, labels, w.flag, w.cw.scan_tmp, w.sc, s)) return MC_E_DEVICE;
    int32_t ns = 0;
    int64_t lo = 0;
    if (hipMemcpyAsync(&ns, nscan_dev, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&lo, lamout_dev, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess)
        return fail(MC_E_DEVICE, "step: readback failed");
    if (order_dev &&
        hipMemcpyAsync(order, order_dev, sizeof(int32_t) * (size_t)order_len, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(MC_E_DEVICE, "step: order copy failed");
    if ((r = sync_read(c, w)) != MC_OK) return r;
    DevScalars h = *c->hsc;
    if (n2) *n2 = h.n2;
    if (nscan) *nscan = ns;
    if (best_alpha) *best_alpha = h.best_alpha;
    if (best_len) *best_len = h.best_len;
    if (lam_out) *lam_out = lo;
    return MC_OK;
}
