// Host side of the libqfs C ABI (include/qfs.h): argument checks, workspace
// layouts and the launch sequences.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <atomic>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/qfs.h"
#include "qfs_internal.h"

using namespace qfs;

namespace {

thread_local char g_err[512] = "";

// process-wide options (qfs_set_option)
std::atomic<bool> g_opt_height_band{true};
std::atomic<bool> g_opt_height_graph{true};
std::atomic<int> g_opt_deep_slots{0};  // persistent deep workgroups; 0 = one per compute unit
std::atomic<int> g_opt_gpow_per_cu{8};  // workgroups per compute unit of the g = f^(p-1) kernel

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

bool supported(int p) { return prime_index(p) >= 0; }

int device_cus()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return n;
}

bool aligned(const void *p) { return ((uintptr_t)p & 255u) == 0; }

int deep_slots()
{
    const int v = g_opt_deep_slots.load();
    return v > 0 ? v : device_cus();
}

// persistent workgroups of the g = f^(p-1) kernel: a few per compute unit
int gpow_workgroups(int batch)
{
    const int n = g_opt_gpow_per_cu.load() * device_cus();
    return batch < n ? batch : n;
}

// ---- stage timing: hipEvents recorded on the caller's stream ----
struct ProfRec {
    hipEvent_t ev[16];
    int stage[16];  // stage index of the interval ending at ev[i] (-1: none)
    int n;
};
struct Prof {
    std::mutex m;
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<ProfRec> recs;
    hipEvent_t get()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
} g_prof;

struct ProfCall {
    ProfRec r{};
    bool on;
    hipStream_t s;
    explicit ProfCall(hipStream_t st) : on(false), s(st)
    {
        std::lock_guard<std::mutex> lk(g_prof.m);
        on = g_prof.on;
        r.n = 0;
    }
    void mark(int stage)
    {
        if (!on || r.n >= 16) return;
        hipEvent_t e;
        {
            std::lock_guard<std::mutex> lk(g_prof.m);
            e = g_prof.get();
        }
        if (!e) return;
        hipEventRecord(e, s);
        r.ev[r.n] = e;
        r.stage[r.n] = stage;
        r.n++;
    }
    ~ProfCall()
    {
        if (!on || r.n == 0) return;
        std::lock_guard<std::mutex> lk(g_prof.m);
        g_prof.recs.push_back(r);
    }
};

int hip_fail(hipError_t e, const char *what)
{
    return fail(QFS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ---- graphs of the qfs_height launch sequence, keyed by every argument ----
struct GraphKey {
    int dev, batch, bound, max_p, band, slots, gwg;
    const void *p, *f, *h, *ws;
    size_t ws_bytes;
    bool operator==(const GraphKey &o) const
    {
        return dev == o.dev && batch == o.batch && bound == o.bound && max_p == o.max_p && band == o.band &&
               slots == o.slots && gwg == o.gwg && p == o.p && f == o.f && h == o.h && ws == o.ws &&
               ws_bytes == o.ws_bytes;
    }
};
struct GraphEntry {
    GraphKey key;
    hipGraph_t graph;
    hipGraphExec_t exec;
    uint64_t used;
};
constexpr size_t GRAPH_CACHE = 8;
constexpr int MAX_DEV = 16;
struct GraphCache {
    std::mutex m;
    std::vector<GraphEntry> v;
    std::vector<GraphKey> seen;     // argument sets met once: captured when they come back
    hipStream_t cap[MAX_DEV] = {};  // capture streams (default priority), one per device
    uint64_t tick = 0;
} g_graphs;

void destroy_entry(GraphEntry &en)
{
    hipGraphExecDestroy(en.exec);
    hipGraphDestroy(en.graph);
}

}  // namespace

extern "C" {

int64_t qfs_num_monomials(int deg) { return num_mono(deg); }

int64_t qfs_monomial_rank(const int32_t e[4])
{
    if (!e || e[0] < 0 || e[1] < 0 || e[2] < 0 || e[3] < 0) return -1;
    return cns_rank(e[1], e[2], e[3]);
}

int qfs_monomial_unrank(int deg, int64_t rank, int32_t e[4])
{
    if (!e || deg < 0 || rank < 0 || rank >= num_mono(deg))
        return fail(QFS_EINVAL, "qfs_monomial_unrank: rank %lld outside [0, %lld)", (long long)rank,
                    (long long)num_mono(deg));
    int a, b, c, d;
    cns_unrank(deg, rank, a, b, c, d);
    e[0] = a;
    e[1] = b;
    e[2] = c;
    e[3] = d;
    return QFS_OK;
}

int64_t qfs_len_g(int p) { return supported(p) ? num_mono(4 * (p - 1)) : -1; }
int64_t qfs_len_delta(int p) { return supported(p) ? num_mono(4 * p * (p - 1)) : -1; }

const char *qfs_last_error(void) { return g_err; }

void qfs_shutdown(void)
{
    std::lock_guard<std::mutex> lk(g_graphs.m);
    if (!g_graphs.v.empty()) hipDeviceSynchronize();
    for (GraphEntry &en : g_graphs.v) destroy_entry(en);
    g_graphs.v.clear();
    g_graphs.seen.clear();
    for (int d = 0; d < MAX_DEV; ++d)
        if (g_graphs.cap[d]) {
            hipStreamDestroy(g_graphs.cap[d]);
            g_graphs.cap[d] = nullptr;
        }
}

// ---------------------------------------------------------------------------
size_t qfs_delta1_workspace_bytes(int p, int batch)
{
    if (!supported(p) || batch < 0) return 0;
    bool present[4] = {false, false, false, false};
    present[prime_index(p)] = true;
    return make_batch_layout(present, batch, deep_slots()).total;
}

int qfs_delta1(int p, int batch, const uint8_t *f, uint8_t *g_out, uint8_t *delta_out, int32_t *status_out,
               void *ws, size_t ws_bytes, hipStream_t stream)
{
    g_err[0] = 0;
    if (!supported(p)) return fail(QFS_EUNSUPPORTED, "qfs_delta1: p=%d not in {3,5,7,11}", p);
    if (batch < 0) return fail(QFS_EINVAL, "qfs_delta1: batch=%d < 0", batch);
    if (batch == 0) return QFS_OK;
    if (!f || !delta_out || !ws) return fail(QFS_EINVAL, "qfs_delta1: null pointer argument");
    if (!aligned(ws)) return fail(QFS_EINVAL, "qfs_delta1: workspace not 256-byte aligned");
    const int ncu = device_cus();
    if (ncu <= 0) return fail(QFS_EDEVICE, "qfs_delta1: no HIP device");
    bool present[4] = {false, false, false, false};
    const int pi = prime_index(p);
    present[pi] = true;
    const BatchLayout L = make_batch_layout(present, batch, deep_slots());
    if (ws_bytes < L.total)
        return fail(QFS_ENOMEM, "qfs_delta1: workspace %zu bytes < %zu needed", ws_bytes, L.total);
    uint8_t *w = (uint8_t *)ws;
    int32_t *counters = (int32_t *)(w + L.counters);
    hipError_t e;
    if ((e = launch_reset(counters, stream)) != hipSuccess) return hip_fail(e, "reset");
    Stage1Args s1{};
    s1.batch = batch;
    s1.mode = MODE_DELTA;
    s1.fixed_p = p;
    s1.bound = 10;
    s1.f = f;
    s1.status = status_out;
    s1.g_out = g_out;
    s1.counters = counters;
    for (int i = 0; i < 4; ++i) {
        s1.queue[i] = L.present[i] ? (int32_t *)(w + L.queue[i]) : nullptr;
        s1.gq[i] = L.present[i] ? w + L.gq[i] : nullptr;
    }
    s1.present_mask = 1 << pi;
    if ((e = launch_stage1(s1, stream)) != hipSuccess) return hip_fail(e, "stage1");
    if (gpow_needed(p) && (e = launch_gpow(p, s1, gpow_workgroups(batch), stream)) != hipSuccess)
        return hip_fail(e, "g");
    if ((e = launch_plan(p, (uint32_t *)(w + L.plan[pi]), stream)) != hipSuccess) return hip_fail(e, "plan");
    DeepArgs da{};
    da.mode = MODE_DELTA;
    da.bound = 10;
    da.status = status_out;
    da.delta_out = delta_out;
    da.counters = counters;
    da.queue = (const int32_t *)(w + L.queue[pi]);
    da.gq = w + L.gq[pi];
    da.f = f;
    da.g_out = g_out;
    da.plan = (const uint32_t *)(w + L.plan[pi]);
    da.slots = w + L.slots;
    da.slot_bytes = L.slot_stride[pi];
    da.zero_halo = 1;
    const int nslots = batch < L.nslots[pi] ? batch : L.nslots[pi];
    if ((e = launch_deep(p, false, da, nslots, stream)) != hipSuccess) return hip_fail(e, "deep");
    return QFS_OK;
}

// ---------------------------------------------------------------------------
size_t qfs_theta_workspace_bytes(int p, int batch)
{
    if (!supported(p) || batch < 0) return 0;
    const int ncu = device_cus();
    const int slots = batch < ncu ? batch : ncu;
    return (size_t)(slots > 0 ? slots : 1) * theta_scratch_bytes(p);
}

int qfs_theta(int p, int batch, const uint8_t *delta, const uint8_t *a, uint8_t *out, int iters, void *ws,
              size_t ws_bytes, hipStream_t stream)
{
    g_err[0] = 0;
    if (!supported(p)) return fail(QFS_EUNSUPPORTED, "qfs_theta: p=%d not in {3,5,7,11}", p);
    if (batch < 0) return fail(QFS_EINVAL, "qfs_theta: batch=%d < 0", batch);
    if (iters < 0 || iters > 64) return fail(QFS_EINVAL, "qfs_theta: iters=%d outside 0..64", iters);
    if (batch == 0) return QFS_OK;
    if (!delta || !a || !out || !ws) return fail(QFS_EINVAL, "qfs_theta: null pointer argument");
    if (out == a) return fail(QFS_EINVAL, "qfs_theta: out aliases a");
    if (!aligned(ws)) return fail(QFS_EINVAL, "qfs_theta: workspace not 256-byte aligned");
    const int ncu = device_cus();
    if (ncu <= 0) return fail(QFS_EDEVICE, "qfs_theta: no HIP device");
    const size_t need = qfs_theta_workspace_bytes(p, batch);
    if (ws_bytes < need) return fail(QFS_ENOMEM, "qfs_theta: workspace %zu bytes < %zu needed", ws_bytes, need);
    const int slots = batch < ncu ? batch : ncu;
    hipError_t e = launch_theta(p, batch, delta, a, out, iters, (uint8_t *)ws, slots, stream);
    if (e != hipSuccess) return hip_fail(e, "theta");
    return QFS_OK;
}

// ---------------------------------------------------------------------------
static void present_upto(int max_p, bool present[4])
{
    for (int i = 0; i < 4; ++i) present[i] = kPrimes[i] <= max_p;
}

size_t qfs_height_workspace_bytes(int batch, int max_p)
{
    if (batch < 0 || max_p < 3 || max_p > 11) return 0;
    bool present[4];
    present_upto(max_p, present);
    return make_batch_layout(present, batch, deep_slots()).total;
}

// The launch sequence of qfs_height on `stream` (validated arguments).
static int enqueue_height(int batch, const int32_t *p, const uint8_t *f, int bound, const BatchLayout &L,
                          int32_t *heights, uint8_t *w, bool band, int gpow_wg, hipStream_t stream, ProfCall &prof)
{
    int32_t *counters = (int32_t *)(w + L.counters);
    hipError_t e;
    prof.mark(-1);
    if ((e = launch_reset(counters, stream)) != hipSuccess) return hip_fail(e, "reset");
    Stage1Args s1{};
    s1.batch = batch;
    s1.mode = MODE_HEIGHT;
    s1.fixed_p = 0;
    s1.bound = bound;
    s1.p = p;
    s1.f = f;
    s1.heights = heights;
    s1.counters = counters;
    int mask = 0;
    for (int i = 0; i < 4; ++i) {
        s1.queue[i] = L.present[i] ? (int32_t *)(w + L.queue[i]) : nullptr;
        s1.gq[i] = L.present[i] ? w + L.gq[i] : nullptr;
        if (L.present[i]) mask |= 1 << i;
    }
    s1.present_mask = mask;
    if ((e = launch_stage1(s1, stream)) != hipSuccess) return hip_fail(e, "stage1");
    for (int i = 0; i < 4; ++i)
        if (L.present[i] && gpow_needed(kPrimes[i]) && (e = launch_gpow(kPrimes[i], s1, gpow_wg, stream)) != hipSuccess)
            return hip_fail(e, "g");
    prof.mark(0);
    for (int i = 0; i < 4; ++i) {
        if (!L.present[i]) continue;
        const int pp = kPrimes[i];
        if ((e = launch_plan(pp, (uint32_t *)(w + L.plan[i]), stream)) != hipSuccess) return hip_fail(e, "plan");
        prof.mark(1);
        DeepArgs da{};
        da.mode = MODE_HEIGHT;
        da.bound = bound;
        da.heights = heights;
        da.counters = counters;
        da.queue = (const int32_t *)(w + L.queue[i]);
        da.queue2 = (int32_t *)(w + L.queue2[i]);
        da.gq = w + L.gq[i];
        da.f = f;
        da.plan = (const uint32_t *)(w + L.plan[i]);
        da.slots = w + L.slots;
        da.slot_bytes = L.slot_stride[i];
        const int nslots = batch < L.nslots[i] ? batch : L.nslots[i];
        // the capped chain decides h = 2 for every deep surface; the rest take
        // the full chain in a second launch (balanced over all workgroups)
        if (band) {
            da.zero_halo = 1;
            if ((e = launch_deep(pp, true, da, nslots, stream)) != hipSuccess) return hip_fail(e, "deep band");
        }
        prof.mark(2 + i);
        da.from_q2 = band ? 1 : 0;
        da.zero_halo = band ? 0 : 1;
        if ((e = launch_deep(pp, false, da, nslots, stream)) != hipSuccess) return hip_fail(e, "deep");
        prof.mark(6 + i);
    }
    return QFS_OK;
}

int qfs_height(int batch, const int32_t *p, const uint8_t *f, int bound, int max_p, int32_t *heights, void *ws,
               size_t ws_bytes, hipStream_t stream)
{
    g_err[0] = 0;
    if (batch < 0) return fail(QFS_EINVAL, "qfs_height: batch=%d < 0", batch);
    if (bound < 1 || bound > 10) return fail(QFS_EINVAL, "qfs_height: bound=%d outside 1..10", bound);
    if (max_p < 3 || max_p > 11 || !supported(max_p))
        return fail(QFS_EUNSUPPORTED, "qfs_height: max_p=%d not in {3,5,7,11}", max_p);
    if (batch == 0) return QFS_OK;
    if (!p || !f || !heights || !ws) return fail(QFS_EINVAL, "qfs_height: null pointer argument");
    if (!aligned(ws)) return fail(QFS_EINVAL, "qfs_height: workspace not 256-byte aligned");
    const int ncu = device_cus();
    if (ncu <= 0) return fail(QFS_EDEVICE, "qfs_height: no HIP device");
    bool present[4];
    present_upto(max_p, present);
    const BatchLayout L = make_batch_layout(present, batch, deep_slots());
    if (ws_bytes < L.total)
        return fail(QFS_ENOMEM, "qfs_height: workspace %zu bytes < %zu needed", ws_bytes, L.total);
    const bool band = g_opt_height_band.load() && bound >= 2;
    const int gwg = gpow_workgroups(batch);
    for (int i = 0; i < 4; ++i) {
        hipError_t e;
        if (L.present[i] && (e = prepare_deep(kPrimes[i])) != hipSuccess) return hip_fail(e, "deep attributes");
    }
    ProfCall prof(stream);
    if (!g_opt_height_graph.load() || prof.on)
        return enqueue_height(batch, p, f, bound, L, heights, (uint8_t *)ws, band, gwg, stream, prof);

    // replay the graph of this exact call, or capture it on a library stream first
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEV) return fail(QFS_EDEVICE, "qfs_height: device");
    const GraphKey key{dev, batch, bound, max_p, band ? 1 : 0, deep_slots(), gwg, p, f, heights, ws, ws_bytes};
    std::lock_guard<std::mutex> lk(g_graphs.m);
    for (GraphEntry &en : g_graphs.v)
        if (en.key == key) {
            en.used = ++g_graphs.tick;
            const hipError_t e = hipGraphLaunch(en.exec, stream);
            return e == hipSuccess ? QFS_OK : hip_fail(e, "graph launch");
        }
    bool again = false;
    for (size_t i = 0; i < g_graphs.seen.size() && !again; ++i)
        if (g_graphs.seen[i] == key) {
            g_graphs.seen.erase(g_graphs.seen.begin() + i);
            again = true;
        }
    if (!again) {  // first time: launch directly and remember the arguments
        if (g_graphs.seen.size() >= 2 * GRAPH_CACHE) g_graphs.seen.erase(g_graphs.seen.begin());
        g_graphs.seen.push_back(key);
        return enqueue_height(batch, p, f, bound, L, heights, (uint8_t *)ws, band, gwg, stream, prof);
    }
    hipError_t e;
    if (!g_graphs.cap[dev] && (e = hipStreamCreateWithFlags(&g_graphs.cap[dev], hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "capture stream");
    hipStream_t cs = g_graphs.cap[dev];
    if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) return hip_fail(e, "capture");
    const int rc = enqueue_height(batch, p, f, bound, L, heights, (uint8_t *)ws, band, gwg, cs, prof);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    if (rc != QFS_OK || e != hipSuccess) {
        if (graph) hipGraphDestroy(graph);
        return rc != QFS_OK ? rc : hip_fail(e, "end capture");
    }
    hipGraphExec_t exec = nullptr;
    if ((e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
        hipGraphDestroy(graph);
        return hip_fail(e, "graph instantiate");
    }
    if (g_graphs.v.size() >= GRAPH_CACHE) {
        // evict the least recently used graph; its last launch must have finished
        size_t lru = 0;
        for (size_t i = 1; i < g_graphs.v.size(); ++i)
            if (g_graphs.v[i].used < g_graphs.v[lru].used) lru = i;
        hipDeviceSynchronize();
        destroy_entry(g_graphs.v[lru]);
        g_graphs.v.erase(g_graphs.v.begin() + lru);
    }
    g_graphs.v.push_back({key, graph, exec, ++g_graphs.tick});
    e = hipGraphLaunch(exec, stream);
    return e == hipSuccess ? QFS_OK : hip_fail(e, "graph launch");
}

int qfs_profile_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_prof.m);
    g_prof.on = on != 0;
    return QFS_OK;
}

int qfs_profile_collect(double ms[QFS_PROFILE_STAGES], int *calls)
{
    if (!ms || !calls) return fail(QFS_EINVAL, "qfs_profile_collect: null pointer");
    std::lock_guard<std::mutex> lk(g_prof.m);
    for (int i = 0; i < QFS_PROFILE_STAGES; ++i) ms[i] = 0;
    *calls = (int)g_prof.recs.size();
    int rc = QFS_OK;
    for (ProfRec &r : g_prof.recs) {
        for (int i = 0; i < r.n; ++i)
            if (hipEventSynchronize(r.ev[i]) != hipSuccess) rc = fail(QFS_EDEVICE, "qfs_profile_collect: event wait");
        for (int i = 1; i < r.n; ++i) {
            float t = 0;
            if (r.stage[i] >= 0 && hipEventElapsedTime(&t, r.ev[i - 1], r.ev[i]) == hipSuccess) ms[r.stage[i]] += t;
        }
        for (int i = 0; i < r.n; ++i) g_prof.pool.push_back(r.ev[i]);
    }
    g_prof.recs.clear();
    return rc;
}

int64_t qfs_mfma_per_surface(int p, int pass)
{
    if (!supported(p) || (pass != 0 && pass != 1)) return -1;
    return mfma_count(p, pass == 1);
}

int qfs_mfma_peak(int iters, int32_t *sink, double *tops, hipStream_t stream)
{
    g_err[0] = 0;
    if (iters < 1 || iters > 10000000 || !sink || !tops) return fail(QFS_EINVAL, "qfs_mfma_peak: bad argument");
    const int ncu = device_cus();
    if (ncu <= 0) return fail(QFS_EDEVICE, "qfs_mfma_peak: no HIP device");
    const int nwg = 8 * ncu;
    float ms = 0.0f;
    const hipError_t e = mfma_peak(iters, nwg, sink, &ms, stream);
    if (e != hipSuccess) return hip_fail(e, "mfma peak");
    *tops = ms > 0.0f ? (double)mfma_peak_ops(iters, nwg) / (ms * 1e-3) / 1e12 : 0.0;
    return QFS_OK;
}

int qfs_set_option(const char *name, int64_t value)
{
    if (!name) return fail(QFS_EINVAL, "qfs_set_option: null name");
    if (std::strcmp(name, "height_band") == 0) {
        if (value != 0 && value != 1) return fail(QFS_EINVAL, "qfs_set_option: height_band must be 0 or 1");
        g_opt_height_band.store(value != 0);
        return QFS_OK;
    }
    if (std::strcmp(name, "height_graph") == 0) {
        if (value != 0 && value != 1) return fail(QFS_EINVAL, "qfs_set_option: height_graph must be 0 or 1");
        g_opt_height_graph.store(value != 0);
        return QFS_OK;
    }
    if (std::strcmp(name, "deep_slots") == 0) {
        if (value < 0 || value > 65536) return fail(QFS_EINVAL, "qfs_set_option: deep_slots must be 0..65536");
        g_opt_deep_slots.store((int)value);
        return QFS_OK;
    }
    if (std::strcmp(name, "gpow_per_cu") == 0) {
        if (value < 1 || value > 64) return fail(QFS_EINVAL, "qfs_set_option: gpow_per_cu must be 1..64");
        g_opt_gpow_per_cu.store((int)value);
        return QFS_OK;
    }
    return fail(QFS_EINVAL, "qfs_set_option: unknown option '%s'", name);
}

int64_t qfs_get_option(const char *name)
{
    if (name && std::strcmp(name, "height_band") == 0) return g_opt_height_band.load() ? 1 : 0;
    if (name && std::strcmp(name, "height_graph") == 0) return g_opt_height_graph.load() ? 1 : 0;
    if (name && std::strcmp(name, "deep_slots") == 0) return g_opt_deep_slots.load();
    if (name && std::strcmp(name, "gpow_per_cu") == 0) return g_opt_gpow_per_cu.load();
    if (name && std::strcmp(name, "height_graphs_cached") == 0) {
        std::lock_guard<std::mutex> lk(g_graphs.m);
        return (int64_t)g_graphs.v.size();
    }
    if (name && std::strcmp(name, "chain_power_p3") == 0) return Geo<3>::J;
    if (name && std::strcmp(name, "chain_power_p5") == 0) return Geo<5>::J;
    if (name && std::strcmp(name, "chain_power_p7") == 0) return Geo<7>::J;
    if (name && std::strcmp(name, "chain_power_p11") == 0) return Geo<11>::J;
    return fail(QFS_EINVAL, "qfs_get_option: unknown option");
}

// ---------------------------------------------------------------------------
// Launch-configuration autotuner for qfs_height.
// ---------------------------------------------------------------------------
static void device_name(char *out, size_t n)
{
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        std::snprintf(out, n, "unknown");
        return;
    }
    std::snprintf(out, n, "%s", prop.gcnArchName);
    for (char *c = out; *c; ++c)
        if (*c == '"' || *c == '\\') *c = '_';
}

int qfs_autotune(int batch, const int32_t *p, const uint8_t *f, int bound, int max_p, int32_t *heights, void *ws,
                 size_t ws_bytes, hipStream_t stream, const char *cache_path, int reps)
{
    g_err[0] = 0;
    if (batch <= 0) return fail(QFS_EINVAL, "qfs_autotune: batch=%d must be positive", batch);
    if (reps < 1 || reps > 100) return fail(QFS_EINVAL, "qfs_autotune: reps=%d outside 1..100", reps);
    const int ncu = device_cus();
    if (ncu <= 0) return fail(QFS_EDEVICE, "qfs_autotune: no HIP device");
    if (max_p < 3 || max_p > 11 || !supported(max_p))
        return fail(QFS_EUNSUPPORTED, "qfs_autotune: max_p=%d not in {3,5,7,11}", max_p);
    {
        bool present[4];
        present_upto(max_p, present);
        if (ws_bytes < make_batch_layout(present, batch, ncu).total)
            return fail(QFS_ENOMEM, "qfs_autotune: workspace smaller than qfs_height needs with one slot per CU");
    }
    const int slots_save = g_opt_deep_slots.load(), gpow_save = g_opt_gpow_per_cu.load();
    const bool graph_save = g_opt_height_graph.load();
    g_opt_height_graph.store(false);  // time direct launches
    const int slot_c[3] = {ncu / 2, (3 * ncu) / 4, ncu};
    const int gpow_c[3] = {4, 8, 16};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = QFS_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = fail(QFS_EDEVICE, "qfs_autotune: events");
    float best = 1e30f, trial[9];
    int bs = ncu, bg = 8;
    for (int i = 0; i < 9 && rc == QFS_OK; ++i) {
        g_opt_deep_slots.store(slot_c[i / 3] > 0 ? slot_c[i / 3] : 1);
        g_opt_gpow_per_cu.store(gpow_c[i % 3]);
        rc = qfs_height(batch, p, f, bound, max_p, heights, ws, ws_bytes, stream);  // warm-up
        if (rc != QFS_OK) break;
        hipEventRecord(e0, stream);
        for (int r = 0; r < reps && rc == QFS_OK; ++r) rc = qfs_height(batch, p, f, bound, max_p, heights, ws, ws_bytes, stream);
        hipEventRecord(e1, stream);
        if (hipEventSynchronize(e1) != hipSuccess) rc = fail(QFS_EDEVICE, "qfs_autotune: event wait");
        float ms = 0;
        hipEventElapsedTime(&ms, e0, e1);
        trial[i] = ms / reps;
        if (rc == QFS_OK && trial[i] < best) {
            best = trial[i];
            bs = g_opt_deep_slots.load();
            bg = g_opt_gpow_per_cu.load();
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    g_opt_height_graph.store(graph_save);
    if (rc != QFS_OK) {
        g_opt_deep_slots.store(slots_save);
        g_opt_gpow_per_cu.store(gpow_save);
        return rc;
    }
    g_opt_deep_slots.store(bs == ncu ? 0 : bs);
    g_opt_gpow_per_cu.store(bg);
    if (cache_path) {
        FILE *fp = std::fopen(cache_path, "a");
        if (!fp) return fail(QFS_EINVAL, "qfs_autotune: cannot append to %s", cache_path);
        char name[128];
        device_name(name, sizeof name);
        std::fprintf(fp, "{\"device\": \"%s\", \"cus\": %d, \"max_p\": %d, \"batch\": %d, \"deep_slots\": %d, "
                         "\"gpow_per_cu\": %d, \"ms\": %.4f, \"trials_ms\": [",
                     name, ncu, max_p, batch, bs == ncu ? 0 : bs, bg, best);
        for (int i = 0; i < 9; ++i) std::fprintf(fp, "%s%.4f", i ? ", " : "", trial[i]);
        std::fprintf(fp, "]}\n");
        std::fclose(fp);
    }
    return QFS_OK;
}

int qfs_load_tuning(const char *cache_path, int max_p)
{
    g_err[0] = 0;
    if (!cache_path) return fail(QFS_EINVAL, "qfs_load_tuning: null path");
    FILE *fp = std::fopen(cache_path, "r");
    if (!fp) return fail(QFS_EINVAL, "qfs_load_tuning: cannot read %s", cache_path);
    char name[128], line[1024];
    device_name(name, sizeof name);
    const int ncu = device_cus();
    int found = 0, slots = 0, gpow = 8;
    while (std::fgets(line, sizeof line, fp)) {
        char dev[128] = "";
        int cus = 0, mp = 0, b = 0, ds = 0, gp = 0;
        if (std::sscanf(line, "{\"device\": \"%127[^\"]\", \"cus\": %d, \"max_p\": %d, \"batch\": %d, \"deep_slots\": %d, "
                              "\"gpow_per_cu\": %d",
                        dev, &cus, &mp, &b, &ds, &gp) == 6 &&
            std::strcmp(dev, name) == 0 && cus == ncu && mp == max_p && ds >= 0 && gp >= 1 && gp <= 64) {
            found = 1;  // the last matching line wins
            slots = ds;
            gpow = gp;
        }
    }
    std::fclose(fp);
    if (!found) return fail(QFS_EINVAL, "qfs_load_tuning: no entry for this device and max_p=%d", max_p);
    g_opt_deep_slots.store(slots);
    g_opt_gpow_per_cu.store(gpow);
    return QFS_OK;
}

// ---------------------------------------------------------------------------
size_t qfs_height_plain_workspace_bytes(int p) { return supported(p) ? plain_scratch_bytes(p) : 0; }

// ---------------------------------------------------------------------------
// Reduced heights: stage 1 (Fedder's test and the deep queues), then one
// persistent kernel per present prime.
// ---------------------------------------------------------------------------
static size_t reduced_layout(const bool present[4], int batch, size_t queue[4])
{
    size_t off = align256(CNT_WORDS * sizeof(int32_t));
    for (int i = 0; i < 4; ++i) {
        queue[i] = 0;
        if (!present[i]) continue;
        queue[i] = off;
        off += align256((size_t)batch * sizeof(int32_t));
    }
    return off;
}

size_t qfs_height_reduced_workspace_bytes(int batch, int max_p)
{
    if (batch < 0 || max_p < 3 || max_p > 11) return 0;
    bool present[4];
    present_upto(max_p, present);
    size_t q[4];
    return reduced_layout(present, batch, q);
}

int qfs_height_reduced(int batch, const int32_t *p, const uint8_t *f, int bound, int max_p, int32_t *heights,
                       void *ws, size_t ws_bytes, hipStream_t stream)
{
    g_err[0] = 0;
    if (batch < 0) return fail(QFS_EINVAL, "qfs_height_reduced: batch=%d < 0", batch);
    if (bound < 1 || bound > 10) return fail(QFS_EINVAL, "qfs_height_reduced: bound=%d outside 1..10", bound);
    if (max_p < 3 || max_p > 11 || !supported(max_p))
        return fail(QFS_EUNSUPPORTED, "qfs_height_reduced: max_p=%d not in {3,5,7,11}", max_p);
    if (batch == 0) return QFS_OK;
    if (!p || !f || !heights || !ws) return fail(QFS_EINVAL, "qfs_height_reduced: null pointer argument");
    if (!aligned(ws)) return fail(QFS_EINVAL, "qfs_height_reduced: workspace not 256-byte aligned");
    const int ncu = device_cus();
    if (ncu <= 0) return fail(QFS_EDEVICE, "qfs_height_reduced: no HIP device");
    bool present[4];
    present_upto(max_p, present);
    size_t qoff[4];
    const size_t need = reduced_layout(present, batch, qoff);
    if (ws_bytes < need)
        return fail(QFS_ENOMEM, "qfs_height_reduced: workspace %zu bytes < %zu needed", ws_bytes, need);
    uint8_t *w = (uint8_t *)ws;
    int32_t *counters = (int32_t *)w;
    hipError_t e;
    if ((e = launch_reset(counters, stream)) != hipSuccess) return hip_fail(e, "reset");
    Stage1Args s1{};
    s1.batch = batch;
    s1.mode = MODE_HEIGHT;
    s1.fixed_p = 0;
    s1.bound = bound;
    s1.p = p;
    s1.f = f;
    s1.heights = heights;
    s1.counters = counters;
    int mask = 0;
    for (int i = 0; i < 4; ++i) {
        s1.queue[i] = present[i] ? (int32_t *)(w + qoff[i]) : nullptr;
        s1.gq[i] = nullptr;
        if (present[i]) mask |= 1 << i;
    }
    s1.present_mask = mask;
    if ((e = launch_stage1(s1, stream)) != hipSuccess) return hip_fail(e, "stage1");
    for (int i = 0; i < 4; ++i) {
        if (!present[i]) continue;
        // LDS per workgroup grows with p; 8 per compute unit at p <= 7, 3 at p = 11
        const int nwg = ncu * (kPrimes[i] == 11 ? 3 : 8);
        if ((e = launch_reduced(kPrimes[i], s1, nwg, stream)) != hipSuccess) return hip_fail(e, "reduced");
    }
    return QFS_OK;
}

int qfs_height_plain(int p, int batch, const uint8_t *f, int bound, int32_t *heights, void *ws, size_t ws_bytes,
                     hipStream_t stream)
{
    g_err[0] = 0;
    if (!supported(p)) return fail(QFS_EUNSUPPORTED, "qfs_height_plain: p=%d not in {3,5,7,11}", p);
    if (batch < 0) return fail(QFS_EINVAL, "qfs_height_plain: batch=%d < 0", batch);
    if (bound < 1 || bound > 10) return fail(QFS_EINVAL, "qfs_height_plain: bound=%d outside 1..10", bound);
    if (batch == 0) return QFS_OK;
    if (!f || !heights || !ws) return fail(QFS_EINVAL, "qfs_height_plain: null pointer argument");
    if (!aligned(ws)) return fail(QFS_EINVAL, "qfs_height_plain: workspace not 256-byte aligned");
    const size_t need = plain_scratch_bytes(p);
    if (ws_bytes < need) return fail(QFS_ENOMEM, "qfs_height_plain: workspace %zu bytes < %zu needed", ws_bytes, need);
    for (int i = 0; i < batch; ++i) {
        hipError_t e = launch_plain_surface(p, f + (size_t)i * 35, bound, heights + i, (uint8_t *)ws, stream);
        if (e != hipSuccess) return hip_fail(e, "plain");
    }
    return QFS_OK;
}

}  // extern "C"
