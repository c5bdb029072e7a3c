// capi.hip -- the extern "C" entry points of libinim (declared in inim.h):
// argument validation, workspace layout and the launch sequence of each call.
#include <hip/hip_runtime.h>


#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "inim.h"
#include "inim_plan.h"
#include "launch.h"
#include "reg_layout.h"

using namespace inim;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* where) {
    return fail(INIM_EHIP, "%s: %s", where, hipGetErrorString(e));
}

bool valid_res(int32_t res) { return res >= 2 && res <= 16384 && (res & (res - 1)) == 0; }

int check_res(int32_t res) {
    if (!valid_res(res)) return fail(INIM_EINVAL, "res=%d is not a power of two in [2, 16384]", (int)res);
    return INIM_OK;
}

struct Params {
    int radius;
    double sigma;
    double d0;  // < 0: n / res^2
};

int resolve_params(const inim_params* p, Params& out) {
    inim_params d;
    inim_default_params(&d);
    if (p == nullptr) p = &d;
    if (p->radius < 0 || p->radius > kMaxRadius)
        return fail(INIM_EINVAL, "radius=%d outside [0, %d]", (int)p->radius, kMaxRadius);
    if (!std::isfinite(p->sigma)) return fail(INIM_EINVAL, "sigma is not finite");
    if (!std::isfinite(p->d0)) return fail(INIM_EINVAL, "d0 is not finite");
    out.radius = p->radius;
    out.sigma = p->sigma > 0.0f ? (double)p->sigma : 0.5 * (double)p->radius;
    out.d0 = p->d0;
    return INIM_OK;
}

// Normalised Gaussian taps exp(-m^2 / (2 sigma^2)), |m| <= r, summed in double.
BlurTaps make_taps(int r, double sigma) {
    BlurTaps t;
    std::memset(&t, 0, sizeof t);
    t.r = r;
    if (r == 0) {
        t.w[0] = 1.0f;
        return t;
    }
    double w[2 * kMaxRadius + 1], s = 0.0;
    for (int m = -r; m <= r; ++m) {
        w[m + r] = std::exp(-(double)m * m / (2.0 * sigma * sigma));
        s += w[m + r];
    }
    for (int k = 0; k <= 2 * r; ++k) t.w[k] = (float)(w[k] / s);
    return t;
}


int check_ws(const void* ws, size_t ws_bytes, size_t need) {
    if (ws == nullptr) return fail(INIM_EWORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws & 255u) != 0) return fail(INIM_EWORKSPACE, "workspace is not 256-byte aligned");
    if (ws_bytes < need) return fail(INIM_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    return INIM_OK;
}

int check_xy(const void* xy, int64_t n) {
    if (n < 0) return fail(INIM_EINVAL, "n=%lld is negative", (long long)n);
    if (n > 0 && xy == nullptr) return fail(INIM_EINVAL, "xy is NULL with n=%lld", (long long)n);
    if (n >= ((int64_t)1 << 32)) return fail(INIM_ERANGE, "n=%lld does not fit 32-bit counts", (long long)n);
    return INIM_OK;
}

// Events of the timed variant: per call the sort prologue and epilogue
// (recorded between launches), per iteration the start of the first and the
// end of the last kernel of each of the four stages (a StageClock).
struct StageEvents {
    hipEvent_t pre[2];
    hipEvent_t start[4], stop[4];
};

// Arms the stage clock for stage k while in scope (nothing without events).
struct ClockScope {
    StageClock c;
    bool on;
    ClockScope(StageEvents* ev, int k) : on(ev != nullptr) {
        if (on) {
            c.start = ev->start[k];
            c.stop = ev->stop[k];
            stage_clock() = &c;
        }
    }
    ~ClockScope() {
        if (on) stage_clock() = nullptr;
    }
};

// The whole call (Sec. 4.3) on the caller's stream.  The samples are first
// sorted by texel into the workspace (so that the splats of a wave mostly hit
// the same few texels and the field gathers are local), the iterations run on
// that copy, and the results are moved back to the caller's order.
// Iteration k reads the count raster counts[k % 2]; its advection splats the
// moved samples into counts[(k+1) % 2], which the smoothing of iteration k has
// zeroed.
// `status` is the call's status word: the workspace's own (ws + L.status) or
// one the caller keeps apart from the workspace.
int enqueue_regularize(float* xy, int64_t n, float* probe, int64_t m, int32_t res, int32_t iters, double d0,
                       const BlurTaps& taps, const RegLayout& L, char* ws, int* status, hipStream_t st,
                       StageEvents* ev, double* stage_ms) {
    uint32_t* counts[2] = {reinterpret_cast<uint32_t*>(ws + L.counts[0]), reinterpret_cast<uint32_t*>(ws + L.counts[1])};
    float* density = reinterpret_cast<float*>(ws + L.density);
    float2* field = reinterpret_cast<float2*>(ws + L.field);
    float2* pts = reinterpret_cast<float2*>(ws + L.sxy);
    uint32_t* map = reinterpret_cast<uint32_t*>(ws + L.rank);
    void* scratch = ws + L.scratch;
    const size_t NN = (size_t)res * res;
    const bool fused = L.f32 && blur_aggregate_fits(L.g);
    float2* defect = reinterpret_cast<float2*>(ws + L.defect);
    hipError_t e;
    if (ev) (void)hipEventRecord(ev->pre[0], st);
    // the density raster is free until the first smoothing: row totals
    e = launch_sort_by_texel(reinterpret_cast<const float2*>(xy), n, res, counts[0], map, counts[1],
                             reinterpret_cast<uint32_t*>(ws + L.partial), reinterpret_cast<uint32_t*>(density), pts,
                             reinterpret_cast<float2*>(ws + L.stage), reinterpret_cast<uint32_t*>(ws + L.idx), defect,
                             status, st);
    if (e != hipSuccess) return hip_fail(e, "sort by texel");
    if (m > 0 && (e = launch_validate(reinterpret_cast<const float2*>(probe), m, status, st)) != hipSuccess)
        return hip_fail(e, "validate probes");
    if (ev) {
        (void)hipEventRecord(ev->pre[1], st);
        if (hipEventSynchronize(ev->pre[1]) != hipSuccess) return fail(INIM_EHIP, "hipEventSynchronize failed");
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, ev->pre[0], ev->pre[1]);
        stage_ms[0] += ms;
    }
    for (int it = 0; it < iters; ++it) {
        uint32_t* cur = counts[it & 1];
        uint32_t* nxt = (it + 1 < iters) ? counts[(it + 1) & 1] : nullptr;
        {
            ClockScope clock(ev, 0);
            if (fused) {
                e = launch_blur_aggregate(cur, density, nxt, res, taps, L.g, scratch, status, st);
            } else if (L.f32) {
                e = launch_blur(cur, density, res, taps, status, st);
                if (e == hipSuccess && nxt) e = launch_fill(nxt, NN, status, false, st);
                if (e == hipSuccess) e = launch_inim_aggregate<float, double>(density, L.g, scratch, status, st);
            } else {
                e = launch_inim_aggregate<uint32_t, uint32_t>(cur, L.g, scratch, status, st);
            }
        }
        if (e != hipSuccess) return hip_fail(e, "smooth + aggregate");
        {
            ClockScope clock(ev, 1);
            e = L.f32 ? launch_inim_scans<double>(L.g, scratch, status, st)
                      : launch_inim_scans<uint32_t>(L.g, scratch, status, st);
        }
        if (e != hipSuccess) return hip_fail(e, "integral-image scans");
        {
            ClockScope clock(ev, 2);
            if (L.f32)
                e = launch_inim_final<float, double>(density, L.g, scratch, 0u, nullptr, field, defect, d0, nullptr,
                                                     status, st);
            else
                e = launch_inim_final<uint32_t, uint32_t>(cur, L.g, scratch, 0u, nullptr, field, defect, d0, nullptr,
                                                          status, st);
            if (e == hipSuccess && !L.f32 && nxt) e = launch_fill(nxt, NN, status, false, st);
        }
        if (e != hipSuccess) return hip_fail(e, "integral images + deformation");
        {
            ClockScope clock(ev, 3);
            e = launch_advect(field, res, pts, n, nxt, status, st);
            if (e == hipSuccess && m > 0)
                e = launch_advect(field, res, reinterpret_cast<float2*>(probe), m, nullptr, status, st);
        }
        if (e != hipSuccess) return hip_fail(e, "advect");
        if (ev) {
            if (hipEventSynchronize(ev->stop[3]) != hipSuccess) return fail(INIM_EHIP, "hipEventSynchronize failed");
            for (int k = 0; k < 4; ++k) {
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, ev->start[k], ev->stop[k]);
                stage_ms[1 + k] += ms;
            }
        }
    }
    if (ev) (void)hipEventRecord(ev->pre[0], st);
    if ((e = launch_unpermute(pts, map, n, res, reinterpret_cast<float2*>(xy), status, st)) != hipSuccess)
        return hip_fail(e, "unpermute");
    if (ev) {
        (void)hipEventRecord(ev->pre[1], st);
        if (hipEventSynchronize(ev->pre[1]) != hipSuccess) return fail(INIM_EHIP, "hipEventSynchronize failed");
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, ev->pre[0], ev->pre[1]);
        stage_ms[0] += ms;
    }
    return INIM_OK;
}

int regularize_impl(float* xy, int64_t n, float* probe, int64_t m, int32_t res, int32_t iters, const inim_params* p,
                    void* ws, size_t ws_bytes, hipStream_t stream, double* stage_ms) {
    int s;
    if ((s = check_res(res)) != INIM_OK) return s;
    if ((s = check_xy(xy, n)) != INIM_OK) return s;
    if (m < 0) return fail(INIM_EINVAL, "m=%lld is negative", (long long)m);
    if (m > 0 && probe == nullptr) return fail(INIM_EINVAL, "probe is NULL with m=%lld", (long long)m);
    if (iters < 0) return fail(INIM_EINVAL, "iters=%d is negative", (int)iters);
    Params P;
    if ((s = resolve_params(p, P)) != INIM_OK) return s;
    const RegLayout L = reg_layout(res, n, P.radius);
    if ((s = check_ws(ws, ws_bytes, L.total)) != INIM_OK) return s;
    if (n == 0 || iters == 0) {
        // nothing to do, but the call still resets the status word it reports
        hipError_t e = launch_fill(nullptr, 0, reinterpret_cast<int*>((char*)ws + L.status), true, stream);
        return e == hipSuccess ? INIM_OK : hip_fail(e, "fill");
    }
    const double d0 = P.d0 < 0.0 ? (double)n / ((double)res * (double)res) : P.d0;
    const BlurTaps taps = make_taps(P.radius, P.sigma);
    if (stage_ms == nullptr)
        return enqueue_regularize(xy, n, probe, m, res, iters, d0, taps, L, (char*)ws,
                                  reinterpret_cast<int*>((char*)ws + L.status), stream, nullptr, nullptr);

    StageEvents ev;
    hipEvent_t t0, t1;
    hipEvent_t* all[12] = {&ev.pre[0], &ev.pre[1], &ev.start[0], &ev.start[1], &ev.start[2], &ev.start[3],
                           &ev.stop[0],   &ev.stop[1],  &ev.stop[2],  &ev.stop[3],  &t0,           &t1};
    for (auto* h : all)
        if (hipEventCreate(h) != hipSuccess) return fail(INIM_EHIP, "hipEventCreate failed");
    (void)hipEventRecord(t0, stream);
    s = enqueue_regularize(xy, n, probe, m, res, iters, d0, taps, L, (char*)ws,
                           reinterpret_cast<int*>((char*)ws + L.status), stream, &ev, stage_ms);
    (void)hipEventRecord(t1, stream);
    if (s == INIM_OK && hipEventSynchronize(t1) == hipSuccess) {
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, t0, t1);
        stage_ms[5] += ms;
    }
    for (auto* h : all) (void)hipEventDestroy(*h);
    return s;
}

}  // namespace

namespace {

// ------------------------------------------------------------------ batched plots
// The plots of one batched call that have samples (plots with n == 0 are
// left untouched, as inim_regularize leaves them), in input order.
struct BatchPlan {
    BatchArgs a;
    int index[kMaxBatch];  // input position of each active plot
    unsigned blocks[kBStages];
    size_t total;
    BlurTaps taps;
};

int batch_plan(float* const* xy, const int64_t* n, const int32_t* res, int32_t count, const inim_params* p,
               const inim_batch_config* cfg, BatchPlan& B) {
    int s;
    if (count < 0 || count > kMaxBatch) return fail(INIM_EINVAL, "count=%d outside [0, %d]", (int)count, kMaxBatch);
    if (count > 0 && (xy == nullptr || n == nullptr || res == nullptr))
        return fail(INIM_EINVAL, "xy, n or res is NULL");
    Params P;
    if ((s = resolve_params(p, P)) != INIM_OK) return s;
    if (P.radius < 1) return fail(INIM_EINVAL, "batched plots need radius >= 1");
    const int wpb = (cfg && cfg->waves_per_block) ? cfg->waves_per_block : 4;
    if (wpb != 1 && wpb != 2 && wpb != 4 && wpb != 8)
        return fail(INIM_EINVAL, "waves_per_block=%d is not 1, 2, 4 or 8", (int)wpb);
    const int order = cfg ? cfg->order : 0;
    if (order != 0 && order != 1) return fail(INIM_EINVAL, "order=%d is not 0 or 1", (int)order);
    std::memset(&B.a, 0, sizeof B.a);
    int m = 0;
    for (int k = 0; k < count; ++k) {
        if ((s = check_res(res[k])) != INIM_OK) return s;
        if (res[k] < 64 || res[k] > 2048) return fail(INIM_EINVAL, "plot %d: res=%d outside [64, 2048]", k, (int)res[k]);
        if ((s = check_xy(xy[k], n[k])) != INIM_OK) return s;
        if (n[k] == 0) continue;
        B.a.in[m].xy = xy[k];
        B.a.in[m].n = n[k];
        B.a.in[m].N = res[k];
        B.index[m] = k;
        ++m;
    }
    B.a.count = m;
    B.a.wpb = wpb;
    B.a.radius = P.radius;
    B.a.d0 = P.d0;
    for (int q = 0; q < m; ++q) B.a.order[q] = q;
    if (order == 1)  // larger rasters first (then more samples), ties in input order
        std::stable_sort(B.a.order, B.a.order + m, [&](int u, int v) {
            const BatchInput &U = B.a.in[u], &V = B.a.in[v];
            return U.N != V.N ? U.N > V.N : U.n > V.n;
        });
    for (int st = 0; st < kBStages; ++st) {
        unsigned run = 0;
        for (int q = 0; q < m; ++q) {
            bool own = true;
            for (int r = 0; r < q; ++r)
                if (B.a.in[r].N == B.a.in[q].N) { own = false; break; }
            run += batch_stage_blocks(st, B.a.in[q].N, B.a.in[q].n, wpb, own);
        }
        B.blocks[st] = run;
    }
    B.total = batch_plot_offset(m, B.a.in, P.radius);
    B.taps = make_taps(P.radius, P.sigma);
    return INIM_OK;
}

// The batched call on `st`; with `dry` the results stay in the workspace
// (the samples' positions in the caller's arrays are not written).
int enqueue_batch(BatchPlan& B, int32_t iters, char* ws, hipStream_t st, bool dry) {
    B.a.ws = ws;
    int* status = reinterpret_cast<int*>(ws);
    BatchTable* T = reinterpret_cast<BatchTable*>(ws + batch_table_offset());
    hipError_t e = launch_batch_init(B.a, T, st);
    for (int s : {kBFill, kBSplatRank, kBScanReduce, kBScanPartials, kBScanDown, kBScatter, kBRowHist, kBRowScan,
                  kBRowBucket, kBRowSort})
        if (e == hipSuccess) e = launch_batch_raster(s, T, B.blocks[s], 0, iters, status, st);
    if (e == hipSuccess) e = launch_batch_inim(kBDefect, T, B.blocks[kBDefect], B.a.wpb, B.taps, 0, iters, status, st);
    for (int it = 0; it < iters && e == hipSuccess; ++it) {
        for (int s : {kBBlurAgg, kBScanCol, kBScanDiag, kBDeform})
            if (e == hipSuccess) e = launch_batch_inim(s, T, B.blocks[s], B.a.wpb, B.taps, it, iters, status, st);
        if (e == hipSuccess) e = launch_batch_raster(kBAdvect, T, B.blocks[kBAdvect], it, iters, status, st);
    }
    if (e == hipSuccess && !dry) e = launch_batch_raster(kBUnpermute, T, B.blocks[kBUnpermute], 0, iters, status, st);
    return e == hipSuccess ? INIM_OK : hip_fail(e, "batched regularisation");
}

}  // namespace

struct inim_graph_cache {
    bool valid = false;
    std::vector<char> key;  // every argument of the captured call, as bytes
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    void drop() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        valid = false;
    }
};

namespace {

// Argument bytes of a call, the key of a captured graph.
struct KeyWriter {
    std::vector<char> bytes;
    template <typename T>
    KeyWriter& put(const T& v) {
        const char* p = reinterpret_cast<const char*>(&v);
        bytes.insert(bytes.end(), p, p + sizeof(T));
        return *this;
    }
};

// Launches the graph of G on `stream`, first capturing `enqueue` (on G's
// private stream) when `key` differs from the captured call's.
template <typename Enqueue>
int graph_launch(inim_graph_cache* G, const std::vector<char>& key, hipStream_t stream, Enqueue enqueue) {
    if (!(G->valid && G->key == key)) {
        G->drop();
        if (G->capture == nullptr && hipStreamCreateWithFlags(&G->capture, hipStreamNonBlocking) != hipSuccess)
            return fail(INIM_EHIP, "hipStreamCreate failed");
        hipError_t e = hipStreamBeginCapture(G->capture, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        const int s = enqueue(G->capture);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(G->capture, &g);
        if (s != INIM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        G->graph = g;
        e = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            G->drop();
            return hip_fail(e, "hipGraphInstantiate");
        }
        G->valid = true;
        G->key = key;
    }
    hipError_t e = hipGraphLaunch(G->exec, stream);
    return e == hipSuccess ? INIM_OK : hip_fail(e, "hipGraphLaunch");
}

}  // namespace

// ------------------------------------------------------------------ static scratch
// The workspace of inim_regularize_noalloc: a fixed array in device memory,
// one copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol); it looks up each device's address once, with that device current,
// and uses that address.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices];

// The device address of `scratch` on the current device, which must be the
// device of `stream` (the null stream: the current device).
int static_scratch(hipStream_t stream, char** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (stream != nullptr) {
        int sdev = -1;
        if ((e = hipStreamGetDevice(stream, &sdev)) != hipSuccess) return hip_fail(e, "hipStreamGetDevice");
        if (sdev != dev) return fail(INIM_EINVAL, "stream is on device %d, the current device is %d", sdev, dev);
    }
    if (dev < 0 || dev >= kMaxDevices) return fail(INIM_EINVAL, "device %d is beyond the first %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* ptr = nullptr;
        if ((e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != hipSuccess)
            return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (ptr == nullptr || ((uintptr_t)ptr & 255u) != 0)
            return fail(INIM_EHIP, "static scratch at %p is not 256-byte aligned", ptr);
        g_scratch_ptr[dev] = static_cast<char*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return INIM_OK;
}

}  // namespace

extern "C" {

void inim_default_params(inim_params* p) {
    if (!p) return;
    p->radius = 8;
    p->sigma = 0.0f;  // unset: radius / 2 at resolve time
    p->d0 = -1.0;
}

const char* inim_strerror(int status) {
    switch (status) {
        case INIM_OK: return "ok";
        case INIM_EINVAL: return "invalid argument";
        case INIM_EDOMAIN: return "a sample is NaN or outside the unit square";
        case INIM_ERANGE: return "sample count exceeds 32-bit counts";
        case INIM_EWORKSPACE: return "workspace missing, misaligned or too small";
        case INIM_EHIP: return "HIP runtime error";
    }
    return "unknown status";
}

const char* inim_last_error(void) { return g_last_error.c_str(); }

int inim_workspace_size(int32_t res, int64_t n, const inim_params* p, size_t* bytes) {
    int s;
    if (bytes == nullptr) return fail(INIM_EINVAL, "bytes is NULL");
    if ((s = check_res(res)) != INIM_OK) return s;
    if (n < 0) return fail(INIM_EINVAL, "n=%lld is negative", (long long)n);
    Params P;
    if ((s = resolve_params(p, P)) != INIM_OK) return s;
    *bytes = reg_layout(res, n, P.radius).total;
    return INIM_OK;
}

int inim_inim_workspace_size(int32_t res, inim_dtype dt, size_t* bytes) {
    int s;
    if (bytes == nullptr) return fail(INIM_EINVAL, "bytes is NULL");
    if ((s = check_res(res)) != INIM_OK) return s;
    if (dt != INIM_U32 && dt != INIM_F32) return fail(INIM_EINVAL, "unknown dtype %d", (int)dt);
    // float rasters: the exact accumulators' scratch, which also holds the
    // double-accumulated pass of alpha + alpha_t calls (same tiling, half the bytes)
    *bytes = kStatusBytes + inim_scratch_bytes(make_geom(res, dt == INIM_F32 ? 16 : 4), dt == INIM_F32 ? 16 : 4);
    return INIM_OK;
}

int inim_rasterize(const float* xy, int64_t n, int32_t res, const inim_params* p, uint32_t* counts, float* density,
                   void* ws, size_t ws_bytes, hipStream_t stream) {
    int s;
    if ((s = check_res(res)) != INIM_OK) return s;
    if ((s = check_xy(xy, n)) != INIM_OK) return s;
    if (counts == nullptr) return fail(INIM_EINVAL, "counts is NULL");
    Params P;
    if ((s = resolve_params(p, P)) != INIM_OK) return s;
    if ((s = check_ws(ws, ws_bytes, kStatusBytes)) != INIM_OK) return s;
    int* status = reinterpret_cast<int*>(ws);
    const size_t NN = (size_t)res * res;
    hipError_t e;
    if ((e = launch_fill(counts, NN, status, true, stream)) != hipSuccess) return hip_fail(e, "fill");
    if ((e = launch_splat(reinterpret_cast<const float2*>(xy), n, res, counts, status, stream)) != hipSuccess)
        return hip_fail(e, "splat");
    if (density != nullptr) {
        const BlurTaps taps = make_taps(P.radius, P.sigma);
        if ((e = launch_blur(counts, density, res, taps, status, stream)) != hipSuccess) return hip_fail(e, "blur");
    }
    return INIM_OK;
}

// The sets of a *_many call, checked, into a SetTable.
static int set_table(float* const* xy, const int64_t* n, int32_t count, SetTable& t) {
    if (count < 1 || count > kMaxSets) return fail(INIM_EINVAL, "count=%d outside [1, %d]", (int)count, kMaxSets);
    if (xy == nullptr || n == nullptr) return fail(INIM_EINVAL, "xy or n is NULL");
    t.count = count;
    for (int q = 0; q < count; ++q) {
        int s;
        if ((s = check_xy(xy[q], n[q])) != INIM_OK) return s;
        t.xy[q] = reinterpret_cast<float2*>(xy[q]);
        t.n[q] = n[q];
    }
    return INIM_OK;
}

int inim_rasterize_many(float* const* xy, const int64_t* n, int32_t count, int32_t res, const inim_params* p,
                        uint32_t* counts, float* density, void* ws, size_t ws_bytes, hipStream_t stream) {
    int s;
    if ((s = check_res(res)) != INIM_OK) return s;
    SetTable t;
    if ((s = set_table(xy, n, count, t)) != INIM_OK) return s;
    if (counts == nullptr) return fail(INIM_EINVAL, "counts is NULL");
    Params P;
    if ((s = resolve_params(p, P)) != INIM_OK) return s;
    if ((s = check_ws(ws, ws_bytes, kStatusBytes)) != INIM_OK) return s;
    int* status = reinterpret_cast<int*>(ws);
    const size_t NN = (size_t)res * res;
    hipError_t e;
    if ((e = launch_fill(counts, NN * count, status, true, stream)) != hipSuccess) return hip_fail(e, "fill");
    if ((e = launch_splat_many(t, res, counts, status, stream)) != hipSuccess) return hip_fail(e, "splat");
    if (density != nullptr) {
        const BlurTaps taps = make_taps(P.radius, P.sigma);
        if ((e = launch_blur_many(counts, density, res, count, taps, status, stream)) != hipSuccess)
            return hip_fail(e, "blur");
    }
    return INIM_OK;
}

int inim_advect_many(const float* field, int32_t res, float* const* xy, const int64_t* n, int32_t count, void* ws,
                     size_t ws_bytes, hipStream_t stream) {
    int s;
    if ((s = check_res(res)) != INIM_OK) return s;
    SetTable t;
    if ((s = set_table(xy, n, count, t)) != INIM_OK) return s;
    if (field == nullptr) return fail(INIM_EINVAL, "field is NULL");
    if ((s = check_ws(ws, ws_bytes, kStatusBytes)) != INIM_OK) return s;
    int* status = reinterpret_cast<int*>(ws);
    hipError_t e;
    if ((e = launch_fill(nullptr, 0, status, true, stream)) != hipSuccess) return hip_fail(e, "fill");
    if ((e = launch_advect_many(t, reinterpret_cast<const float2*>(field), res, status, stream)) != hipSuccess)
        return hip_fail(e, "advect");
    return INIM_OK;
}

static int inim_common(const void* img, int32_t res, uint32_t mask, const void* planes, void* ws, size_t ws_bytes,
                       inim_dtype dt) {
    int s;
    if ((s = check_res(res)) != INIM_OK) return s;
    if (img == nullptr) return fail(INIM_EINVAL, "img is NULL");
    if (mask & ~(uint32_t)INIM_ALL) return fail(INIM_EINVAL, "mask 0x%x has unknown bits", mask);
    if (mask != 0 && planes == nullptr) return fail(INIM_EINVAL, "planes is NULL with mask 0x%x", mask);
    size_t need;
    inim_inim_workspace_size(res, dt, &need);
    return check_ws(ws, ws_bytes, need);
}

int inim_inim_u32(const uint32_t* img, int32_t res, uint32_t mask, uint32_t* planes, double* marg, void* ws,
                  size_t ws_bytes, hipStream_t stream) {
    int s = inim_common(img, res, mask, planes, ws, ws_bytes, INIM_U32);
    if (s != INIM_OK) return s;
    if (mask == 0 && marg == nullptr) return INIM_OK;
    void* scratch = (char*)ws + kStatusBytes;
    const Geom g = make_geom(res, 4);
    hipError_t e = launch_inim_carries<uint32_t, uint32_t>(img, g, scratch, nullptr, stream);
    if (e == hipSuccess) e = launch_inim_final<uint32_t, uint32_t>(img, g, scratch, mask, planes, nullptr, nullptr, 0.0, marg, nullptr,
                                                                stream);
    return e == hipSuccess ? INIM_OK : hip_fail(e, "integral images");
}

int inim_inim_f32(const float* img, int32_t res, uint32_t mask, float* planes, double* marg, void* ws,
                  size_t ws_bytes, hipStream_t stream) {
    int s = inim_common(img, res, mask, planes, ws, ws_bytes, INIM_F32);
    if (s != INIM_OK) return s;
    if (mask == 0 && marg == nullptr) return INIM_OK;
    const Geom g = make_geom(res, 16);
    void* scratch = (char*)ws + kStatusBytes;
    const int* skip = nullptr;
    if ((mask & ~(uint32_t)INIM_MIN) == 0) {
        // alpha and alpha_t only: no complement, so for rasters without
        // negative or non-finite values the sums run in double (no
        // cancellation); the aggregate pass clears the skip word (the second
        // word of ws) when it meets such a value, and the exact path below,
        // which runs only then, redoes the call
        int* words = reinterpret_cast<int*>(ws);
        const Geom gd = make_geom(res, 8);
        hipError_t e1 = launch_set_word(words + 1, 1, stream);
        if (e1 == hipSuccess) e1 = launch_inim_aggregate<float, double>(img, gd, scratch, nullptr, stream, words + 1);
        if (e1 == hipSuccess) e1 = launch_inim_scans<double>(gd, scratch, nullptr, stream);
        if (e1 == hipSuccess)
            e1 = launch_inim_final<float, double>(img, gd, scratch, mask, planes, nullptr, nullptr, 0.0, marg, nullptr,
                                                 stream);
        if (e1 != hipSuccess) return hip_fail(e1, "integral images");
        skip = words + 1;
    }
    hipError_t e = launch_inim_carries<float, u128>(img, g, scratch, skip, stream);
    if (e == hipSuccess) e = launch_inim_final<float, u128>(img, g, scratch, mask, planes, nullptr, nullptr, 0.0, marg, skip,
                                                         stream);
    return e == hipSuccess ? INIM_OK : hip_fail(e, "integral images");
}

int inim_deform(const void* alpha, const void* alpha_t, inim_dtype dt, const double* marg, int32_t res, double d0,
                float* field, hipStream_t stream) {
    int s;
    if ((s = check_res(res)) != INIM_OK) return s;
    if (alpha == nullptr || alpha_t == nullptr || marg == nullptr || field == nullptr)
        return fail(INIM_EINVAL, "NULL pointer argument");
    if (dt != INIM_U32 && dt != INIM_F32) return fail(INIM_EINVAL, "unknown dtype %d", (int)dt);
    if (!(d0 >= 0.0) || !std::isfinite(d0)) return fail(INIM_EINVAL, "d0 must be finite and >= 0");
    hipError_t e = launch_deform_planes(alpha, alpha_t, (int)dt, marg, res, d0, reinterpret_cast<float2*>(field),
                                        stream);
    return e == hipSuccess ? INIM_OK : hip_fail(e, "deform");
}

int inim_deform_density_workspace_size(int32_t res, size_t* bytes) {
    int s;
    if (bytes == nullptr) return fail(INIM_EINVAL, "bytes is NULL");
    if ((s = check_res(res)) != INIM_OK) return s;
    const size_t NN = (size_t)res * (size_t)res;
    *bytes = align256(NN * sizeof(float2)) + inim_scratch_bytes(make_geom(res, 8), 8);
    return INIM_OK;
}

int inim_deform_density(const float* density, int32_t res, double d0, float* field, void* ws, size_t ws_bytes,
                        hipStream_t stream) {
    int s;
    size_t need = 0;
    if ((s = inim_deform_density_workspace_size(res, &need)) != INIM_OK) return s;
    if (density == nullptr || field == nullptr) return fail(INIM_EINVAL, "NULL pointer argument");
    if (!(d0 >= 0.0) || !std::isfinite(d0)) return fail(INIM_EINVAL, "d0 must be finite and >= 0");
    if ((s = check_ws(ws, ws_bytes, need)) != INIM_OK) return s;
    const size_t NN = (size_t)res * (size_t)res;
    float2* defect = reinterpret_cast<float2*>(ws);
    void* scratch = static_cast<char*>(ws) + align256(NN * sizeof(float2));
    const Geom g = make_geom(res, 8);
    hipError_t e = launch_defect_field(res, defect, stream);
    if (e == hipSuccess) e = launch_inim_aggregate<float, double>(density, g, scratch, nullptr, stream);
    if (e == hipSuccess) e = launch_inim_scans<double>(g, scratch, nullptr, stream);
    if (e == hipSuccess)
        e = launch_inim_final<float, double>(density, g, scratch, 0u, nullptr, reinterpret_cast<float2*>(field),
                                             defect, d0, nullptr, nullptr, stream);
    return e == hipSuccess ? INIM_OK : hip_fail(e, "deform density");
}

int inim_advect(const float* field, int32_t res, float* xy, int64_t n, void* ws, size_t ws_bytes,
                hipStream_t stream) {
    int s;
    if ((s = check_res(res)) != INIM_OK) return s;
    if ((s = check_xy(xy, n)) != INIM_OK) return s;
    if (field == nullptr) return fail(INIM_EINVAL, "field is NULL");
    if ((s = check_ws(ws, ws_bytes, kStatusBytes)) != INIM_OK) return s;
    int* status = reinterpret_cast<int*>(ws);
    hipError_t e;
    if ((e = launch_fill(nullptr, 0, status, true, stream)) != hipSuccess) return hip_fail(e, "fill");
    if (n == 0) return INIM_OK;
    if ((e = launch_validate(reinterpret_cast<const float2*>(xy), n, status, stream)) != hipSuccess)
        return hip_fail(e, "validate");
    if ((e = launch_advect(reinterpret_cast<const float2*>(field), res, reinterpret_cast<float2*>(xy), n, nullptr,
                           status, stream)) != hipSuccess)
        return hip_fail(e, "advect");
    return INIM_OK;
}

int inim_regularize(float* xy, int64_t n, int32_t res, int32_t iters, const inim_params* p, void* ws,
                    size_t ws_bytes, hipStream_t stream) {
    return regularize_impl(xy, n, nullptr, 0, res, iters, p, ws, ws_bytes, stream, nullptr);
}

int inim_regularize_probes(float* xy, int64_t n, float* probe, int64_t m, int32_t res, int32_t iters,
                           const inim_params* p, void* ws, size_t ws_bytes, hipStream_t stream) {
    return regularize_impl(xy, n, probe, m, res, iters, p, ws, ws_bytes, stream, nullptr);
}

int inim_regularize_timed(float* xy, int64_t n, int32_t res, int32_t iters, const inim_params* p, void* ws,
                          size_t ws_bytes, hipStream_t stream, double* stage_ms) {
    if (stage_ms == nullptr) return fail(INIM_EINVAL, "stage_ms is NULL");
    return regularize_impl(xy, n, nullptr, 0, res, iters, p, ws, ws_bytes, stream, stage_ms);
}

int inim_graph_create(void** graph) {
    if (graph == nullptr) return fail(INIM_EINVAL, "graph is NULL");
    *graph = new inim_graph_cache();
    return INIM_OK;
}

int inim_graph_destroy(void* graph) {
    auto* G = static_cast<inim_graph_cache*>(graph);
    if (G == nullptr) return INIM_OK;
    G->drop();
    if (G->capture) (void)hipStreamDestroy(G->capture);
    delete G;
    return INIM_OK;
}

int inim_regularize_graph(float* xy, int64_t n, int32_t res, int32_t iters, const inim_params* p, void* ws,
                          size_t ws_bytes, void* graph, hipStream_t stream) {
    auto* G = static_cast<inim_graph_cache*>(graph);
    if (G == nullptr) return fail(INIM_EINVAL, "graph is NULL");
    int s;
    if ((s = check_res(res)) != INIM_OK) return s;
    if ((s = check_xy(xy, n)) != INIM_OK) return s;
    if (iters < 0) return fail(INIM_EINVAL, "iters=%d is negative", (int)iters);
    Params P;
    if ((s = resolve_params(p, P)) != INIM_OK) return s;
    const RegLayout L = reg_layout(res, n, P.radius);
    if ((s = check_ws(ws, ws_bytes, L.total)) != INIM_OK) return s;
    if (n == 0 || iters == 0) return regularize_impl(xy, n, nullptr, 0, res, iters, p, ws, ws_bytes, stream, nullptr);
    KeyWriter k;
    k.put(1).put(xy).put(n).put(res).put(iters).put(P.radius).put(P.sigma).put(P.d0).put(ws).put(ws_bytes);
    const double d0 = P.d0 < 0.0 ? (double)n / ((double)res * (double)res) : P.d0;
    const BlurTaps taps = make_taps(P.radius, P.sigma);
    return graph_launch(G, k.bytes, stream, [&](hipStream_t cs) {
        return enqueue_regularize(xy, n, nullptr, 0, res, iters, d0, taps, L, (char*)ws,
                                  reinterpret_cast<int*>((char*)ws + L.status), cs, nullptr, nullptr);
    });
}

int inim_batch_workspace_size(float* const* xy, const int64_t* n, const int32_t* res, int32_t count,
                              const inim_params* p, size_t* bytes) {
    if (bytes == nullptr) return fail(INIM_EINVAL, "bytes is NULL");
    BatchPlan B;
    const int s = batch_plan(xy, n, res, count, p, nullptr, B);
    if (s != INIM_OK) return s;
    *bytes = B.total;
    return INIM_OK;
}

int inim_regularize_batch(float* const* xy, const int64_t* n, const int32_t* res, int32_t count, int32_t iters,
                          const inim_params* p, const inim_batch_config* cfg, void* ws, size_t ws_bytes, void* graph,
                          hipStream_t stream) {
    BatchPlan B;
    int s = batch_plan(xy, n, res, count, p, cfg, B);
    if (s != INIM_OK) return s;
    if (iters < 0) return fail(INIM_EINVAL, "iters=%d is negative", (int)iters);
    if ((s = check_ws(ws, ws_bytes, B.total)) != INIM_OK) return s;
    if (B.a.count == 0 || iters == 0) {
        hipError_t e = launch_fill(nullptr, 0, reinterpret_cast<int*>(ws), true, stream);
        return e == hipSuccess ? INIM_OK : hip_fail(e, "fill");
    }
    if (graph == nullptr) return enqueue_batch(B, iters, (char*)ws, stream, false);
    KeyWriter k;
    k.put(2).put(iters).put(ws).put(ws_bytes).put(B.a).put(B.taps);
    return graph_launch(static_cast<inim_graph_cache*>(graph), k.bytes, stream,
                        [&](hipStream_t cs) { return enqueue_batch(B, iters, (char*)ws, cs, false); });
}

int inim_batch_autotune(float* const* xy, const int64_t* n, const int32_t* res, int32_t count, int32_t iters,
                        const inim_params* p, void* ws, size_t ws_bytes, hipStream_t stream,
                        inim_batch_config* best, double* best_ms) {
    if (best == nullptr) return fail(INIM_EINVAL, "best is NULL");
    BatchPlan B;
    int s = batch_plan(xy, n, res, count, p, nullptr, B);
    if (s != INIM_OK) return s;
    if (iters < 1) return fail(INIM_EINVAL, "iters=%d: tuning needs at least one iteration", (int)iters);
    if ((s = check_ws(ws, ws_bytes, B.total)) != INIM_OK) return s;
    best->waves_per_block = 4;
    best->order = 0;
    if (best_ms) *best_ms = 0.0;
    if (B.a.count == 0) return INIM_OK;
    hipEvent_t t0, t1;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)
        return fail(INIM_EHIP, "hipEventCreate failed");
    double bestv = 1e300;
    for (int order = 0; order < 2 && s == INIM_OK; ++order) {
        for (int wpb : {1, 2, 4, 8}) {
            const inim_batch_config c{wpb, order};
            BatchPlan C;
            if ((s = batch_plan(xy, n, res, count, p, &c, C)) != INIM_OK) break;
            float ms_min = 1e30f;
            for (int rep = 0; rep < 3 && s == INIM_OK; ++rep) {  // the first run warms up
                (void)hipEventRecord(t0, stream);
                s = enqueue_batch(C, iters, (char*)ws, stream, true);
                (void)hipEventRecord(t1, stream);
                if (s == INIM_OK && hipEventSynchronize(t1) != hipSuccess) s = fail(INIM_EHIP, "hipEventSynchronize");
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, t0, t1);
                if (rep > 0 && ms < ms_min) ms_min = ms;
            }
            if (s != INIM_OK) break;
            if (ms_min < bestv) {
                bestv = ms_min;
                *best = c;
            }
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (s == INIM_OK && best_ms) *best_ms = bestv;
    return s;
}

int inim_regularize_noalloc(float* xy, int64_t n, int32_t res, int32_t iters, const inim_params* p, int* status,
                            hipStream_t stream) {
    int s;
    if ((s = check_res(res)) != INIM_OK) return s;
    if ((s = check_xy(xy, n)) != INIM_OK) return s;
    if (iters < 0) return fail(INIM_EINVAL, "iters=%d is negative", (int)iters);
    Params P;
    if ((s = resolve_params(p, P)) != INIM_OK) return s;
    const RegLayout L = reg_layout(res, n, P.radius);
    if (L.total > kStaticScratchBytes)
        return fail(INIM_EWORKSPACE, "res=%d with n=%lld needs %zu bytes of scratch; the static scratch holds %zu",
                    (int)res, (long long)n, L.total, kStaticScratchBytes);
    char* ws = nullptr;
    if ((s = static_scratch(stream, &ws)) != INIM_OK) return s;
    int* st = status ? status : reinterpret_cast<int*>(ws + L.status);
    if (n == 0 || iters == 0) {
        hipError_t e = launch_fill(nullptr, 0, st, true, stream);
        return e == hipSuccess ? INIM_OK : hip_fail(e, "fill");
    }
    const double d0 = P.d0 < 0.0 ? (double)n / ((double)res * (double)res) : P.d0;
    const BlurTaps taps = make_taps(P.radius, P.sigma);
    return enqueue_regularize(xy, n, nullptr, 0, res, iters, d0, taps, L, ws, st, stream, nullptr, nullptr);
}

int inim_sync_status(void* ws, hipStream_t stream) {
    if (ws == nullptr) return fail(INIM_EWORKSPACE, "workspace is NULL");
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    int v = 0;
    e = hipMemcpy(&v, ws, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(status)");
    const int zero = 0;
    e = hipMemcpy(ws, &zero, sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(status clear)");
    return v == 0 ? INIM_OK : INIM_EDOMAIN;
}

}  // extern "C"
