// C-ABI entry points (include/ffa.h): validation, plan cache, workspace, and
// the launch sequence of a plan on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/ffa.h"
#include "field.h"
#include "plan.h"

using namespace ffa;

struct ffa_ctx {
    int device = 0;
    std::string arch;  // gcnArchName up to the first ':'
    // second stream for the pre-additions and the products that need them, and
    // the events that fork it from and join it back to the caller's stream
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;

    hipStream_t stream = nullptr;
    char* ws = nullptr;
    int64_t ws_bytes = 0;
    int32_t* d_err = nullptr;
    int last_err = 0;
    std::map<std::string, std::unique_ptr<Plan>> cache;
    std::map<std::string, ffa_opts> tuned;  // autotuner's choice per shape and per size class
    std::map<int, bool> coresident;         // per product configuration: fits beside the pre-additions
    // kernels of different streams may not run at the same time in this process (a
    // launch-blocking or kernel-serializing setting, a profiler collecting counters):
    // nothing then runs beside the product launch
    bool serialized = false;
    // phase timing: bit q set = phase q is recorded
    int prof = 0;
    struct Pending {
        hipEvent_t a, b;
        int phase;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    double total_ms[4] = {0, 0, 0, 0};
    int64_t calls[4] = {0, 0, 0, 0};
};

struct ffa_batch {
    ffa_ctx* ctx = nullptr;
    std::vector<Problem> prs;
    Plan plan;
    char* ws = nullptr;  // the plan's own workspace
    int64_t ws_bytes = 0;
    // captured launch sequence for one set of buffers (A, C; and A_im, C_im over F_p[i])
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec = nullptr;
    const void* gA = nullptr;
    void* gC = nullptr;
    const void* gA2 = nullptr;
    void* gC2 = nullptr;
};

namespace {

// Runs the body of an entry point.  A C++ exception thrown inside (a host
// allocation that fails, a length error) becomes a status code here instead
// of crossing the C interface: FFA_ENOMEM for an allocation failure,
// FFA_EINVAL for anything else.
template <typename F>
auto guarded(F&& f) noexcept -> decltype(f())
{
    try {
        return f();
    } catch (const std::bad_alloc&) {
        return FFA_ENOMEM;
    } catch (...) {
        return FFA_EINVAL;
    }
}

ffa_opts default_opts()
{
    ffa_opts o;
    std::memset(&o, 0, sizeof(o));
    o.levels = -1;
    return o;
}

std::string key_of(const Problem& p)
{
    char buf[256];
    snprintf(buf, sizeof(buf), "%lld|%lld|%lld|%lld|%u|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d|%u|%u|%d",
             (long long)p.n, (long long)p.k, (long long)p.lda, (long long)p.ldc, p.p, p.herm, p.dA,
             p.dC, p.opts.algo, p.opts.levels, p.opts.cutoff, p.opts.carrier, p.opts.check_inputs,
             p.opts.kernel, p.opts.operands, p.opts.streams * 16 + p.opts.herk_base * 4 + p.opts.general,
             p.opts.wino_min, p.aligned ? 1 : 0, p.trans, p.alpha, p.beta, p.opts.persist);
    return buf;
}

// keys of the autotuner's records: the exact shape, and its size class (n and k
// by half-octave)
std::string tune_key(int64_t n, int64_t k, uint32_t p, int herm, int dA, int dC)
{
    char buf[128];
    snprintf(buf, sizeof(buf), "%lld|%lld|%u|%d|%d|%d", (long long)n, (long long)k, p, herm, dA, dC);
    return buf;
}

// 2 floor(log2 x) + (x >= 1.5 * 2^floor(log2 x)); -1 for x <= 0
int half_octave(int64_t x)
{
    if (x <= 0) return -1;
    int e = 0;
    while ((x >> (e + 1)) > 0) ++e;
    const int64_t base = (int64_t)1 << e;
    return 2 * e + (x >= base + base / 2 ? 1 : 0);
}

std::string tune_class_key(int64_t n, int64_t k, uint32_t p, int herm, int dA, int dC)
{
    char buf[128];
    snprintf(buf, sizeof(buf), "c%d|%d|%u|%d|%d|%d", half_octave(n), half_octave(k), p, herm, dA, dC);
    return buf;
}

bool tuned_opts(const ffa_ctx* c, int64_t n, int64_t k, uint32_t p, int herm, int dA, int dC,
                ffa_opts* o)
{
    auto it = c->tuned.find(tune_key(n, k, p, herm, dA, dC));
    if (it == c->tuned.end()) it = c->tuned.find(tune_class_key(n, k, p, herm, dA, dC));
    if (it == c->tuned.end()) return false;
    *o = it->second;
    return true;
}

int dev_fail(ffa_ctx* c, int e)
{
    c->last_err = e;
    return FFA_EDEVICE;
}

hipEvent_t take_event(ffa_ctx* c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// Records the start event of a phase (no-op when that phase is not profiled).
hipEvent_t phase_begin(ffa_ctx* c, hipStream_t s, int phase)
{
    if (!((c->prof >> phase) & 1)) return nullptr;
    hipEvent_t e = take_event(c);
    if (e) (void)hipEventRecord(e, s);
    return e;
}

void phase_end(ffa_ctx* c, hipStream_t s, hipEvent_t start, int phase)
{
    if (!start) return;
    hipEvent_t e = take_event(c);
    if (!e) return;
    (void)hipEventRecord(e, s);
    c->pending.push_back({start, e, phase});
}

void resolve_events(ffa_ctx* c)
{
    for (auto& pe : c->pending) {
        float ms = 0.f;
        if (hipEventSynchronize(pe.b) == hipSuccess && hipEventElapsedTime(&ms, pe.a, pe.b) == hipSuccess) {
            c->total_ms[pe.phase] += ms;
            c->calls[pe.phase] += 1;
        }
        c->pool.push_back(pe.a);
        c->pool.push_back(pe.b);
    }
    c->pending.clear();
}

int ensure_workspace(ffa_ctx* c, int64_t bytes)
{
    if (bytes <= c->ws_bytes) return FFA_OK;
    if (c->ws) {
        hipError_t e = hipFree(c->ws);
        c->ws = nullptr;
        c->ws_bytes = 0;
        if (e != hipSuccess) return dev_fail(c, e);
    }
    const int64_t want = bytes + (bytes >> 3);
    hipError_t e = hipMalloc((void**)&c->ws, (size_t)want);
    if (e != hipSuccess) {
        c->ws = nullptr;
        (void)hipGetLastError();
        return FFA_ENOMEM;
    }
    c->ws_bytes = want;
    return FFA_OK;
}

// The plan's task tables packed on the host (once; the host copy is kept).
const std::vector<char>& host_tables(Plan& pl)
{
    if (pl.h_blob.empty()) pl.h_blob = pack_tables(pl);
    return pl.h_blob;
}

int upload_tables(ffa_ctx* c, Plan& pl)
{
    if (pl.d_blob) return FFA_OK;
    const std::vector<char>& blob = host_tables(pl);
    if (blob.empty()) return FFA_OK;
    hipError_t e = hipMalloc(&pl.d_blob, blob.size());
    if (e != hipSuccess) {
        pl.d_blob = nullptr;
        (void)hipGetLastError();
        return FFA_ENOMEM;
    }
    e = hipMemcpy(pl.d_blob, blob.data(), blob.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return dev_fail(c, e);
    return FFA_OK;
}

void free_tables(Plan& pl)
{
    if (pl.d_blob) (void)hipFree(pl.d_blob);
    pl.d_blob = nullptr;
}

// Settings under which kernels of different streams do not run concurrently, so
// that a product tile waiting for a kernel on another stream would wait in vain.
bool env_serializes()
{
    auto set = [](const char* name) {
        const char* v = getenv(name);
        return v && *v && strcmp(v, "0") != 0 && strcmp(v, "false") != 0;
    };
    if (set("AMD_SERIALIZE_KERNEL") || set("HIP_LAUNCH_BLOCKING") || set("CUDA_LAUNCH_BLOCKING")) return true;
    // rocprofv3 collecting counters or thread traces serializes the dispatches
    if (set("ROCPROF_COUNTER_COLLECTION") || set("ROCPROF_COUNTERS") || set("ROCPROF_ADVANCED_THREAD_TRACE"))
        return true;
    const char* q = getenv("GPU_MAX_HW_QUEUES");
    return q && atoi(q) == 1;
}

// Whether the signalling pre-addition kernel fits a CU beside a workgroup of the
// plan's product kernel (gfx950: 512 VGPRs per SIMD lane, 160 KiB of LDS per CU),
// so that it runs while the product launch holds every CU.  Measured once per
// product configuration and context.
bool coresident(ffa_ctx* c, const Plan& pl)
{
    if (pl.carrier != CAR_I8 || c->serialized) return false;
    auto it = c->coresident.find(pl.gemm_cfg);
    if (it != c->coresident.end()) return it->second;
    bool ok = false;
    int gv = 0, gt = 0, glds = 0, pv = 0, pt = 0;
    if (c->arch == "gfx950" && gemm_i8_config_regs(pl.gemm_cfg, &gv, &gt, &glds) == 0 &&
        preadd_signal_regs(&pv, &pt) == 0 && gv > 0 && pv > 0 && gv <= 256 && pv <= 256) {
        auto waves_per_simd = [](int threads) { return (threads / 64 + 3) / 4; };
        auto granule = [](int v) { return (v + 7) / 8 * 8; };
        const int regs = waves_per_simd(gt) * granule(gv) + waves_per_simd(pt) * granule(pv);
        ok = regs <= 512 && glds <= 160 * 1024 && waves_per_simd(gt) + waves_per_simd(pt) <= 8;
    }
    (void)hipGetLastError();
    c->coresident[pl.gemm_cfg] = ok;
    return ok;
}

// The launch sequence: conditioning, pre-additions (top-down), all products in
// one grouped launch, post-additions (bottom-up).
// The workspace (at least pl.ws_bytes) and the uploaded tables are the caller's
// to provide.  With pl.fork the pre-additions and the second product group run
// on the context's second stream, forked from the caller's stream after the
// conditioning and joined back before the post-additions; the first product
// group (products that read only A) runs on the caller's stream meanwhile.
int run_plan(ffa_ctx* c, const Plan& pl, Bases b, char* ws, const char* blob)
{
    b.p[BUF_WS] = ws;
    b.p[BUF_ERR] = (char*)c->d_err;
    hipStream_t ms = c->stream;
    void* s = (void*)ms;
    int e;
    if (!pl.cond.empty()) {
        if (pl.check_inputs && (e = launch_zero_flag(c->d_err, s))) return dev_fail(c, e);
        hipEvent_t ev = phase_begin(c, ms, 0);
        const CondTask* ct = (const CondTask*)(blob + pl.off_cond);
        e = pl.cond_trans ? launch_condition_trans(ct, (int)pl.cond.size(), pl.cond_max_blocks,
                                                   pl.cond[0].dt_in, b, pl.fp, pl.carrier, c->d_err, s)
                          : launch_condition(ct, (int)pl.cond.size(), pl.cond_max_blocks,
                                             pl.cond[0].dt_in, b, pl.fp, pl.carrier, c->d_err, s);
        if (e) return dev_fail(c, e);
        phase_end(c, ms, ev, 0);
        if (pl.check_inputs) {
            int32_t h_err = 0;
            hipError_t he = hipMemcpyAsync(&h_err, c->d_err, sizeof(int32_t),
                                           hipMemcpyDeviceToHost, ms);
            if (he == hipSuccess) he = hipStreamSynchronize(ms);
            if (he != hipSuccess) return dev_fail(c, he);
            if (h_err) return FFA_ERANGE;
        }
    }
    // pre-additions beside the product launch: the counter the waiting tiles read is
    // zeroed first; the pre-addition kernel runs on the second stream when both kernels
    // fit a CU together, else before the products on this stream (the waits then pass)
    const bool beside = pl.overlap_pre && coresident(c, pl);
    const bool fork = (pl.fork && !pl.sched2.empty()) || beside;
    hipStream_t ps = fork ? c->aux : ms;  // stream of the pre-additions
    if (pl.overlap_pre && (e = launch_zero_words(b, pl.wait_off, 2, s))) return dev_fail(c, e);
    if (fork) {
        hipError_t he = hipEventRecord(c->ev_fork, ms);
        if (he == hipSuccess) he = hipStreamWaitEvent(ps, c->ev_fork, 0);
        if (he != hipSuccess) return dev_fail(c, he);
    }
    const GemmTask* g = (const GemmTask*)(blob + pl.off_gemm);
    auto products = [&](hipStream_t st, int64_t off, size_t nsched) -> int {
        if (nsched == 0) return 0;
        const TileEnt* sc = (const TileEnt*)(blob + off);
        return pl.carrier == CAR_F64
                   ? launch_gemm_f64(g, sc, (int)nsched, b, pl.fp, (void*)st)
                   : launch_gemm_i8(pl.gemm_cfg, pl.gemm_src, g, sc, (int)nsched, b, pl.fp, (void*)st);
    };
    hipEvent_t ev = pl.levels > 0 ? phase_begin(c, ps, 1) : nullptr;
    for (int l = 0; l < pl.levels; ++l) {
        if (pl.pre[l].empty()) continue;
        if (pl.overlap_pre) {
            e = launch_preadd_signal((const PreaddTask*)(blob + pl.off_pre[l]), (int)pl.pre[l].size(),
                                     pl.pre_max_h[l], pl.pre_max_w[l], b, pl.fp, pl.pre_blocks, pl.wait_off,
                                     (void*)ps);
        } else {
            e = launch_preadd((const PreaddTask*)(blob + pl.off_pre[l]), (int)pl.pre[l].size(),
                              pl.pre_max_h[l], pl.pre_max_w[l], b, pl.fp, pl.carrier, (void*)ps);
        }
        if (e) return dev_fail(c, e);
    }
    if (!pl.wpre.empty()) {
        // Strassen-Winograd operand sums (after every pre-addition, before the products)
        e = launch_wino_pre((const WinoPreTask*)(blob + pl.off_wpre), (int)pl.wpre.size(), pl.wpre_max_h,
                            pl.wpre_max_w, b, pl.fp, pl.carrier, (void*)ps);
        if (e) return dev_fail(c, e);
    }
    phase_end(c, ps, ev, 1);
    if (beside) {
        hipError_t he = hipEventRecord(c->ev_join, ps);
        if (he != hipSuccess) return dev_fail(c, he);
    } else if (fork) {
        hipEvent_t pev = phase_begin(c, ps, 2);
        if ((e = products(ps, pl.off_sched2, pl.sched2.size()))) return dev_fail(c, e);
        phase_end(c, ps, pev, 2);
        hipError_t he = hipEventRecord(c->ev_join, ps);
        if (he != hipSuccess) return dev_fail(c, he);
    }
    // one event pair around the grouped product launch and its last-round sums
    hipEvent_t pev = pl.sched.empty() ? nullptr : phase_begin(c, ms, 2);
    if (pl.persist && !pl.sched.empty()) {
        // persistent: the queue counters start at zero (a fill kernel: graph-capturable)
        if ((e = launch_zero_words(b, pl.queue_off, 8, s))) return dev_fail(c, e);
        FieldParams fq = pl.fp;
        fq.nent = (int32_t)pl.sched.size();
        fq.queue_off = pl.queue_off;
        e = launch_gemm_i8(pl.gemm_cfg, pl.gemm_src, g, (const TileEnt*)(blob + pl.off_sched), (int)pl.sched.size(),
                           b, fq, (void*)ms);
    } else {
        e = products(ms, pl.off_sched, pl.sched.size());
    }
    if (e) return dev_fail(c, e);
    if (!pl.tail.empty()) {
        // the K-pieces of the launch's split last-round tiles, added into their places;
        // one launch per output format (the planner groups the tasks by it)
        for (size_t i0 = 0; i0 < pl.tail.size();) {
            size_t i1 = i0 + 1;
            while (i1 < pl.tail.size() && pl.tail[i1].out.dt == pl.tail[i0].out.dt) ++i1;
            e = launch_tail_sum((const TailTask*)(blob + pl.off_tail) + i0, (int)(i1 - i0), pl.tile,
                                pl.tail[i0].out.dt, b, pl.fp, s);
            if (e) return dev_fail(c, e);
            i0 = i1;
        }
    }
    phase_end(c, ms, pev, 2);
    if (!pl.gemm_r.empty()) {
        // the real products of the 2M base case, then their combination into the leaves
        hipEvent_t pev = phase_begin(c, ms, 2);
        e = launch_gemm_i8(pl.gemm_cfg_r, SRC_CARRIER, (const GemmTask*)(blob + pl.off_gemm_r),
                           (const TileEnt*)(blob + pl.off_sched_r), (int)pl.sched_r.size(), b, pl.fp, s);
        if (e) return dev_fail(c, e);
        phase_end(c, ms, pev, 2);
        // one launch per output format (the planner groups the tasks by it)
        for (size_t i0 = 0; i0 < pl.h2m.size();) {
            size_t i1 = i0 + 1;
            while (i1 < pl.h2m.size() && pl.h2m[i1].out.dt == pl.h2m[i0].out.dt) ++i1;
            e = launch_herk2m((const Herk2mTask*)(blob + pl.off_h2m) + i0, (int)(i1 - i0), pl.h2m_max_n,
                              pl.h2m[i0].g.dt, pl.h2m[i0].out.dt, b, pl.fp, s);
            if (e) return dev_fail(c, e);
            i0 = i1;
        }
    }
    if (fork) {
        hipError_t he = hipStreamWaitEvent(ms, c->ev_join, 0);
        if (he != hipSuccess) return dev_fail(c, he);
    }
    ev = pl.levels > 0 ? phase_begin(c, ms, 3) : nullptr;
    if (!pl.wpost.empty()) {
        // Strassen-Winograd combinations (before the post-additions that read P3, P4)
        e = launch_wino_post((const WinoPostTask*)(blob + pl.off_wpost), (int)pl.wpost.size(),
                             pl.wpost_max_h, b, pl.fp, s);
        if (e) return dev_fail(c, e);
    }
    for (int l = pl.levels - 1; l >= 0; --l) {
        if (pl.post[l].empty()) continue;
        // every task of a level writes the same format: the caller's C at level 0,
        // product residues below
        e = launch_postadd((const PostaddTask*)(blob + pl.off_post[l]), (int)pl.post[l].size(),
                           pl.post_max_h[l], pl.post[l][0].c.dt, b, pl.fp, s);
        if (e) return dev_fail(c, e);
    }
    if (!pl.upd.empty()) {
        // C <- alpha X + beta C (counted with the post-additions)
        if (!ev) ev = phase_begin(c, ms, 3);
        e = launch_update((const UpdateTask*)(blob + pl.off_upd), (int)pl.upd.size(), pl.upd_max_n,
                          pl.upd[0].x.dt, pl.upd[0].c.dt, b, pl.fp, s);
        if (e) return dev_fail(c, e);
    }
    phase_end(c, ms, ev, 3);
    return FFA_OK;
}

Plan* cached_plan(ffa_ctx* c, const Problem& pr)
{
    const std::string key = key_of(pr);
    auto it = c->cache.find(key);
    if (it != c->cache.end()) return it->second.get();
    std::unique_ptr<Plan> pl(new Plan(make_plan(pr)));
    Plan* raw = pl.get();
    c->cache.emplace(key, std::move(pl));
    return raw;
}

int run_call(ffa_ctx* c, const Problem& pr, const void* A, const void* A2, void* C, void* C2)
{
    if (!c) return FFA_EINVAL;
    if (pr.n > 0 && (!C || (pr.herm && !C2))) return FFA_EINVAL;
    if (pr.n > 0 && pr.k > 0 && (!A || (pr.herm && !A2))) return FFA_EINVAL;
    Plan* pl = cached_plan(c, pr);
    if (pl->status) return pl->status;
    if (pr.n == 0) return FFA_OK;
    hipError_t he = hipSetDevice(c->device);
    if (he != hipSuccess) return dev_fail(c, he);
    Bases b{};
    b.p[BUF_A] = (char*)A;
    b.p[BUF_A2] = (char*)A2;
    b.p[BUF_C] = (char*)C;
    b.p[BUF_C2] = (char*)C2;
    int st = ensure_workspace(c, pl->ws_bytes);
    if (!st) st = upload_tables(c, *pl);
    if (st) return st;
    return run_plan(c, *pl, b, c->ws, (const char*)pl->d_blob);
}

// The batch plan's own workspace, sized for its plan; drops a captured graph
// (which holds the old addresses).
void drop_graph(ffa_batch* b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
    b->gA = nullptr;
    b->gC = nullptr;
}

int batch_workspace(ffa_batch* b)
{
    if (b->plan.ws_bytes <= b->ws_bytes) return FFA_OK;
    drop_graph(b);
    if (b->ws) {
        (void)hipDeviceSynchronize();
        (void)hipFree(b->ws);
        b->ws = nullptr;
        b->ws_bytes = 0;
    }
    if (hipMalloc((void**)&b->ws, (size_t)b->plan.ws_bytes) != hipSuccess) {
        b->ws = nullptr;
        (void)hipGetLastError();
        return FFA_ENOMEM;
    }
    b->ws_bytes = b->plan.ws_bytes;
    return FFA_OK;
}

// Captures the plan's launch sequence for buffers bs on the batch's private
// stream and instantiates (or updates) the executable graph.
int capture_graph(ffa_batch* b, const Bases& bs)
{
    ffa_ctx* c = b->ctx;
    hipError_t he = hipSuccess;
    if (!b->cap) {
        he = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
        if (he != hipSuccess) {
            b->cap = nullptr;
            return dev_fail(c, he);
        }
    }
    he = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (he != hipSuccess) return dev_fail(c, he);
    hipStream_t user = c->stream;
    c->stream = b->cap;
    const int st = run_plan(c, b->plan, bs, b->ws, (const char*)b->plan.d_blob);
    c->stream = user;
    hipGraph_t g = nullptr;
    he = hipStreamEndCapture(b->cap, &g);
    if (st || he != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        drop_graph(b);
        return st ? st : dev_fail(c, he);
    }
    bool updated = false;
    if (b->gexec) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res;
        updated = hipGraphExecUpdate(b->gexec, g, &err_node, &res) == hipSuccess &&
                  res == hipGraphExecUpdateSuccess;
        if (!updated) {
            (void)hipGetLastError();
            drop_graph(b);
        }
    }
    if (!updated) {
        he = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
        if (he != hipSuccess) {
            b->gexec = nullptr;
            (void)hipGraphDestroy(g);
            return dev_fail(c, he);
        }
    }
    (void)hipGraphDestroy(g);
    b->gA = bs.p[BUF_A];
    b->gC = bs.p[BUF_C];
    b->gA2 = bs.p[BUF_A2];
    b->gC2 = bs.p[BUF_C2];
    return FFA_OK;
}

// Runs a batch plan on its packed buffers: directly, or by replaying the
// captured graph (captured again when a buffer changes).
int batch_exec(ffa_batch* b, const Bases& bs)
{
    ffa_ctx* c = b->ctx;
    hipError_t he = hipSetDevice(c->device);
    if (he != hipSuccess) return dev_fail(c, he);
    bool direct = b->prs[0].opts.launch == FFA_LAUNCH_DIRECT || c->prof || b->plan.check_inputs;
    if (!direct) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        he = hipStreamIsCapturing(c->stream, &cs);
        if (he != hipSuccess) return dev_fail(c, he);
        direct = cs != hipStreamCaptureStatusNone;  // the caller's capture records the kernels
    }
    if (direct) return run_plan(c, b->plan, bs, b->ws, (const char*)b->plan.d_blob);
    if (!b->gexec || b->gA != bs.p[BUF_A] || b->gC != bs.p[BUF_C] || b->gA2 != bs.p[BUF_A2] ||
        b->gC2 != bs.p[BUF_C2]) {
        const int st = capture_graph(b, bs);
        if (st) return st;
    }
    he = hipGraphLaunch(b->gexec, c->stream);
    return he == hipSuccess ? FFA_OK : dev_fail(c, he);
}

int batch_plan(ffa_ctx* ctx, int64_t count, const int64_t* n, const int64_t* k, uint32_t p, int herm,
               int dA, int dC, const ffa_opts* opts, ffa_batch** out);

}  // namespace

extern "C" {

int ffa_create(ffa_ctx** out, int device, void* hip_stream)
{
    return guarded([&]() -> int {
        if (!out) return FFA_EINVAL;
        *out = nullptr;
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
            (void)hipGetLastError();
            return FFA_EINVAL;
        }
        std::unique_ptr<ffa_ctx> owner(new ffa_ctx);
        ffa_ctx* c = owner.get();
        c->device = device;
        c->serialized = env_serializes();
        c->stream = (hipStream_t)hip_stream;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
            c->arch = prop.gcnArchName;
            const size_t colon = c->arch.find(':');
            if (colon != std::string::npos) c->arch.resize(colon);
        }
        hipError_t e = hipSetDevice(device);
        // the fixed scratch of ffa_syrk_modp_noalloc: its address on this device
        if (e == hipSuccess) e = (hipError_t)scratch_setup(device);
        if (e == hipSuccess) e = hipMalloc((void**)&c->d_err, 256);
        if (e == hipSuccess) e = hipMemset(c->d_err, 0, 256);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
        if (e != hipSuccess) {
            if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
            if (c->aux) (void)hipStreamDestroy(c->aux);
            if (c->d_err) (void)hipFree(c->d_err);
            return FFA_EDEVICE;
        }
        *out = owner.release();
        return FFA_OK;
    });
}

int ffa_destroy(ffa_ctx* c)
{
    return guarded([&]() -> int {
        if (!c) return FFA_EINVAL;
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
        resolve_events(c);
        for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
        for (auto& kv : c->cache) free_tables(*kv.second);
        if (c->ws) (void)hipFree(c->ws);
        if (c->d_err) (void)hipFree(c->d_err);
        if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
        if (c->ev_join) (void)hipEventDestroy(c->ev_join);
        if (c->aux) (void)hipStreamDestroy(c->aux);
        delete c;
        return FFA_OK;
    });
}

int ffa_set_stream(ffa_ctx* c, void* hip_stream)
{
    return guarded([&]() -> int {
        if (!c) return FFA_EINVAL;
        c->stream = (hipStream_t)hip_stream;
        return FFA_OK;
    });
}

int ffa_last_device_error(const ffa_ctx* c) { return c ? c->last_err : 0; }

int ffa_device_status(ffa_ctx* c)
{
    return guarded([&]() -> int {
        if (!c) return FFA_EINVAL;
        hipError_t he = hipSetDevice(c->device);
        if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
        if (he == hipSuccess) he = hipStreamSynchronize(c->aux);
        int32_t h = 0;
        if (he == hipSuccess) he = hipMemcpy(&h, c->d_err + 1, sizeof(int32_t), hipMemcpyDeviceToHost);
        if (he != hipSuccess) return dev_fail(c, he);
        if (!h) return FFA_OK;
        const int32_t zero = 0;
        he = hipMemcpy(c->d_err + 1, &zero, sizeof(int32_t), hipMemcpyHostToDevice);
        if (he != hipSuccess) return dev_fail(c, he);
        return FFA_EWAIT;
    });
}

int ffa_profile_enable(ffa_ctx* c, int on)
{
    return guarded([&]() -> int {
        if (!c) return FFA_EINVAL;
        c->prof = on & 15;
        return FFA_OK;
    });
}

int ffa_profile_read(ffa_ctx* c, int phase, double* total_ms, int64_t* calls)
{
    return guarded([&]() -> int {
        if (!c || phase < 0 || phase > 3) return FFA_EINVAL;
        resolve_events(c);
        if (total_ms) *total_ms = c->total_ms[phase];
        if (calls) *calls = c->calls[phase];
        return FFA_OK;
    });
}

int ffa_profile_reset(ffa_ctx* c)
{
    return guarded([&]() -> int {
        if (!c) return FFA_EINVAL;
        resolve_events(c);
        for (int i = 0; i < 4; ++i) {
            c->total_ms[i] = 0;
            c->calls[i] = 0;
        }
        return FFA_OK;
    });
}

const char* ffa_status_string(int s)
{
    switch (s) {
    case FFA_OK: return "ok";
    case FFA_EINVAL: return "invalid argument";
    case FFA_EPRIME: return "p is not an odd prime supported by the carrier";
    case FFA_ERANGE: return "input entry outside the residue range";
    case FFA_ENOMEM: return "device workspace allocation failed";
    case FFA_EDEVICE: return "HIP call failed";
    case FFA_EUNSUPPORTED: return "unsupported request";
    case FFA_EBOUND: return "exact accumulation bound exceeded";
    case FFA_ESCRATCH: return "the call needs more than the fixed scratch of the no-allocation entry point";
    case FFA_EWAIT: return "a bounded wait inside a kernel gave up; results since the last check are not valid";
    }
    return "unknown status";
}

int ffa_skew_unitary(uint32_t p, int hermitian, uint32_t* a, uint32_t* b, int* kind)
{
    return guarded([&]() -> int {
        if (!a || !b || !kind) return FFA_EINVAL;
        if (!is_odd_prime(p)) return FFA_EPRIME;
        if (hermitian && p % 4 != 3) return FFA_EUNSUPPORTED;
        uint64_t x, y;
        int k;
        if (skew_unitary_params(p, hermitian != 0, &k, &x, &y)) return FFA_EPRIME;
        *a = (uint32_t)x;
        *b = (uint32_t)y;
        *kind = k;
        return FFA_OK;
    });
}

int ffa_syrk_modp(ffa_ctx* ctx, int64_t n, int64_t k, uint32_t p, int dA, const void* A,
                  int64_t lda, int dC, void* C, int64_t ldc, const ffa_opts* opts)
{
    return guarded([&]() -> int {
        Problem pr;
        pr.n = n;
        pr.k = k;
        pr.lda = lda;
        pr.ldc = ldc;
        pr.p = p;
        pr.dA = dA;
        pr.dC = dC;
        pr.opts = opts ? *opts : default_opts();
        if (!opts && ctx) (void)tuned_opts(ctx, n, k, p, 0, dA, dC, &pr.opts);
        pr.aligned = ((uintptr_t)A % 16) == 0;
        return run_call(ctx, pr, A, nullptr, C, nullptr);
    });
}

int ffa_syrk_modp_noalloc(ffa_ctx* ctx, int64_t n, int64_t k, uint32_t p, int dA, const void* A,
                          int64_t lda, int dC, void* C, int64_t ldc, const ffa_opts* opts)
{
    return guarded([&]() -> int {
        Problem pr;
        pr.n = n;
        pr.k = k;
        pr.lda = lda;
        pr.ldc = ldc;
        pr.p = p;
        pr.dA = dA;
        pr.dC = dC;
        pr.opts = opts ? *opts : default_opts();
        if (!opts && ctx) (void)tuned_opts(ctx, n, k, p, 0, dA, dC, &pr.opts);
        pr.aligned = ((uintptr_t)A % 16) == 0;
        if (!ctx) return FFA_EINVAL;
        if (pr.n > 0 && !C) return FFA_EINVAL;
        if (pr.n > 0 && pr.k > 0 && !A) return FFA_EINVAL;
        Plan* pl = cached_plan(ctx, pr);
        if (pl->status) return pl->status;
        if (pr.n == 0) return FFA_OK;
        // tables first, then the workspace, in the fixed scratch
        const std::vector<char>& tables = host_tables(*pl);
        const int64_t tbytes = ((int64_t)tables.size() + 255) / 256 * 256;
        if (tbytes + pl->ws_bytes > FFA_SCRATCH_BYTES) return FFA_ESCRATCH;
        hipError_t he = hipSetDevice(ctx->device);
        if (he != hipSuccess) return dev_fail(ctx, he);
        char* base = scratch_base(ctx->device);
        if (!base) return FFA_EDEVICE;
        if (!tables.empty()) {
            he = hipMemcpyAsync(base, tables.data(), tables.size(), hipMemcpyHostToDevice, ctx->stream);
            if (he != hipSuccess) return dev_fail(ctx, he);
        }
        Bases b{};
        b.p[BUF_A] = (char*)A;
        b.p[BUF_C] = (char*)C;
        return run_plan(ctx, *pl, b, base + tbytes, base);
    });
}

int ffa_syrk_modp_ex(ffa_ctx* ctx, int trans, int64_t n, int64_t k, uint32_t p, uint32_t alpha, int dA,
                     const void* A, int64_t lda, uint32_t beta, int dC, void* C, int64_t ldc,
                     const ffa_opts* opts)
{
    return guarded([&]() -> int {
        Problem pr;
        pr.n = n;
        pr.k = k;
        pr.lda = lda;
        pr.ldc = ldc;
        pr.p = p;
        pr.dA = dA;
        pr.dC = dC;
        pr.trans = trans;
        pr.alpha = alpha;
        pr.beta = beta;
        pr.opts = opts ? *opts : default_opts();
        if (!opts && ctx) (void)tuned_opts(ctx, n, k, p, 0, dA, dC, &pr.opts);
        pr.aligned = ((uintptr_t)A % 16) == 0;
        return run_call(ctx, pr, A, nullptr, C, nullptr);
    });
}

int ffa_herk_modp2(ffa_ctx* ctx, int64_t n, int64_t k, uint32_t p, int dA, const void* A_re,
                   const void* A_im, int64_t lda, int dC, void* C_re, void* C_im, int64_t ldc,
                   const ffa_opts* opts)
{
    return guarded([&]() -> int {
        Problem pr;
        pr.n = n;
        pr.k = k;
        pr.lda = lda;
        pr.ldc = ldc;
        pr.p = p;
        pr.herm = 1;
        pr.dA = dA;
        pr.dC = dC;
        pr.opts = opts ? *opts : default_opts();
        if (!opts && ctx) (void)tuned_opts(ctx, n, k, p, 1, dA, dC, &pr.opts);
        pr.aligned = false;  // the conditioning always builds the complex planes
        return run_call(ctx, pr, A_re, A_im, C_re, C_im);
    });
}

int ffa_batch_syrk_plan(ffa_ctx* ctx, int64_t count, const int64_t* n, const int64_t* k,
                        uint32_t p, int dA, int dC, const ffa_opts* opts, ffa_batch** out)
{
    return guarded([&]() -> int {
        return batch_plan(ctx, count, n, k, p, 0, dA, dC, opts, out);
    });
}

int ffa_batch_herk_plan(ffa_ctx* ctx, int64_t count, const int64_t* n, const int64_t* k,
                        uint32_t p, int dA, int dC, const ffa_opts* opts, ffa_batch** out)
{
    return guarded([&]() -> int {
        return batch_plan(ctx, count, n, k, p, 1, dA, dC, opts, out);
    });
}

}  // extern "C"

namespace {

int batch_plan(ffa_ctx* ctx, int64_t count, const int64_t* n, const int64_t* k, uint32_t p, int herm,
               int dA, int dC, const ffa_opts* opts, ffa_batch** out)
{
    if (!ctx || !out || count <= 0 || count > FFA_BATCH_MAX || !n || !k) return FFA_EINVAL;
    *out = nullptr;
    std::vector<Problem> prs(count);
    const ffa_opts o = opts ? *opts : default_opts();
    if (o.launch != FFA_LAUNCH_GRAPH && o.launch != FFA_LAUNCH_DIRECT) return FFA_EINVAL;
    for (int64_t i = 0; i < count; ++i) {
        prs[i].n = n[i];
        prs[i].k = k[i];
        prs[i].p = p;
        prs[i].herm = herm;
        prs[i].dA = dA;
        prs[i].dC = dC;
        prs[i].opts = o;
    }
    std::unique_ptr<ffa_batch> owner(new ffa_batch);
    ffa_batch* b = owner.get();
    b->ctx = ctx;
    b->prs = std::move(prs);
    b->plan = make_batch_plan(b->prs);
    if (b->plan.status) return b->plan.status;
    (void)hipSetDevice(ctx->device);
    int st = FFA_OK;
    try {
        st = batch_workspace(b);
        if (!st) st = upload_tables(ctx, b->plan);
    } catch (...) {
        free_tables(b->plan);
        if (b->ws) (void)hipFree(b->ws);
        throw;
    }
    if (st) {
        free_tables(b->plan);
        if (b->ws) (void)hipFree(b->ws);
        return st;
    }
    *out = owner.release();
    return FFA_OK;
}

}  // namespace

extern "C" {

int ffa_batch_offsets(const ffa_batch* b, int64_t* a_off, int64_t* lda, int64_t* c_off,
                      int64_t* a_total, int64_t* c_total)
{
    return guarded([&]() -> int {
        if (!b) return FFA_EINVAL;
        const size_t cnt = b->plan.a_off.size();
        if (a_off) std::memcpy(a_off, b->plan.a_off.data(), cnt * sizeof(int64_t));
        if (lda) std::memcpy(lda, b->plan.a_ld.data(), cnt * sizeof(int64_t));
        if (c_off) std::memcpy(c_off, b->plan.c_off.data(), cnt * sizeof(int64_t));
        if (a_total) *a_total = b->plan.a_total;
        if (c_total) *c_total = b->plan.c_total;
        return FFA_OK;
    });
}

int ffa_batch_syrk_exec(ffa_batch* b, const void* A_packed, void* C_packed)
{
    return guarded([&]() -> int {
        if (!b || b->plan.cplx || !C_packed || (!A_packed && b->plan.a_total > 0)) return FFA_EINVAL;
        if (((uintptr_t)A_packed % 16) || ((uintptr_t)C_packed % 16)) return FFA_EINVAL;
        Bases bs{};
        bs.p[BUF_A] = (char*)A_packed;
        bs.p[BUF_C] = (char*)C_packed;
        return batch_exec(b, bs);
    });
}

int ffa_batch_herk_exec(ffa_batch* b, const void* A_re, const void* A_im, void* C_re, void* C_im)
{
    return guarded([&]() -> int {
        if (!b || !b->plan.cplx || !C_re || !C_im) return FFA_EINVAL;
        if (b->plan.a_total > 0 && (!A_re || !A_im)) return FFA_EINVAL;
        if (((uintptr_t)A_re | (uintptr_t)A_im | (uintptr_t)C_re | (uintptr_t)C_im) % 16) return FFA_EINVAL;
        Bases bs{};
        bs.p[BUF_A] = (char*)A_re;
        bs.p[BUF_A2] = (char*)A_im;
        bs.p[BUF_C] = (char*)C_re;
        bs.p[BUF_C2] = (char*)C_im;
        return batch_exec(b, bs);
    });
}

int ffa_batch_describe(const ffa_batch* b, char* buf, int64_t size)
{
    return guarded([&]() -> int {
        if (!b) return FFA_EINVAL;
        if (buf && size > 0) {
            const std::string d = describe(b->plan);
            const size_t m = std::min<size_t>(d.size(), (size_t)size - 1);
            std::memcpy(buf, d.data(), m);
            buf[m] = 0;
        }
        return FFA_OK;
    });
}

int ffa_batch_destroy(ffa_batch* b)
{
    return guarded([&]() -> int {
        if (!b) return FFA_EINVAL;
        (void)hipSetDevice(b->ctx->device);
        (void)hipDeviceSynchronize();
        drop_graph(b);
        if (b->cap) (void)hipStreamDestroy(b->cap);
        free_tables(b->plan);
        if (b->ws) (void)hipFree(b->ws);
        delete b;
        return FFA_OK;
    });
}

}  // extern "C"

namespace {

// Time of `reps` calls of f on the context's stream (HIP events), after one untimed call.
template <typename F>
int time_calls(ffa_ctx* c, int reps, F f, double* ms_out)
{
    int st = f();
    if (st) return st;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return dev_fail(c, hipGetLastError());
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return dev_fail(c, hipGetLastError());
    }
    (void)hipEventRecord(e0, c->stream);
    for (int r = 0; r < reps && st == FFA_OK; ++r) st = f();
    (void)hipEventRecord(e1, c->stream);
    float ms = 0.f;
    hipError_t he = hipEventSynchronize(e1);
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    if (he != hipSuccess) return dev_fail(c, he);
    *ms_out = ms / reps;
    return FFA_OK;
}

// INT8 product-kernel configurations that fit a plan's carrier ({0} for fp64).
std::vector<int> kernel_candidates(const Plan& pl)
{
    std::vector<int> out;
    if (pl.carrier != CAR_I8) return {0};
    for (int cfg = 0; cfg < 64; ++cfg)
        if (gemm_i8_config_valid(cfg, pl.nl, pl.cplx)) out.push_back(cfg + 1);
    return out;
}

// Carriers worth timing: INT8 limbs always; FP64 where the problem allows it
// (real field, p below its limit, bound held) and limbs are needed (p > 255).
std::vector<int> carrier_candidates(const Problem& base)
{
    std::vector<int> out{FFA_CARRIER_INT8};
    if (base.herm || base.p < 256) return out;
    Problem q = base;
    q.opts = default_opts();
    q.opts.carrier = FFA_CARRIER_F64;
    q.opts.levels = 0;
    q.opts.algo = FFA_ALGO_CLASSICAL;
    if (make_plan(q).status == FFA_OK) out.push_back(FFA_CARRIER_F64);
    return out;
}

void record_tuned(ffa_ctx* c, int64_t n, int64_t k, uint32_t p, int herm, int dA, int dC,
                  const ffa_opts& o)
{
    c->tuned[tune_key(n, k, p, herm, dA, dC)] = o;
    c->tuned[tune_class_key(n, k, p, herm, dA, dC)] = o;
}

}  // namespace

extern "C" {

int ffa_autotune_syrk(ffa_ctx* ctx, int64_t n, int64_t k, uint32_t p, int dA, const void* A,
                      int64_t lda, int dC, void* C, int64_t ldc, int reps, ffa_opts* best,
                      double* best_ms)
{
    return guarded([&]() -> int {
        if (!ctx || reps <= 0) return FFA_EINVAL;
        Problem base;
        base.n = n;
        base.k = k;
        base.lda = lda;
        base.ldc = ldc;
        base.p = p;
        base.dA = dA;
        base.dC = dC;
        base.opts = default_opts();
        base.aligned = ((uintptr_t)A % 16) == 0;
        Plan probe = make_plan(base);
        if (probe.status) return probe.status;
        double best_t = 1e30;
        ffa_opts best_o = default_opts();
        bool found = false;
        for (int car : carrier_candidates(base)) {
            Problem cb = base;
            cb.opts.carrier = car;
            const Plan cprobe = make_plan(cb);
            if (cprobe.status) continue;
            for (int L = 0; L <= 4; ++L) {
                if (L > 0 && ((n >> L) < 64 || k == 0)) break;
                for (int kc : kernel_candidates(cprobe))
                for (int opr : {FFA_OPERANDS_PLANES, FFA_OPERANDS_RAW}) {
                // general products: single tasks, or Winograd down to 0 / 2048 / 4096 rows
                // (each distinct plan timed once)
                std::vector<size_t> wino_seen;
                for (int wi = 0; wi < 4; ++wi) {
                    const int gen = wi == 0 ? FFA_GENERAL_CLASSICAL : FFA_GENERAL_WINOGRAD;
                    const int wmin = wi <= 1 ? 0 : (wi == 2 ? 2048 : 4096);
                    ffa_opts o = default_opts();
                    o.algo = L == 0 ? FFA_ALGO_CLASSICAL : FFA_ALGO_RECURSIVE;
                    o.levels = L;
                    o.kernel = kc;
                    o.carrier = car;
                    o.operands = opr;
                    o.general = gen;
                    o.wino_min = wmin;
                    Problem pr = base;
                    pr.opts = o;
                    // raw operands and Winograd only where the planner takes them
                    const Plan tp = make_plan(pr);
                    if (opr == FFA_OPERANDS_RAW && tp.gemm_src != SRC_RAW_U16) continue;
                    if (gen == FFA_GENERAL_WINOGRAD) {
                        if (tp.wpre.empty() || std::find(wino_seen.begin(), wino_seen.end(), tp.wpre.size()) !=
                                                   wino_seen.end())
                            continue;
                        wino_seen.push_back(tp.wpre.size());
                    }
                    double ms = 0;
                    const int st =
                        time_calls(ctx, reps, [&] { return run_call(ctx, pr, A, nullptr, C, nullptr); }, &ms);
                    if (st == FFA_EBOUND || st == FFA_EUNSUPPORTED || st == FFA_EINVAL) continue;
                    if (st) return st;
                    if (ms < best_t) {
                        best_t = ms;
                        best_o = o;
                        found = true;
                    }
                }
                }
            }
        }
        if (!found) return FFA_EUNSUPPORTED;
        record_tuned(ctx, n, k, p, 0, dA, dC, best_o);
        if (best) *best = best_o;
        if (best_ms) *best_ms = best_t;
        return FFA_OK;
    });
}

int ffa_batch_autotune(ffa_batch* b, const void* A_packed, void* C_packed, int reps, ffa_opts* best,
                       double* best_ms)
{
    return guarded([&]() -> int {
        if (!b || reps <= 0) return FFA_EINVAL;
        if (b->plan.cplx) return FFA_EUNSUPPORTED;
        ffa_ctx* c = b->ctx;
        const int64_t cutoffs[] = {0, 256, 384};
        double best_t = 1e30;
        ffa_opts best_o = b->prs[0].opts;
        bool found = false;
        for (int car : carrier_candidates(b->prs[0])) {
            std::vector<Problem> cprs = b->prs;
            for (auto& q : cprs) q.opts.carrier = car;
            const Plan cprobe = make_batch_plan(cprs);
            if (cprobe.status) continue;
            for (int kc : kernel_candidates(cprobe)) {
                for (int64_t cut : cutoffs)
                for (int opr : {FFA_OPERANDS_PLANES, FFA_OPERANDS_RAW})
                for (int per : {FFA_PERSIST_ON, FFA_PERSIST_OFF}) {
                    std::vector<Problem> prs = cprs;
                    for (auto& q : prs) {
                        q.opts.kernel = kc;
                        q.opts.cutoff = (int32_t)cut;
                        q.opts.levels = -1;
                        q.opts.algo = cut == 0 ? FFA_ALGO_CLASSICAL : FFA_ALGO_AUTO;
                        q.opts.operands = opr;
                        q.opts.persist = per;
                    }
                    ffa_batch trial;
                    trial.ctx = c;
                    trial.prs = prs;
                    trial.plan = make_batch_plan(prs);
                    if (trial.plan.status) continue;
                    if (opr == FFA_OPERANDS_RAW && trial.plan.gemm_src != SRC_RAW_U16) {
                        free_tables(trial.plan);
                        continue;
                    }
                    if (trial.plan.a_total != b->plan.a_total || trial.plan.c_total != b->plan.c_total) continue;
                    int st = batch_workspace(&trial);
                    if (!st) st = upload_tables(c, trial.plan);
                    double ms = 0;
                    if (!st)
                        st = time_calls(c, reps, [&] { return ffa_batch_syrk_exec(&trial, A_packed, C_packed); },
                                        &ms);
                    (void)hipDeviceSynchronize();
                    drop_graph(&trial);
                    if (trial.cap) (void)hipStreamDestroy(trial.cap);
                    trial.cap = nullptr;
                    const bool better = !st && ms < best_t;
                    if (better) {
                        // the trial's plan, tables and workspace move into the batch
                        best_t = ms;
                        best_o = prs[0].opts;
                        found = true;
                        drop_graph(b);
                        free_tables(b->plan);
                        if (b->ws) (void)hipFree(b->ws);
                        b->prs = prs;
                        b->plan = std::move(trial.plan);
                        b->ws = trial.ws;
                        b->ws_bytes = trial.ws_bytes;
                        trial.plan.d_blob = nullptr;
                        trial.ws = nullptr;
                    } else {
                        free_tables(trial.plan);
                        if (trial.ws) (void)hipFree(trial.ws);
                        trial.ws = nullptr;
                    }
                    if (st) return st;
                }
            }
        }
        if (!found) return FFA_EUNSUPPORTED;
        if (best) *best = best_o;
        if (best_ms) *best_ms = best_t;
        return FFA_OK;
    });
}

namespace {

// "key":<integer> inside one record object [p, e); false when missing
bool json_int(const char* p, const char* e, const char* key, long long* v)
{
    char pat[32];
    snprintf(pat, sizeof(pat), "\"%s\"", key);
    const size_t m = strlen(pat);
    for (const char* q = p; q + m <= e; ++q) {
        if (strncmp(q, pat, m)) continue;
        q += m;
        while (q < e && (*q == ' ' || *q == ':' || *q == '\t' || *q == '\n')) ++q;
        char* end = nullptr;
        *v = strtoll(q, &end, 10);
        return end != q && end <= e;
    }
    return false;
}

}  // namespace

int64_t ffa_tune_export(const ffa_ctx* c, char* buf, int64_t size)
{
    return guarded([&]() -> int64_t {
        if (!c) return FFA_EINVAL;
        std::string s = "{\"arch\":\"" + c->arch + "\",\"records\":[";
        bool first = true;
        for (const auto& kv : c->tuned) {
            if (kv.first.empty() || kv.first[0] == 'c') continue;  // size-class entries follow the exact ones
            long long n, k;
            unsigned p;
            int herm, dA, dC;
            if (sscanf(kv.first.c_str(), "%lld|%lld|%u|%d|%d|%d", &n, &k, &p, &herm, &dA, &dC) != 6) continue;
            const ffa_opts& o = kv.second;
            char rec[320];
            snprintf(rec, sizeof(rec),
                     "%s{\"n\":%lld,\"k\":%lld,\"p\":%u,\"herm\":%d,\"dA\":%d,\"dC\":%d,\"algo\":%d,"
                     "\"levels\":%d,\"cutoff\":%d,\"carrier\":%d,\"kernel\":%d,\"operands\":%d,"
                     "\"general\":%d,\"wino_min\":%d,\"persist\":%d}",
                     first ? "" : ",", n, k, p, herm, dA, dC, o.algo, o.levels, o.cutoff, o.carrier, o.kernel,
                     o.operands, o.general, o.wino_min, o.persist);
            s += rec;
            first = false;
        }
        s += "]}";
        if (buf && size > (int64_t)s.size()) std::memcpy(buf, s.c_str(), s.size() + 1);
        return (int64_t)s.size();
    });
}

int ffa_tune_import(ffa_ctx* c, const char* json)
{
    return guarded([&]() -> int {
        if (!c || !json) return FFA_EINVAL;
        const char* arch = strstr(json, "\"arch\"");
        const char* recs = strstr(json, "\"records\"");
        if (!arch || !recs) return FFA_EINVAL;
        const char* q1 = strchr(arch + 6, '"');
        const char* q2 = q1 ? strchr(q1 + 1, '"') : nullptr;
        if (!q2) return FFA_EINVAL;
        if (std::string(q1 + 1, q2) != c->arch) return 0;
        const char* p = strchr(recs, '[');
        if (!p) return FFA_EINVAL;
        int taken = 0;
        while ((p = strchr(p, '{')) != nullptr) {
            const char* e = strchr(p, '}');
            if (!e) return FFA_EINVAL;
            long long n, k, pp, herm, dA, dC, algo, levels, cutoff, carrier, kernel;
            if (!json_int(p, e, "n", &n) || !json_int(p, e, "k", &k) || !json_int(p, e, "p", &pp) ||
                !json_int(p, e, "herm", &herm) || !json_int(p, e, "dA", &dA) || !json_int(p, e, "dC", &dC) ||
                !json_int(p, e, "algo", &algo) || !json_int(p, e, "levels", &levels) ||
                !json_int(p, e, "cutoff", &cutoff) || !json_int(p, e, "carrier", &carrier) ||
                !json_int(p, e, "kernel", &kernel))
                return FFA_EINVAL;
            ffa_opts o = default_opts();
            o.algo = (int32_t)algo;
            o.levels = (int32_t)levels;
            o.cutoff = (int32_t)cutoff;
            o.carrier = (int32_t)carrier;
            o.kernel = (int32_t)kernel;
            long long v;  // fields added later: absent means the built-in choice
            if (json_int(p, e, "operands", &v)) o.operands = (int32_t)v;
            if (json_int(p, e, "general", &v)) o.general = (int32_t)v;
            if (json_int(p, e, "wino_min", &v)) o.wino_min = (int32_t)v;
            if (json_int(p, e, "persist", &v)) o.persist = (int32_t)v;
            record_tuned(c, n, k, (uint32_t)pp, (int)herm, (int)dA, (int)dC, o);
            ++taken;
            p = e + 1;
        }
        return taken;
    });
}

int ffa_plan_describe(int64_t n, int64_t k, uint32_t p, int hermitian, int dA, int dC,
                      int64_t lda, int64_t ldc, const ffa_opts* opts, char* buf, int64_t size)
{
    return guarded([&]() -> int {
        Problem pr;
        pr.n = n;
        pr.k = k;
        pr.lda = lda;
        pr.ldc = ldc;
        pr.p = p;
        pr.herm = hermitian ? 1 : 0;
        pr.dA = dA;
        pr.dC = dC;
        pr.opts = opts ? *opts : default_opts();
        pr.aligned = !hermitian;
        Plan pl = make_plan(pr);
        if (buf && size > 0) {
            const std::string s = describe(pl);
            const size_t m = std::min<size_t>(s.size(), (size_t)size - 1);
            std::memcpy(buf, s.data(), m);
            buf[m] = 0;
        }
        return pl.status;
    });
}

}  // extern "C"
