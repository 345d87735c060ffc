// C-ABI entry points (include/ffa.h): validation, plan cache, workspace, and
// the launch sequence of a plan on the context's stream.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/ffa.h"
#include "field.h"
#include "plan.h"

using namespace ffa;

struct ffa_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    int64_t ws_bytes = 0;
    int32_t* d_err = nullptr;
    int last_err = 0;
    std::map<std::string, std::unique_ptr<Plan>> cache;
    // phase timing
    bool prof = false;
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
    Plan plan;
};

namespace {

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
    snprintf(buf, sizeof(buf), "%lld|%lld|%lld|%lld|%u|%d|%d|%d|%d|%d|%d|%d|%d|%d", (long long)p.n,
             (long long)p.k, (long long)p.lda, (long long)p.ldc, p.p, p.herm, p.dA, p.dC,
             p.opts.algo, p.opts.levels, p.opts.cutoff, p.opts.carrier, p.opts.check_inputs,
             p.aligned ? 1 : 0);
    return buf;
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

// Records the start event of a phase (no-op when profiling is off).
hipEvent_t phase_begin(ffa_ctx* c)
{
    if (!c->prof) return nullptr;
    hipEvent_t e = take_event(c);
    if (e) (void)hipEventRecord(e, c->stream);
    return e;
}

void phase_end(ffa_ctx* c, hipEvent_t start, int phase)
{
    if (!c->prof || !start) return;
    hipEvent_t e = take_event(c);
    if (!e) return;
    (void)hipEventRecord(e, c->stream);
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

int upload_tables(ffa_ctx* c, Plan& pl)
{
    if (pl.d_blob) return FFA_OK;
    std::vector<char> blob = pack_tables(pl);
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

// The launch sequence: conditioning, pre-additions (top-down), all products in
// one grouped launch, post-additions (bottom-up).
int run_plan(ffa_ctx* c, Plan& pl, Bases b)
{
    int st = ensure_workspace(c, pl.ws_bytes);
    if (st) return st;
    st = upload_tables(c, pl);
    if (st) return st;
    b.p[BUF_WS] = c->ws;
    char* blob = (char*)pl.d_blob;
    void* s = (void*)c->stream;
    int e;
    if (!pl.cond.empty()) {
        if (pl.check_inputs && (e = launch_zero_flag(c->d_err, s))) return dev_fail(c, e);
        hipEvent_t ev = phase_begin(c);
        e = launch_condition((const CondTask*)(blob + pl.off_cond), (int)pl.cond.size(),
                             pl.cond_max_blocks, pl.cond[0].dt_in, b, pl.fp, pl.carrier, c->d_err, s);
        if (e) return dev_fail(c, e);
        phase_end(c, ev, 0);
        if (pl.check_inputs) {
            int32_t h_err = 0;
            hipError_t he = hipMemcpyAsync(&h_err, c->d_err, sizeof(int32_t),
                                           hipMemcpyDeviceToHost, c->stream);
            if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
            if (he != hipSuccess) return dev_fail(c, he);
            if (h_err) return FFA_ERANGE;
        }
    }
    hipEvent_t ev = pl.levels > 0 ? phase_begin(c) : nullptr;
    for (int l = 0; l < pl.levels; ++l) {
        if (pl.pre[l].empty()) continue;
        e = launch_preadd((const PreaddTask*)(blob + pl.off_pre[l]), (int)pl.pre[l].size(),
                          pl.pre_max_h[l], pl.pre_max_w[l], b, pl.fp, pl.carrier, s);
        if (e) return dev_fail(c, e);
    }
    phase_end(c, ev, 1);
    if (!pl.gemm.empty()) {
        ev = phase_begin(c);
        const GemmTask* g = (const GemmTask*)(blob + pl.off_gemm);
        const TileEnt* sc = (const TileEnt*)(blob + pl.off_sched);
        const int nb = (int)pl.sched.size();
        e = pl.carrier == CAR_F64 ? launch_gemm_f64(g, sc, nb, b, pl.fp, s)
                                  : launch_gemm_i8(pl.gemm_cfg, g, sc, nb, b, pl.fp, s);
        if (e) return dev_fail(c, e);
        phase_end(c, ev, 2);
    }
    ev = pl.levels > 0 ? phase_begin(c) : nullptr;
    for (int l = pl.levels - 1; l >= 0; --l) {
        if (pl.post[l].empty()) continue;
        // every task of a level writes the same format: the caller's C at level 0,
        // product residues below
        e = launch_postadd((const PostaddTask*)(blob + pl.off_post[l]), (int)pl.post[l].size(),
                           pl.post_max_h[l], pl.post[l][0].c.dt, b, pl.fp, s);
        if (e) return dev_fail(c, e);
    }
    phase_end(c, ev, 3);
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
    return run_plan(c, *pl, b);
}

}  // namespace

extern "C" {

int ffa_create(ffa_ctx** out, int device, void* hip_stream)
{
    if (!out) return FFA_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return FFA_EINVAL;
    }
    ffa_ctx* c = new ffa_ctx;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipMalloc((void**)&c->d_err, 256);
    if (e != hipSuccess) {
        delete c;
        return FFA_EDEVICE;
    }
    *out = c;
    return FFA_OK;
}

int ffa_destroy(ffa_ctx* c)
{
    if (!c) return FFA_EINVAL;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    resolve_events(c);
    for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
    for (auto& kv : c->cache) free_tables(*kv.second);
    if (c->ws) (void)hipFree(c->ws);
    if (c->d_err) (void)hipFree(c->d_err);
    delete c;
    return FFA_OK;
}

int ffa_set_stream(ffa_ctx* c, void* hip_stream)
{
    if (!c) return FFA_EINVAL;
    c->stream = (hipStream_t)hip_stream;
    return FFA_OK;
}

int ffa_last_device_error(const ffa_ctx* c) { return c ? c->last_err : 0; }

int ffa_profile_enable(ffa_ctx* c, int on)
{
    if (!c) return FFA_EINVAL;
    c->prof = on != 0;
    return FFA_OK;
}

int ffa_profile_read(ffa_ctx* c, int phase, double* total_ms, int64_t* calls)
{
    if (!c || phase < 0 || phase > 3) return FFA_EINVAL;
    resolve_events(c);
    if (total_ms) *total_ms = c->total_ms[phase];
    if (calls) *calls = c->calls[phase];
    return FFA_OK;
}

int ffa_profile_reset(ffa_ctx* c)
{
    if (!c) return FFA_EINVAL;
    resolve_events(c);
    for (int i = 0; i < 4; ++i) {
        c->total_ms[i] = 0;
        c->calls[i] = 0;
    }
    return FFA_OK;
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
    }
    return "unknown status";
}

int ffa_skew_unitary(uint32_t p, int hermitian, uint32_t* a, uint32_t* b, int* kind)
{
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
}

int ffa_syrk_modp(ffa_ctx* ctx, int64_t n, int64_t k, uint32_t p, int dA, const void* A,
                  int64_t lda, int dC, void* C, int64_t ldc, const ffa_opts* opts)
{
    Problem pr;
    pr.n = n;
    pr.k = k;
    pr.lda = lda;
    pr.ldc = ldc;
    pr.p = p;
    pr.dA = dA;
    pr.dC = dC;
    pr.opts = opts ? *opts : default_opts();
    pr.aligned = ((uintptr_t)A % 16) == 0;
    return run_call(ctx, pr, A, nullptr, C, nullptr);
}

int ffa_herk_modp2(ffa_ctx* ctx, int64_t n, int64_t k, uint32_t p, int dA, const void* A_re,
                   const void* A_im, int64_t lda, int dC, void* C_re, void* C_im, int64_t ldc,
                   const ffa_opts* opts)
{
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
    pr.aligned = false;  // the conditioning always builds the complex planes
    return run_call(ctx, pr, A_re, A_im, C_re, C_im);
}

int ffa_batch_syrk_plan(ffa_ctx* ctx, int64_t count, const int64_t* n, const int64_t* k,
                        uint32_t p, int dA, int dC, const ffa_opts* opts, ffa_batch** out)
{
    if (!ctx || !out || count <= 0 || !n || !k) return FFA_EINVAL;
    *out = nullptr;
    std::vector<Problem> prs(count);
    const ffa_opts o = opts ? *opts : default_opts();
    for (int64_t i = 0; i < count; ++i) {
        prs[i].n = n[i];
        prs[i].k = k[i];
        prs[i].p = p;
        prs[i].dA = dA;
        prs[i].dC = dC;
        prs[i].opts = o;
    }
    ffa_batch* b = new ffa_batch;
    b->ctx = ctx;
    b->plan = make_batch_plan(prs);
    if (b->plan.status) {
        const int st = b->plan.status;
        delete b;
        return st;
    }
    (void)hipSetDevice(ctx->device);
    int st = ensure_workspace(ctx, b->plan.ws_bytes);
    if (!st) st = upload_tables(ctx, b->plan);
    if (st) {
        free_tables(b->plan);
        delete b;
        return st;
    }
    *out = b;
    return FFA_OK;
}

int ffa_batch_offsets(const ffa_batch* b, int64_t* a_off, int64_t* c_off, int64_t* a_total,
                      int64_t* c_total)
{
    if (!b) return FFA_EINVAL;
    const size_t cnt = b->plan.a_off.size();
    if (a_off) std::memcpy(a_off, b->plan.a_off.data(), cnt * sizeof(int64_t));
    if (c_off) std::memcpy(c_off, b->plan.c_off.data(), cnt * sizeof(int64_t));
    if (a_total) *a_total = b->plan.a_total;
    if (c_total) *c_total = b->plan.c_total;
    return FFA_OK;
}

int ffa_batch_syrk_exec(ffa_batch* b, const void* A_packed, void* C_packed)
{
    if (!b || !C_packed || (!A_packed && b->plan.a_total > 0)) return FFA_EINVAL;
    if (((uintptr_t)A_packed % 16) || ((uintptr_t)C_packed % 16)) return FFA_EINVAL;
    ffa_ctx* c = b->ctx;
    hipError_t he = hipSetDevice(c->device);
    if (he != hipSuccess) return dev_fail(c, he);
    Bases bs{};
    bs.p[BUF_A] = (char*)A_packed;
    bs.p[BUF_C] = (char*)C_packed;
    return run_plan(c, b->plan, bs);
}

int ffa_batch_destroy(ffa_batch* b)
{
    if (!b) return FFA_EINVAL;
    (void)hipSetDevice(b->ctx->device);
    (void)hipDeviceSynchronize();
    free_tables(b->plan);
    delete b;
    return FFA_OK;
}

int ffa_plan_describe(int64_t n, int64_t k, uint32_t p, int hermitian, int dA, int dC,
                      int64_t lda, int64_t ldc, const ffa_opts* opts, char* buf, int64_t size)
{
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
}

}  // extern "C"
