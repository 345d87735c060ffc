// Host planner for Algorithm 1 (Section 3) on one GPU.
//
// The paper runs the recursion depth-first and in place, with C's unused upper
// triangle as scratch (schedule table of Section 7).  On the GPU the recursion
// tree is flattened instead: every node of level i gets its own S1..S4 and
// P1..P5 in a workspace, the pre-additions of all 3^i nodes of a level form
// one launch, all products of all levels form ONE grouped launch, and the
// post-additions run level by level bottom-up.  This order respects every edge
// of the task DAG of Section 7 (S before the products that read them, all five
// products before U1..U5).
//
// Odd sizes are zero-padded (Section 3 allows padding; Section 4.3 pads the
// inner dimension so that the block-structured Y has even order): rows to a
// multiple of 2^levels, columns to a multiple of ktile * 2^levels, which keeps
// every level's blocks even, every Y of even order and every product's K a
// multiple of the kernels' k-tile.  Zero rows give zero rows and columns of
// C, which are not written back; zero columns do not change A A^T.
#include "plan.h"

#include <algorithm>
#include <cstdio>

#include "field.h"

namespace ffa {

static int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

static bool dtype_in_ok(int dt) { return dt >= FFA_I64 && dt <= FFA_I8_CENTRED; }
static bool dtype_out_ok(int dt) { return dt >= FFA_I64 && dt <= FFA_F64; }

// Largest p a format can hold as canonical residues.
static uint64_t dtype_pmax(int dt)
{
    switch (dt) {
    case FFA_U8: return 256;
    case FFA_I8_CENTRED: return 255;
    case FFA_U16: return 65536;
    case FFA_I32: return (1ull << 31);
    case FFA_F64: return (1ull << 52);
    default: return (1ull << 62);
    }
}

namespace {

struct Builder {
    Plan& pl;
    int esize = 1;     // carrier element size in bytes
    int npo = 1;       // planes per carrier matrix: re, or re, im, -re
    int npo_leaf = 1;  // planes of carriers that feed base cases (re + im added for 2M)
    int rdt = 0;       // residue storage of products
    int rsize = 1;
    int bt = 0;        // product tile edge
    int bt_r = 0;      // tile edge of the real launch of the 2M base case
    int64_t ws = 0;

    int64_t alloc(int64_t bytes)
    {
        const int64_t o = ws;
        ws += round_up(std::max<int64_t>(bytes, 1), 256);
        return o;
    }
    CarRef new_car(int64_t rows, int64_t cols, int planes = 0)
    {
        CarRef c;
        c.buf = BUF_WS;
        c.ld = (int32_t)cols;
        c.ps = round_up(rows * cols * esize, 256);
        c.off = alloc(c.ps * (planes ? planes : npo) * pl.nl);
        return c;
    }
    // one plane of residues (the real products of the 2M base case)
    ResRef new_res_real(int64_t h)
    {
        ResRef r;
        r.buf = r.buf2 = BUF_WS;
        r.ld = (int32_t)round_up(h, 64);
        r.dt = rdt;
        r.off = r.off2 = alloc(h * r.ld * rsize);
        return r;
    }
    ResRef new_res(int64_t h)
    {
        ResRef r;
        r.buf = r.buf2 = BUF_WS;
        r.ld = (int32_t)round_up(h, 64);
        r.dt = rdt;
        const int64_t bytes = h * r.ld * rsize;
        r.off = alloc(bytes);
        r.off2 = pl.cplx ? alloc(bytes) : r.off;
        return r;
    }
    CarRef view(const CarRef& a, int64_t row, int64_t col) const
    {
        CarRef v = a;
        v.off += (row * a.ld + col) * esize;
        return v;
    }
    void add_gemm(const CarRef& x, const CarRef& z, const ResRef& c, int64_t M, int64_t N,
                  int64_t K, bool syrk, bool aonly, int64_t kvalid = -1)
    {
        GemmTask g{};
        g.x = x;
        g.z = z;
        g.c = c;
        g.M = (int32_t)M;
        g.N = (int32_t)N;
        g.K = (int32_t)K;
        g.syrk = syrk ? 1 : 0;
        g.kvalid = (int32_t)(kvalid >= 0 ? kvalid : K);
        g.tiles_m = (int32_t)((M + bt - 1) / bt);
        g.tiles_n = (int32_t)((N + bt - 1) / bt);
        // the INT8 kernel addresses an operand panel with 32-bit offsets: the
        // sub-planes it may touch plus one tile of rows must stay below 2 GiB
        if (pl.carrier == CAR_I8) {
            const int64_t nsub = (pl.cplx ? 3 : 1) * pl.nl;
            const int64_t ea = (nsub - 1) * x.ps + (int64_t)bt * x.ld * esize + K;
            const int64_t eb = (nsub - 1) * z.ps + (int64_t)bt * z.ld * esize + K;
            if (ea >= (1ll << 31) || eb >= (1ll << 31)) pl.status = FFA_EUNSUPPORTED;
        }
        pl.gemm.push_back(g);
        pl.gemm_aonly.push_back(aonly ? 1 : 0);
        pl.max_k = std::max(pl.max_k, K);
        // real multiply-accumulates (a complex task is four real products)
        pl.products_macs += (syrk ? M * (M + 1) / 2 * K : M * N * K) * (pl.cplx ? 4 : 1);
    }
    // A real product of the 2M base case: sub-planes x.off + l * x.ps (limbs).
    void add_gemm_real(const CarRef& x, const CarRef& z, const ResRef& c, int64_t M, int64_t N,
                       int64_t K, bool syrk)
    {
        GemmTask g{};
        g.x = x;
        g.z = z;
        g.c = c;
        g.M = (int32_t)M;
        g.N = (int32_t)N;
        g.K = (int32_t)K;
        g.syrk = syrk ? 1 : 0;
        g.kvalid = (int32_t)K;
        g.tiles_m = (int32_t)((M + bt_r - 1) / bt_r);
        g.tiles_n = (int32_t)((N + bt_r - 1) / bt_r);
        const int64_t ea = (pl.nl - 1) * x.ps + (int64_t)bt_r * x.ld + K;
        const int64_t eb = (pl.nl - 1) * z.ps + (int64_t)bt_r * z.ld + K;
        if (ea >= (1ll << 31) || eb >= (1ll << 31)) pl.status = FFA_EUNSUPPORTED;
        pl.gemm_r.push_back(g);
        pl.max_k = std::max(pl.max_k, K);
        pl.products_macs += syrk ? M * (M + 1) / 2 * K : M * N * K;
    }
    // A general product c = x z^T (h x h from h x w operands): one task, or one
    // level of Strassen-Winograd (operand sums, seven half-size products, combination).
    void general(const CarRef& x, const CarRef& z, const ResRef& c, int64_t h, int64_t w)
    {
        if (!pl.wino || h < pl.wino_min) {
            add_gemm(x, z, c, h, h, w, false, false);
            return;
        }
        const int64_t h2 = h / 2, w2 = w / 2;
        WinoPreTask wt{};
        wt.x = x;
        wt.z = z;
        for (int j = 0; j < 4; ++j) {
            wt.s[j] = new_car(h2, w2);
            wt.t[j] = new_car(h2, w2);
        }
        wt.h = (int32_t)h2;
        wt.w = (int32_t)w2;
        pl.wpre.push_back(wt);
        WinoPostTask wp{};
        for (int j = 0; j < 7; ++j) wp.r[j] = new_res(h2);
        wp.c = c;
        wp.h = (int32_t)h2;
        pl.wpost.push_back(wp);
        const CarRef X11 = view(x, 0, 0), X12 = view(x, 0, w2), X22 = view(x, h2, w2);
        const CarRef Z11 = view(z, 0, 0), Z12 = view(z, 0, w2), Z22 = view(z, h2, w2);
        add_gemm(X11, Z11, wp.r[0], h2, h2, w2, false, false);        // R1 = X11 Z11^T
        add_gemm(X12, Z12, wp.r[1], h2, h2, w2, false, false);        // R2 = X12 Z12^T
        add_gemm(wt.s[3], Z22, wp.r[2], h2, h2, w2, false, false);    // R3 = S4 Z22^T
        add_gemm(X22, wt.t[3], wp.r[3], h2, h2, w2, false, false);    // R4 = X22 T4^T
        add_gemm(wt.s[0], wt.t[0], wp.r[4], h2, h2, w2, false, false);  // R5 = S1 T1^T
        add_gemm(wt.s[1], wt.t[1], wp.r[5], h2, h2, w2, false, false);  // R6 = S2 T2^T
        add_gemm(wt.s[2], wt.t[2], wp.r[6], h2, h2, w2, false, false);  // R7 = S3 T3^T
    }
    // One node of the recursion: a is rows x cols, its result goes to c.
    // aonly: a is a block of the (conditioned) input itself.
    void node(int level, const CarRef& a, int64_t rows, int64_t cols, const ResRef& c,
              int64_t nvalid, bool aonly)
    {
        if (level == pl.levels) {
            if (pl.herk2m) {
                // Algorithm 3 with epsilon = 1: G = (Xr + Xi)(Xr + Xi)^T, H = Xr Xi^T
                CarRef re = a, im = a, sum = a;
                im.off += pl.nl * a.ps;
                sum.off += 3 * pl.nl * a.ps;
                const ResRef G = new_res_real(rows), H = new_res_real(rows);
                add_gemm_real(sum, sum, G, rows, rows, cols, true);
                // A long H = Xr Xi^T goes in two halves over K: twice the tiles at half
                // the length, which fill the last round of the launch (the SYRK's
                // tiles and H's whole ones leave it nearly empty)
                const int64_t kt_r = gemm_i8_config_ktile(pl.gemm_cfg_r);
                const bool split = cols >= 2048 && (cols / 2) % kt_r == 0;
                Herk2mTask t{};
                if (split) {
                    const ResRef H2 = new_res_real(rows);
                    add_gemm_real(re, im, H, rows, rows, cols / 2, false);
                    add_gemm_real(view(re, 0, cols / 2), view(im, 0, cols / 2), H2, rows, rows, cols / 2, false);
                    t.h2 = H2;
                    t.split = 1;
                } else {
                    add_gemm_real(re, im, H, rows, rows, cols, false);
                }
                t.g = G;
                t.h = H;
                t.out = c;
                t.n = (int32_t)rows;
                t.nvalid = (int32_t)nvalid;
                pl.h2m.push_back(t);
                pl.h2m_max_n = std::max<int>(pl.h2m_max_n, (int)rows);
                return;
            }
            // a base case that writes the caller's C covers its valid rows only (the
            // padding rows are zero and must not be stored)
            const int64_t m = (c.buf == BUF_C || c.buf == BUF_C2) ? std::min(rows, nvalid) : rows;
            add_gemm(a, a, c, m, m, cols, true, aonly);
            return;
        }
        const int64_t h = rows / 2, w = cols / 2;
        PreaddTask pt{};
        pt.a = a;
        // S3 feeds the base case P5 (and, below, further leaves)
        for (int j = 0; j < 4; ++j) pt.s[j] = new_car(h, w, j == 2 ? npo_leaf : npo);
        pt.h = (int32_t)h;
        pt.w = (int32_t)w;
        pl.pre[level].push_back(pt);
        ResRef P[5];
        for (int j = 0; j < 5; ++j) P[j] = new_res(h);
        const CarRef A11 = view(a, 0, 0), A12 = view(a, 0, w), A22 = view(a, h, w);
        general(A22, pt.s[3], P[2], h, w);     // P3 = A22 phi(S4)
        general(pt.s[0], pt.s[1], P[3], h, w);  // P4 = S1 phi(S2)
        node(level + 1, A11, h, w, P[0], h, aonly);               // P1 = A11 phi(A11)
        node(level + 1, A12, h, w, P[1], h, aonly);               // P2 = A12 phi(A12)
        node(level + 1, pt.s[2], h, w, P[4], h, false);           // P5 = S3 phi(S3)
        PostaddTask qt{};
        for (int j = 0; j < 5; ++j) qt.p[j] = P[j];
        qt.c = c;
        qt.upd = level == 0 && pl.fold_update ? 1 : 0;
        qt.h = (int32_t)h;
        qt.nvalid = (int32_t)nvalid;
        pl.post[level].push_back(qt);
    }
};

struct Common {
    int status = FFA_OK;
    int carrier = CAR_I8, nl = 1;
    FieldParams fp{};
};

// Checks shared by single and batched calls; picks the carrier and Y.
Common common_setup(uint32_t p, int herm, int dA, int dC, const ffa_opts& o)
{
    Common cm;
    if (!dtype_in_ok(dA) || !dtype_out_ok(dC)) { cm.status = FFA_EINVAL; return cm; }
    if (o.algo < FFA_ALGO_AUTO || o.algo > FFA_ALGO_RECURSIVE) { cm.status = FFA_EINVAL; return cm; }
    if (o.carrier < FFA_CARRIER_AUTO || o.carrier > FFA_CARRIER_F64) { cm.status = FFA_EINVAL; return cm; }
    if (o.operands < FFA_OPERANDS_AUTO || o.operands > FFA_OPERANDS_RAW) { cm.status = FFA_EINVAL; return cm; }
    if (o.streams < FFA_STREAMS_AUTO || o.streams > FFA_STREAMS_TWO) { cm.status = FFA_EINVAL; return cm; }
    if (!is_odd_prime(p)) { cm.status = FFA_EPRIME; return cm; }
    if ((uint64_t)p > dtype_pmax(dA) || (uint64_t)p > dtype_pmax(dC)) { cm.status = FFA_EINVAL; return cm; }
    if (herm && p % 4 != 3) { cm.status = FFA_EUNSUPPORTED; return cm; }
    int car = o.carrier;
    if (car == FFA_CARRIER_AUTO) car = (dA == FFA_F64 && !herm) ? FFA_CARRIER_F64 : FFA_CARRIER_INT8;
    if (car == FFA_CARRIER_F64) {
        if (herm) { cm.status = FFA_EUNSUPPORTED; return cm; }
        if (p >= (1u << 26)) { cm.status = FFA_EPRIME; return cm; }
        cm.carrier = CAR_F64;
        cm.nl = 1;
    } else {
        if (p >= 65536) { cm.status = FFA_EPRIME; return cm; }
        cm.carrier = CAR_I8;
        cm.nl = p < 256 ? 1 : 2;
    }
    if (dA == FFA_I8_CENTRED && !(cm.carrier == CAR_I8 && cm.nl == 1)) {
        cm.status = FFA_EINVAL;
        return cm;
    }
    int kind;
    uint64_t a, b;
    if (skew_unitary_params(p, herm != 0, &kind, &a, &b)) { cm.status = FFA_EPRIME; return cm; }
    FieldParams& fp = cm.fp;
    fp.p = (int32_t)p;
    fp.half = (int32_t)((p - 1) / 2);
    fp.rep_max = 32639;
    fp.ykind = kind;
    fp.ya = (int32_t)a;
    fp.yb = (int32_t)b;
    fp.nl = cm.nl;
    fp.cplx = herm ? 1 : 0;
    fp.inv_p = 1.0 / (double)p;
    fp.r20 = (int32_t)(((1 << 20) + p / 2) / p);
    fp.npo = herm ? 3 : 1;
    return cm;
}

// Built-in recursion cutoffs (measured on MI355X: one level wins from n = 32768 for one
// INT8 limb and at n = 16384 for two, four levels at n = 8192 for fp64; F_p[i] with the
// 2M base case: no recursion).
int default_cutoff(int carrier, int nl, int cplx, bool herk2m)
{
    if (carrier == CAR_F64) return 512;
    // F_p[i]: with the 2M base case (1.5 n^2 k real products) one level of Algorithm 1,
    // whose P3, P4 are complex products of four real ones, costs 1.04x more products
    if (cplx) return herk2m ? (1 << 30) : 2048;
    // one limb: the classical product is as fast at n = 16384 (1.72-1.75 ms against 1.76-1.83 ms
    // per call with one level) and slower at n = 32768 (14.40 ms against 13.19 ms for one
    // level, 13.22 ms for two); two limbs: one level wins at 16384 (6.81 against 7.69 ms)
    return nl == 1 ? 16384 : 8192;
}

int choose_levels(int64_t n, int64_t k, const ffa_opts& o, int carrier, int nl, int cplx, bool herk2m)
{
    if (n < 2 || k == 0) return 0;
    if (o.algo == FFA_ALGO_CLASSICAL) return 0;
    int L;
    if (o.levels >= 0) {
        L = o.levels;
    } else {
        const int64_t cut = o.cutoff > 0 ? o.cutoff : default_cutoff(carrier, nl, cplx, herk2m);
        L = 0;
        for (int64_t m = n; m > cut && L < 10; m = (m + 1) / 2) ++L;
        if (o.algo == FFA_ALGO_RECURSIVE && L == 0) L = 1;
    }
    while (L > 0 && (n >> L) < 1) --L;
    return L;
}

// Exact-accumulation bound of the carrier; FFA_OK or FFA_EBOUND.
int check_bound(const Plan& pl)
{
    const double terms = (double)pl.max_k * (pl.cplx ? 2.0 : 1.0);
    if (pl.carrier == CAR_F64) {
        const double m = (double)pl.max_abs;
        return terms * m * m < 9007199254740992.0 ? FFA_OK : FFA_EBOUND;
    }
    if (pl.nl == 1) {
        const double m = (double)pl.max_abs;
        // the int32 epilogue reduction needs a little headroom below 2^31
        return terms * m * m < 2147483648.0 - 131072.0 ? FFA_OK : FFA_EBOUND;
    }
    // two limbs: the middle accumulator sums hi*lo + lo*hi, each at most 128^2
    return 2.0 * terms * 16384.0 < 2147483648.0 ? FFA_OK : FFA_EBOUND;
}

// Tile schedule of the grouped product launch.  Tiles of each task are cut
// into blocks of GR x GC tiles (rows x columns; only the lower triangle for
// base cases) so that the workgroups running together on one XCD share few
// operand panels in that XCD's L2.  Blocks are dealt, costliest first, to the
// XCD with the least work so far (workgroup b runs on XCD b mod 8), and the
// schedule interleaves the eight per-XCD lists; shorter lists are padded with
// idle entries.
constexpr int64_t MAX_SCHEDULE_TILES = 1ll << 27;

int build_schedule(const std::vector<GemmTask>& tasks, bool cplx, size_t first, size_t last,
                   std::vector<TileEnt>& sched, const std::vector<char>* phase = nullptr)
{
    constexpr int GR = 4, GC = 8, NX = 8;
    struct Group {
        double cost;
        int phase;  // groups of phase 0 come before those of phase 1 in every XCD's list
        std::vector<TileEnt> tiles;
    };
    std::vector<Group> groups;
    // a schedule this long would not fit host memory sensibly (and needs no GPU)
    int64_t want = 0;
    for (size_t t = first; t < last; ++t) want += (int64_t)tasks[t].tiles_m * tasks[t].tiles_n;
    if (want > MAX_SCHEDULE_TILES) return -1;
    int tiles = 0;
    for (size_t t = first; t < last; ++t) {
        const GemmTask& g = tasks[t];
        const double kcost = (double)g.K * (cplx ? 2 : 1) + 64.0;
        for (int bi = 0; bi < g.tiles_m; bi += GR) {
            const int bj_end = g.syrk ? std::min(bi + GR, g.tiles_n) : g.tiles_n;
            for (int bj = 0; bj < bj_end; bj += GC) {
                Group gr;
                gr.phase = phase ? (*phase)[t] : 0;
                for (int ti = bi; ti < std::min(bi + GR, g.tiles_m); ++ti)
                    for (int tj = bj; tj < std::min(bj + GC, g.tiles_n); ++tj)
                        if (!g.syrk || tj <= ti) gr.tiles.push_back({(int32_t)t, ti | (tj << 16)});
                if (gr.tiles.empty()) continue;
                gr.cost = kcost * (double)gr.tiles.size();
                tiles += (int)gr.tiles.size();
                groups.push_back(std::move(gr));
            }
        }
    }
    std::stable_sort(groups.begin(), groups.end(), [](const Group& a, const Group& b) {
        return a.phase != b.phase ? a.phase < b.phase : a.cost > b.cost;
    });
    std::vector<std::vector<TileEnt>> bins(NX);
    double load[NX] = {0};
    for (const Group& gr : groups) {
        int x = 0;
        for (int i = 1; i < NX; ++i)
            if (load[i] < load[x]) x = i;
        load[x] += gr.cost;
        bins[x].insert(bins[x].end(), gr.tiles.begin(), gr.tiles.end());
    }
    size_t len = 0;
    for (const auto& b : bins) len = std::max(len, b.size());
    sched.assign(len * NX, TileEnt{-1, 0});
    for (int x = 0; x < NX; ++x)
        for (size_t i = 0; i < bins[x].size(); ++i) sched[i * NX + x] = bins[x][i];
    return tiles;
}

// The last partial round of the launch: on each XCD (32 CUs, entries x, x + 8, ...
// of the schedule) the tiles past its last full round of 32.  When they fill at
// most a quarter (a half) of the XCD, each is replaced by four (two) single-tile
// tasks over a quarter (a half) of K each, writing residue tiles in the
// workspace, and a TailTask adds them into the tile's place mod p before
// anything reads it.  The launch then ends a quarter (half) round after its last
// full round instead of a whole round.  Tiles on the diagonal of a base case
// (written in part) are not split.  A round is 32 tiles per XCD only when one
// workgroup fills a CU; configurations whose LDS lets two or more share a CU are
// not split (their rounds are not known on the host).
void split_tail(Plan& pl)
{
    constexpr int NX = 8, CPX = 32;
    if (pl.carrier != CAR_I8 || pl.cplx || pl.gemm_src != SRC_CARRIER || pl.sched.empty()) return;
    if (2 * gemm_i8_config_lds(pl.gemm_cfg) <= 160 * 1024) return;
    const int bt = pl.tile;
    const size_t len = pl.sched.size() / NX;
    std::vector<std::vector<TileEnt>> bins(NX);
    for (size_t i = 0; i < len; ++i)
        for (int x = 0; x < NX; ++x)
            if (pl.sched[i * NX + x].x >= 0) bins[x].push_back(pl.sched[i * NX + x]);
    int NQ = 4;
    auto splittable = [&](const TileEnt& e) {
        const GemmTask& g = pl.gemm[e.x];
        const int ti = e.y & 0xffff, tj = e.y >> 16;
        return !(g.syrk && ti == tj) && g.K % (NQ * pl.ktile) == 0 && g.kvalid == g.K;
    };
    int64_t ws = round_up(pl.ws_bytes, 256);
    std::vector<TailTask> tail;
    for (auto& v : bins) {
        const int nt = (int)(v.size() % CPX);
        if (nt == 0 || nt * 2 > CPX) continue;
        // quarters when they fit the round and divide K, else halves
        std::vector<char> taken;
        int got = 0;
        for (NQ = nt * 4 <= CPX ? 4 : 2; NQ >= 2; NQ /= 2) {
            taken.assign(v.size(), 0);
            got = 0;
            for (size_t i = v.size(); i-- > 0 && got < nt;)
                if (splittable(v[i])) taken[i] = 1, ++got;
            if (got == nt) break;
        }
        if (got < nt) continue;
        std::vector<TileEnt> keep, pieces;
        for (size_t i = 0; i < v.size(); ++i) {
            if (!taken[i]) {
                keep.push_back(v[i]);
                continue;
            }
            const GemmTask g0 = pl.gemm[v[i].x];
            const int r0 = (v[i].y & 0xffff) * bt, c0 = (v[i].y >> 16) * bt;
            const int64_t es = dtype_size(g0.c.dt);
            TailTask tt{};
            tt.part = g0.c;
            tt.part.buf = tt.part.buf2 = BUF_WS;
            tt.part.off = tt.part.off2 = ws;
            tt.part.ld = bt;
            tt.out = g0.c;
            tt.out.off += ((int64_t)r0 * g0.c.ld + c0) * es;
            tt.pstride = (int64_t)bt * bt * es;
            tt.rows = std::min(bt, g0.M - r0);
            tt.cols = std::min(bt, g0.N - c0);
            tt.nparts = NQ;
            const int kq = g0.K / NQ;
            for (int q = 0; q < NQ; ++q) {
                GemmTask g = g0;
                g.x.off += (int64_t)r0 * g0.x.ld + (int64_t)q * kq;
                g.z.off += (int64_t)c0 * g0.z.ld + (int64_t)q * kq;
                g.M = tt.rows;
                g.N = tt.cols;
                g.K = g.kvalid = kq;
                g.syrk = 0;
                g.tiles_m = g.tiles_n = 1;
                g.c = tt.part;
                g.c.off = g.c.off2 = ws + q * tt.pstride;
                pieces.push_back({(int32_t)pl.gemm.size(), 0});
                pl.gemm.push_back(g);
            }
            ws += round_up(NQ * tt.pstride, 256);
            tail.push_back(tt);
        }
        keep.insert(keep.end(), pieces.begin(), pieces.end());
        v = std::move(keep);
    }
    if (tail.empty()) return;
    size_t nlen = 0;
    for (const auto& v : bins) nlen = std::max(nlen, v.size());
    pl.sched.assign(nlen * NX, TileEnt{-1, 0});
    for (int x = 0; x < NX; ++x)
        for (size_t i = 0; i < bins[x].size(); ++i) pl.sched[i * NX + x] = bins[x][i];
    pl.gemm_aonly.resize(pl.gemm.size(), 0);
    for (const auto& t : tail) pl.total_tiles += t.nparts - 1;
    std::stable_sort(tail.begin(), tail.end(), [](const TailTask& a, const TailTask& b) { return a.out.dt < b.out.dt; });
    pl.tail = std::move(tail);
    pl.ws_bytes = ws;
}

// Orders the products as [reads only A | reads pre-addition outputs] and builds
// one schedule per group when they run on two streams (the second group exists
// only with recursion), else one schedule for all.
void schedule_products(Plan& pl)
{
    if (!pl.fork) {
        pl.gemm_split = (int)pl.gemm.size();
        // with the pre-additions beside the launch, the tiles that wait for them come
        // after every tile that reads only A, on every XCD
        std::vector<char> phase;
        if (pl.overlap_pre)
            for (char a : pl.gemm_aonly) phase.push_back(a ? 0 : 1);
        const int t1 = build_schedule(pl.gemm, pl.cplx, 0, pl.gemm.size(), pl.sched,
                                      pl.overlap_pre ? &phase : nullptr);
        const int t2 = t1 < 0 ? 0 : build_schedule(pl.gemm_r, false, 0, pl.gemm_r.size(), pl.sched_r);
        if (t1 < 0 || t2 < 0) {
            pl.status = FFA_EINVAL;
            return;
        }
        pl.total_tiles = t1;
        if (pl.split_tail) split_tail(pl);
        pl.total_tiles += t2;
        pl.sched2.clear();
        return;
    }
    std::vector<GemmTask> g1, g2;
    for (size_t t = 0; t < pl.gemm.size(); ++t) (pl.gemm_aonly[t] ? g1 : g2).push_back(pl.gemm[t]);
    pl.gemm_split = (int)g1.size();
    pl.gemm = g1;
    pl.gemm.insert(pl.gemm.end(), g2.begin(), g2.end());
    pl.gemm_aonly.assign(pl.gemm_split, 1);
    pl.gemm_aonly.resize(pl.gemm.size(), 0);
    const int t1 = build_schedule(pl.gemm, pl.cplx, 0, pl.gemm_split, pl.sched);
    const int t2 = t1 < 0 ? 0 : build_schedule(pl.gemm, pl.cplx, pl.gemm_split, pl.gemm.size(), pl.sched2);
    if (t1 < 0 || t2 < 0) {
        pl.status = FFA_EINVAL;
        return;
    }
    pl.total_tiles = t1 + t2;
}

// Host check of every workspace reference of the product and addition tasks:
// the bytes a kernel may touch (the planes it reads or writes, rows below the
// task's row count, K columns) lie inside the workspace.  A failure is a
// planner error, reported before anything is launched.
bool extents_ok(const Plan& pl)
{
    const int64_t ws = pl.ws_bytes;
    const int64_t es = pl.carrier == CAR_F64 ? (pl.fp.st32 ? 4 : 8) : 1;
    auto car_ok = [&](const CarRef& r, int64_t rows, int64_t cols, int64_t subplanes) {
        if (r.buf != BUF_WS || rows <= 0 || cols <= 0) return true;
        const int64_t last = r.off + (subplanes - 1) * r.ps + ((rows - 1) * r.ld + cols) * es;
        return r.off >= 0 && last <= ws;
    };
    auto res_ok = [&](const ResRef& r, int64_t rows, int64_t cols, bool both) {
        const int64_t rs = dtype_size(r.dt);
        auto one = [&](int32_t buf, int64_t off) {
            return buf != BUF_WS || rows <= 0 || cols <= 0 || (off >= 0 && off + ((rows - 1) * r.ld + cols) * rs <= ws);
        };
        return one(r.buf, r.off) && (!both || one(r.buf2, r.off2));
    };
    const int64_t nl = pl.carrier == CAR_F64 ? 1 : pl.nl;
    // complex products read planes re, im and -re; real products one plane
    const int64_t sub_main = (pl.cplx ? 3 : 1) * nl;
    for (const auto& g : pl.gemm) {
        if (pl.gemm_src == SRC_RAW_U16) continue;  // reads the caller's rows
        if (!car_ok(g.x, g.M, g.K, sub_main) || !car_ok(g.z, g.N, g.K, sub_main)) return false;
        if (!res_ok(g.c, g.M, g.N, pl.cplx != 0)) return false;
    }
    for (const auto& g : pl.gemm_r)
        if (!car_ok(g.x, g.M, g.K, nl) || !car_ok(g.z, g.N, g.K, nl) || !res_ok(g.c, g.M, g.N, false)) return false;
    for (const auto& lv : pl.pre)
        for (const auto& t : lv) {
            if (!car_ok(t.a, 2 * (int64_t)t.h, 2 * (int64_t)t.w, (pl.cplx ? 2 : 1) * nl)) return false;
            for (int j = 0; j < 4; ++j) {
                const int64_t planes = !pl.cplx ? 1 : (j == 2 ? pl.fp.npo : 3);
                if (!car_ok(t.s[j], t.h, t.w, planes * nl)) return false;
            }
        }
    for (const auto& t : pl.h2m)
        if (!res_ok(t.g, t.n, t.n, false) || !res_ok(t.h, t.n, t.n, false) || !res_ok(t.out, t.n, t.n, true) ||
            (t.split && !res_ok(t.h2, t.n, t.n, false)))
            return false;
    for (const auto& t : pl.tail) {
        if (!res_ok(t.out, t.rows, t.cols, false)) return false;
        ResRef last = t.part;
        last.off += (t.nparts - 1) * t.pstride;
        if (!res_ok(t.part, t.rows, t.cols, false) || !res_ok(last, t.rows, t.cols, false)) return false;
    }
    for (const auto& lv : pl.post)
        for (const auto& t : lv) {
            for (int j = 0; j < 5; ++j)
                if (!res_ok(t.p[j], t.h, t.h, pl.cplx != 0)) return false;
            if (!res_ok(t.c, 2 * (int64_t)t.h, 2 * (int64_t)t.h, pl.cplx != 0)) return false;
        }
    return true;
}

void size_grids(Plan& pl)
{
    pl.pre_max_h.assign(pl.levels, 0);
    pl.pre_max_w.assign(pl.levels, 0);
    pl.post_max_h.assign(pl.levels, 0);
    for (int l = 0; l < pl.levels; ++l) {
        for (const auto& t : pl.pre[l]) {
            pl.pre_max_h[l] = std::max(pl.pre_max_h[l], t.h);
            pl.pre_max_w[l] = std::max(pl.pre_max_w[l], t.w);
        }
        for (const auto& t : pl.post[l]) pl.post_max_h[l] = std::max(pl.post_max_h[l], t.h);
    }
    for (const auto& t : pl.wpre) {
        pl.wpre_max_h = std::max<int>(pl.wpre_max_h, t.h);
        pl.wpre_max_w = std::max<int>(pl.wpre_max_w, t.w);
    }
    for (const auto& t : pl.wpost) pl.wpost_max_h = std::max<int>(pl.wpost_max_h, t.h);
    // 2M combinations write leaves of recursions (workspace residues) and, in a
    // batch, whole problems (the caller's format): one launch per output format
    std::stable_sort(pl.h2m.begin(), pl.h2m.end(),
                     [](const Herk2mTask& a, const Herk2mTask& b) { return a.out.dt < b.out.dt; });
    schedule_products(pl);
    if (pl.status == FFA_OK && !extents_ok(pl)) pl.status = FFA_EINVAL;
}

// Where the product of a whole problem goes: the caller's C, or, when the call
// asks for C <- alpha Low(A A^T) + beta C, a workspace residue matrix that the
// final update pass combines with C.
ResRef root_output(Plan& pl, Builder& B, const Problem& pr)
{
    ResRef c;
    c.buf = BUF_C;
    c.buf2 = BUF_C2;
    c.off = c.off2 = pr.c_off * dtype_size(pr.dC);
    c.ld = (int32_t)pr.ldc;
    c.dt = pr.dC;
    if (pr.alpha == 1 && pr.beta == 0) return c;
    // with recursion the top-level post-additions apply the update as they store
    // (Section 7's schedule for alpha A A^T + beta C needs no pass of its own)
    if (pl.levels > 0) {
        pl.fold_update = true;
        return c;
    }
    const ResRef x = B.new_res(pr.n);
    UpdateTask u{};
    u.x = x;
    u.c = c;
    u.n = (int32_t)pr.n;
    pl.upd.push_back(u);
    pl.upd_max_n = std::max<int>(pl.upd_max_n, (int)pr.n);
    return x;
}

// Adds one problem's conditioning and recursion tree to the plan.
int add_problem(Plan& pl, Builder& B, const Problem& pr, int levels, bool allow_direct)
{
    const int ktile = pl.ktile;
    // one more halving for Strassen-Winograd below the deepest general products
    // (none without recursion: then the whole problem is one base case, whose rows
    // must stay those of the caller's C)
    const int depth = levels + (pl.wino && levels > 0 ? 1 : 0);
    const int64_t npad = round_up(pr.n, (int64_t)1 << depth);
    const int64_t kpad = round_up(pr.k, (int64_t)ktile << depth);
    if (npad >= (1ll << 31) || kpad >= (1ll << 31)) return FFA_EINVAL;
    if (pl.npad == 0) {
        pl.npad = npad;
        pl.kpad = kpad;
    }
    const int in_size = dtype_size(pr.dA);
    if (pl.gemm_src == SRC_RAW_U16) {
        // the product kernel reads the caller's uint16 rows and splits them into limbs
        CarRef a;
        a.buf = BUF_A;
        a.off = pr.a_off * in_size;
        a.ps = 0;
        a.ld = (int32_t)(pr.lda * in_size);
        pl.direct = true;
        pl.max_abs = std::max<int>(pl.max_abs, 32896);
        const ResRef c = root_output(pl, B, pr);
        B.add_gemm(a, a, c, pr.n, pr.n, kpad, true, true, pr.k);
        return FFA_OK;
    }
    const bool in_matches = (pl.carrier == CAR_I8 && pl.nl == 1 && !pl.cplx && pr.dA == FFA_I8_CENTRED) ||
                            (pl.carrier == CAR_F64 && pr.dA == FFA_F64 && !pl.fp.st32);
    const bool direct = allow_direct && in_matches && !pr.trans && !pl.check_inputs && npad == pr.n &&
                        kpad == pr.k && pr.aligned && ((pr.lda * in_size) % 16 == 0) &&
                        ((pr.a_off * in_size) % 16 == 0);
    CarRef a;
    if (direct) {
        a.buf = BUF_A;
        a.off = pr.a_off * in_size;
        a.ps = 0;
        a.ld = (int32_t)pr.lda;
        pl.direct = true;
    } else {
        a = B.new_car(npad, kpad, B.npo_leaf);
        CondTask ct{};
        ct.n = (int32_t)pr.n;
        ct.k = (int32_t)pr.k;
        ct.npad = (int32_t)npad;
        ct.kpad = (int32_t)kpad;
        ct.lda = (int32_t)pr.lda;
        ct.dt_in = pr.dA;
        ct.buf_re = BUF_A;
        ct.buf_im = BUF_A2;
        ct.off_re = ct.off_im = pr.a_off * in_size;
        ct.out = a;
        ct.trans = pr.trans;
        // the 2M base case reads planes re, im and re + im: without recursion (the input
        // itself is the leaf) nothing reads -re
        ct.skip = pl.herk2m && levels == 0 ? 1 << 2 : 0;
        if (pr.trans) {
            // 64 x 64 tiles of the carrier; grid (largest task, tasks)
            pl.cond_trans = true;
            const int64_t tiles = ((npad + 63) / 64) * ((kpad + 63) / 64);
            if (tiles >= (1ll << 31)) return FFA_EINVAL;
            pl.cond_max_blocks = (int)std::max<int64_t>(pl.cond_max_blocks, tiles);
        } else {
            // blocks of 256 threads x 16 (fp64: 4) carrier columns, one grid for all tasks
            const int64_t vec = pl.carrier == CAR_F64 ? 4 : 16;
            const int64_t blocks = (npad * (kpad / vec) + 255) / 256;
            if ((int64_t)pl.cond_max_blocks + blocks >= (1ll << 31)) return FFA_EINVAL;
            ct.blk0 = pl.cond_max_blocks;
            pl.cond_max_blocks += (int)blocks;
        }
        pl.cond.push_back(ct);
    }
    // largest operand magnitude: centred carriers, except direct canonical fp64
    if (pl.carrier == CAR_F64) pl.max_abs = std::max<int>(pl.max_abs, direct ? (int)pl.fp.p - 1 : pl.fp.half);
    else pl.max_abs = std::max<int>(pl.max_abs, pl.nl == 1 ? pl.fp.half : 32896);
    const ResRef c = root_output(pl, B, pr);
    B.node(0, a, npad, kpad, c, pr.n, true);  // with no recursion: the base case itself
    return FFA_OK;
}

// Product kernel configuration: built-in choice by size, or FFA_I8_CFG (tuning).
void choose_kernel(Plan& pl, int64_t max_dim)
{
    if (pl.carrier == CAR_F64) {
        pl.gemm_cfg = 0;
        pl.tile = gemm_tile_f64();
        pl.ktile = KTILE_F64;
        return;
    }
    int cfg = gemm_i8_default_config(pl.nl, pl.cplx, max_dim);
    // recursive one-limb plans: configuration 34 with the thread index's range restated
    // (1.76 vs 1.80 ms per call with one level at 16384^2, p = 251; without recursion it
    // is the slower one: 1.73-1.76 vs 1.70-1.71 ms)
    if (cfg == 34 && pl.levels > 0) cfg = 42;
    if (pl.kernel_req > 0 && gemm_i8_config_valid(pl.kernel_req - 1, pl.nl, pl.cplx))
        cfg = pl.kernel_req - 1;
    pl.gemm_cfg = cfg;
    pl.tile = gemm_i8_config_tile(cfg);
    pl.ktile = gemm_i8_config_ktile(cfg);
    if (pl.herk2m) {
        // the real launch of the 2M base case; K is padded for both k-tiles
        pl.gemm_cfg_r = gemm_i8_default_config(pl.nl, 0, max_dim);
        if (pl.kernel_req > 0 && gemm_i8_config_valid(pl.kernel_req - 1, pl.nl, 0))
            pl.gemm_cfg_r = pl.kernel_req - 1;
        pl.ktile = std::max(pl.ktile, gemm_i8_config_ktile(pl.gemm_cfg_r));
    }
}

// Whether a problem's products can read the caller's uint16 rows directly: two
// limbs of a real field, no recursion (nothing else reads A), no input check,
// 16-byte aligned rows, and a product kernel that loads through registers.  The
// kernel reads whole 16-byte chunks of a row (the columns past k are zeroed after
// the load), so the row's last chunk must be inside the caller's buffer: k a
// multiple of 8, or the library's packed layout, whose rows are padded to 16 bytes.
// Product configuration of the batches that read raw uint16 operands by default.
constexpr int RAW_BATCH_CONFIG = 39;

bool raw_u16_ok(const Plan& pl, const Problem& pr, int levels)
{
    return pl.carrier == CAR_I8 && pl.nl == 2 && !pl.cplx && gemm_i8_config_raw(pl.gemm_cfg) && pr.dA == FFA_U16 &&
           levels == 0 && !pr.trans && (pr.k % 8 == 0 || pr.packed) &&
           !pl.check_inputs && pr.k > 0 && pr.aligned && (pr.lda * 2) % 16 == 0 &&
           (pr.a_off * 2) % 16 == 0 && pr.lda * 2 < (1ll << 31) / 256;
}

Builder make_builder(Plan& pl)
{
    Builder B{pl};
    B.esize = pl.carrier == CAR_F64 ? (pl.fp.st32 ? 4 : 8) : 1;
    B.npo = pl.cplx ? 3 : 1;
    B.npo_leaf = pl.herk2m ? 4 : B.npo;
    B.rdt = pl.fp.p < 256 ? DT_U8 : (pl.fp.p < 65536 ? DT_U16 : DT_I32);
    B.rsize = dtype_size(B.rdt);
    B.bt = pl.tile;
    B.bt_r = pl.herk2m ? gemm_i8_config_tile(pl.gemm_cfg_r) : pl.tile;
    return B;
}

}  // namespace

Plan make_plan(const Problem& pr)
{
    Plan pl;
    const ffa_opts& o = pr.opts;
    if (pr.n < 0 || pr.k < 0) { pl.status = FFA_EINVAL; return pl; }
    Common cm = common_setup(pr.p, pr.herm, pr.dA, pr.dC, o);
    if (cm.status) { pl.status = cm.status; return pl; }
    if (pr.trans != 0 && pr.trans != 1) { pl.status = FFA_EINVAL; return pl; }
    if (pr.n > 0 && pr.k > 0 && pr.lda < (pr.trans ? pr.n : pr.k)) { pl.status = FFA_EINVAL; return pl; }
    if (pr.alpha >= pr.p || pr.beta >= pr.p) { pl.status = FFA_EINVAL; return pl; }
    if (pr.herm && (pr.trans || pr.alpha != 1 || pr.beta != 0)) { pl.status = FFA_EUNSUPPORTED; return pl; }
    if (pr.n > 0 && pr.ldc < pr.n) { pl.status = FFA_EINVAL; return pl; }
    if (pr.lda >= (1ll << 31) || pr.ldc >= (1ll << 31) || pr.n > FFA_N_MAX || pr.k >= (1ll << 31)) {
        pl.status = FFA_EINVAL;
        return pl;
    }
    pl.carrier = cm.carrier;
    pl.nl = cm.nl;
    pl.cplx = pr.herm ? 1 : 0;
    pl.fp = cm.fp;
    pl.check_inputs = o.check_inputs ? 1 : 0;
    pl.fp.alpha = (int32_t)pr.alpha;
    pl.fp.beta = (int32_t)pr.beta;
    if (pr.n == 0) return pl;
    if (o.herk_base < FFA_HERK_AUTO || o.herk_base > FFA_HERK_4M) { pl.status = FFA_EINVAL; return pl; }
    pl.herk2m = pl.cplx && pl.carrier == CAR_I8 && o.herk_base != FFA_HERK_4M;
    pl.fp.npo = pl.herk2m ? 4 : 3;
    pl.levels = choose_levels(pr.n, pr.k, o, pl.carrier, pl.nl, pl.cplx, pl.herk2m);
    // fp64 carrier with recursion: blocks held as fp32 (exact below 2^24), which halves
    // the traffic of the additions; without recursion the products read the caller's
    // doubles directly
    pl.fp.st32 = pl.carrier == CAR_F64 && pl.levels > 0 && !pr.trans && pr.p < (1u << 24) ? 1 : 0;
    pl.pre.assign(pl.levels, {});
    pl.post.assign(pl.levels, {});
    pl.kernel_req = o.kernel;
    if (o.general < FFA_GENERAL_AUTO || o.general > FFA_GENERAL_WINOGRAD || o.wino_min < 0 ||
        o.persist < FFA_PERSIST_AUTO || o.persist > FFA_PERSIST_ON) {
        pl.status = FFA_EINVAL;
        return pl;
    }
    // measured: Winograd's block additions pay off for the large fp64 products, not for
    // the faster INT8 ones; below about 2048 rows the additions cost more than they save
    const bool wino_default = pl.carrier == CAR_F64;
    pl.wino = (o.general == FFA_GENERAL_WINOGRAD || (o.general == FFA_GENERAL_AUTO && wino_default)) &&
              !pl.cplx && pl.levels > 0;
    pl.wino_min = o.wino_min > 0 ? o.wino_min : (o.general == FFA_GENERAL_AUTO ? 2048 : 0);
    choose_kernel(pl, pr.n >> pl.levels);
    // the problem's tasks on top of the settings above (pl is copied so that a
    // second attempt starts from the same state)
    const Plan base = pl;
    auto build = [&](Plan& q, int src) {
        q.gemm_src = src;
        Builder B = make_builder(q);
        const int st = add_problem(q, B, pr, q.levels, true);
        if (st) q.status = st;
        q.ws_bytes = B.ws;
    };
    const bool raw_ok = raw_u16_ok(pl, pr, pl.levels);
    build(pl, raw_ok && o.operands == FFA_OPERANDS_RAW ? SRC_RAW_U16 : SRC_CARRIER);
    if (pl.status == FFA_EUNSUPPORTED && o.operands == FFA_OPERANDS_AUTO) {
        // limb planes too large for the product kernel's 32-bit offsets: raw
        // operands need no planes; they need a configuration that loads through
        // registers (the built-in two-limb one that does, unless one was asked for)
        Plan q = base;
        if (q.kernel_req == 0 && q.carrier == CAR_I8 && q.nl == 2 && !q.cplx && !gemm_i8_config_raw(q.gemm_cfg)) {
            q.gemm_cfg = gemm_i8_default_config(2, 0, 0);
            q.tile = gemm_i8_config_tile(q.gemm_cfg);
            q.ktile = gemm_i8_config_ktile(q.gemm_cfg);
        }
        if (raw_u16_ok(q, pr, q.levels)) {
            pl = q;
            build(pl, SRC_RAW_U16);
        }
    }
    if (pl.status != FFA_OK && pl.status != FFA_EBOUND && pl.status != FFA_EUNSUPPORTED) return pl;
    if (pl.status == FFA_OK) pl.status = check_bound(pl);
    pl.zero_fill = pr.k == 0;
    pl.fork = o.streams == FFA_STREAMS_TWO && pl.levels > 0 && !pl.herk2m && !pl.wino;
    pl.split_tail = !pl.fork;
    // pre-additions beside the product launch (streams AUTO): one limb of a real field,
    // one level, carrier operands, 16-byte column groups in each half of a block
    pl.overlap_pre = o.streams == FFA_STREAMS_AUTO && pl.status == FFA_OK && pl.levels == 1 &&
                     pl.carrier == CAR_I8 && pl.nl == 1 && !pl.cplx && pl.wpre.empty() &&
                     pl.gemm_src == SRC_CARRIER && pl.pre.size() == 1 && pl.pre[0].size() == 1 &&
                     (pl.pre[0][0].w / 2) % 16 == 0;
    if (pl.overlap_pre) {
        pl.pre_blocks = PRE_SIGNAL_BLOCKS;
        pl.wait_off = round_up(pl.ws_bytes, 256);
        pl.ws_bytes = pl.wait_off + 256;  // the counter and the timeout word
        for (size_t t = 0; t < pl.gemm.size(); ++t)
            if (!pl.gemm_aonly[t]) {
                pl.gemm[t].wait = pl.pre_blocks;
                pl.gemm[t].wait_off = pl.wait_off;
            }
    }
    // a single call's product launch runs persistent on request only, and never beside
    // the pre-additions (a waiting tile would hold its slot) or split over two streams
    pl.persist = o.persist == FFA_PERSIST_ON && pl.status == FFA_OK && pl.carrier == CAR_I8 &&
                 !pl.overlap_pre && !pl.fork;
    if (pl.persist) {
        pl.queue_off = round_up(pl.ws_bytes, 256);
        pl.ws_bytes = pl.queue_off + 256;
    }
    size_grids(pl);
    return pl;
}

Plan make_batch_plan(const std::vector<Problem>& prs)
{
    Plan pl;
    if (prs.empty()) { pl.status = FFA_EINVAL; return pl; }
    const Problem& p0 = prs[0];
    Common cm = common_setup(p0.p, p0.herm, p0.dA, p0.dC, p0.opts);
    if (cm.status) { pl.status = cm.status; return pl; }
    pl.carrier = cm.carrier;
    pl.nl = cm.nl;
    pl.cplx = p0.herm ? 1 : 0;
    pl.fp = cm.fp;
    pl.check_inputs = p0.opts.check_inputs ? 1 : 0;
    if (p0.opts.herk_base < FFA_HERK_AUTO || p0.opts.herk_base > FFA_HERK_4M) { pl.status = FFA_EINVAL; return pl; }
    pl.herk2m = pl.cplx && pl.carrier == CAR_I8 && p0.opts.herk_base != FFA_HERK_4M;
    pl.fp.npo = pl.herk2m ? 4 : 3;
    const ffa_opts& o0 = p0.opts;
    if (o0.general < FFA_GENERAL_AUTO || o0.general > FFA_GENERAL_WINOGRAD || o0.wino_min < 0 ||
        o0.persist < FFA_PERSIST_AUTO || o0.persist > FFA_PERSIST_ON) {
        pl.status = FFA_EINVAL;
        return pl;
    }
    int maxL = 0;
    std::vector<int> L(prs.size());
    for (size_t i = 0; i < prs.size(); ++i) {
        if (prs[i].n < 0 || prs[i].k < 0 || prs[i].n > FFA_N_MAX || prs[i].k >= (1ll << 30)) {
            pl.status = FFA_EINVAL;
            return pl;
        }
        L[i] = choose_levels(prs[i].n, prs[i].k, p0.opts, pl.carrier, pl.nl, pl.cplx, pl.herk2m);
        maxL = std::max(maxL, L[i]);
    }
    pl.levels = maxL;
    pl.pre.assign(maxL, {});
    pl.post.assign(maxL, {});
    // Strassen-Winograd for the general products, as for single calls
    pl.wino = (o0.general == FFA_GENERAL_WINOGRAD || (o0.general == FFA_GENERAL_AUTO && pl.carrier == CAR_F64)) &&
              !pl.cplx && maxL > 0;
    pl.wino_min = o0.wino_min > 0 ? o0.wino_min : (o0.general == FFA_GENERAL_AUTO ? 2048 : 0);
    int64_t maxn = 0;
    for (const auto& q : prs) maxn = std::max(maxn, q.n);
    pl.kernel_req = p0.opts.kernel;
    choose_kernel(pl, maxn);
    const int ain = dtype_size(p0.dA), cout = dtype_size(p0.dC);
    // packed layout: A_i rows padded to 16 bytes, every A_i and C_i 16-byte aligned
    auto lda_of = [&](const Problem& q) { return round_up(std::max<int64_t>(q.k, 1), 16 / ain); };
    // Many small two-limb problems without recursion: unless a configuration or the
    // operand source is asked for, the products read the caller's uint16 rows with
    // configuration 39 (no conditioning pass; four workgroups per CU), the plan the
    // autotuner keeps for such batches (1.28-1.31 ms against 1.65-1.78 ms with limb
    // planes for 4096 problems of n in [32, 512] at p = 65521)
    const bool auto_raw = p0.opts.operands == FFA_OPERANDS_AUTO && p0.opts.kernel == 0 && pl.carrier == CAR_I8 &&
                          pl.nl == 2 && !pl.cplx && maxL == 0 && maxn < 2048;
    if (auto_raw) {
        pl.gemm_cfg = RAW_BATCH_CONFIG;
        pl.tile = gemm_i8_config_tile(pl.gemm_cfg);
        pl.ktile = gemm_i8_config_ktile(pl.gemm_cfg);
    }
    if (p0.opts.operands == FFA_OPERANDS_RAW || auto_raw) {
        bool raw = true;
        int64_t off = 0;
        for (size_t i = 0; i < prs.size() && raw; ++i) {
            Problem q = prs[i];
            q.lda = lda_of(q);
            q.a_off = off;
            q.packed = true;
            off += round_up(q.n * q.lda * ain, 16) / ain;
            raw = q.n == 0 || raw_u16_ok(pl, q, L[i]);
        }
        if (raw) pl.gemm_src = SRC_RAW_U16;
        else if (auto_raw) choose_kernel(pl, maxn);  // limb planes with the built-in configuration
    }
    Builder B = make_builder(pl);
    int64_t aoff = 0, coff = 0;
    for (size_t i = 0; i < prs.size(); ++i) {
        Problem q = prs[i];
        q.lda = lda_of(q);
        q.ldc = std::max<int64_t>(q.n, 1);
        q.a_off = aoff;
        q.c_off = coff;
        pl.a_off.push_back(aoff);
        pl.c_off.push_back(coff);
        pl.a_ld.push_back(q.lda);
        aoff += round_up(q.n * q.lda * ain, 16) / ain;
        coff += round_up(q.n * q.n * cout, 16) / cout;
        // packed buffers beyond any device memory (and far from int64 overflow)
        if (aoff > (1ll << 44) || coff > (1ll << 44)) { pl.status = FFA_EINVAL; return pl; }
        if (q.n == 0) continue;
        // problems of one batch share one set of levels per problem; the
        // Builder keeps per-level task lists across problems
        const int saved = pl.levels;
        pl.levels = L[i];
        int st = add_problem(pl, B, q, L[i], true);
        pl.levels = saved;
        if (st) { pl.status = st; return pl; }
    }
    pl.a_total = aoff;
    pl.c_total = coff;
    pl.ws_bytes = B.ws;
    if (pl.status == FFA_OK) pl.status = check_bound(pl);
    pl.fork = p0.opts.streams == FFA_STREAMS_TWO && pl.levels > 0;
    // a batch's many short tiles: persistent unless asked otherwise
    pl.persist = o0.persist != FFA_PERSIST_OFF && pl.status == FFA_OK && pl.carrier == CAR_I8 && !pl.fork;
    if (pl.persist) {
        pl.queue_off = round_up(pl.ws_bytes, 256);
        pl.ws_bytes = pl.queue_off + 256;
    }
    size_grids(pl);
    return pl;
}

std::vector<char> pack_tables(Plan& pl)
{
    std::vector<char> blob;
    auto put = [&](const void* src, size_t bytes) -> int64_t {
        const int64_t off = round_up((int64_t)blob.size(), 256);
        blob.resize(off + bytes);
        if (bytes) std::copy((const char*)src, (const char*)src + bytes, blob.begin() + off);
        return off;
    };
    pl.off_cond = put(pl.cond.data(), pl.cond.size() * sizeof(CondTask));
    pl.off_pre.assign(pl.levels, 0);
    pl.off_post.assign(pl.levels, 0);
    for (int l = 0; l < pl.levels; ++l) {
        pl.off_pre[l] = put(pl.pre[l].data(), pl.pre[l].size() * sizeof(PreaddTask));
        pl.off_post[l] = put(pl.post[l].data(), pl.post[l].size() * sizeof(PostaddTask));
    }
    pl.off_gemm = put(pl.gemm.data(), pl.gemm.size() * sizeof(GemmTask));
    pl.off_sched = put(pl.sched.data(), pl.sched.size() * sizeof(TileEnt));
    pl.off_sched2 = put(pl.sched2.data(), pl.sched2.size() * sizeof(TileEnt));
    pl.off_upd = put(pl.upd.data(), pl.upd.size() * sizeof(UpdateTask));
    pl.off_gemm_r = put(pl.gemm_r.data(), pl.gemm_r.size() * sizeof(GemmTask));
    pl.off_sched_r = put(pl.sched_r.data(), pl.sched_r.size() * sizeof(TileEnt));
    pl.off_h2m = put(pl.h2m.data(), pl.h2m.size() * sizeof(Herk2mTask));
    pl.off_wpre = put(pl.wpre.data(), pl.wpre.size() * sizeof(WinoPreTask));
    pl.off_wpost = put(pl.wpost.data(), pl.wpost.size() * sizeof(WinoPostTask));
    pl.off_tail = put(pl.tail.data(), pl.tail.size() * sizeof(TailTask));
    pl.blob_bytes = (int64_t)blob.size();
    return blob;
}

std::string describe(const Plan& pl)
{
    char buf[2048];
    std::string pre = "[", post = "[";
    for (int l = 0; l < pl.levels; ++l) {
        pre += std::to_string(pl.pre[l].size()) + (l + 1 < pl.levels ? "," : "");
        post += std::to_string(pl.post[l].size()) + (l + 1 < pl.levels ? "," : "");
    }
    pre += "]";
    post += "]";
    snprintf(buf, sizeof(buf),
             "{\"status\":%d,\"levels\":%d,\"carrier\":\"%s\",\"limbs\":%d,\"complex\":%d,"
             "\"npad\":%lld,\"kpad\":%lld,\"direct\":%d,\"max_abs\":%d,\"max_k\":%lld,"
             "\"ws_bytes\":%lld,\"conditioning\":%zu,\"preadd_tasks\":%s,\"postadd_tasks\":%s,"
             "\"gemm_tasks\":%zu,\"tiles\":%d,\"blocks\":%zu,\"cfg\":%d,\"tile\":%d,"
             "\"macs\":%lld,\"ykind\":%d,\"ya\":%d,\"yb\":%d,\"src\":\"%s\",\"streams\":%d,"
             "\"blocks_a_only\":%zu,\"herk_base\":\"%s\",\"real_tasks\":%zu,\"general\":\"%s\","
             "\"wino_tasks\":%zu,\"wino_min\":%lld,\"cfg_real\":%d,\"st32\":%d,\"tail_tiles\":%zu,"
             "\"overlap_pre\":%d,\"persist\":%d}",
             pl.status, pl.levels, pl.carrier == CAR_F64 ? "f64" : "int8", pl.nl, pl.cplx,
             (long long)pl.npad, (long long)pl.kpad, pl.direct ? 1 : 0, pl.max_abs,
             (long long)pl.max_k, (long long)pl.ws_bytes, pl.cond.size(), pre.c_str(), post.c_str(),
             pl.gemm.size(), pl.total_tiles, pl.sched.size() + pl.sched2.size(), pl.gemm_cfg, pl.tile,
             (long long)pl.products_macs, pl.fp.ykind, pl.fp.ya,
             pl.fp.yb, pl.gemm_src == SRC_RAW_U16 ? "raw_u16" : "carrier", pl.fork ? 2 : 1,
             pl.sched.size(), pl.herk2m ? "2m" : (pl.cplx ? "4m" : "none"), pl.gemm_r.size(),
             pl.wpre.empty() ? "classical" : "winograd", pl.wpre.size(), (long long)pl.wino_min,
             pl.herk2m ? pl.gemm_cfg_r : -1, pl.fp.st32, pl.tail.size(), pl.overlap_pre ? 1 : 0,
             pl.persist ? 1 : 0);
    return buf;
}

}  // namespace ffa
