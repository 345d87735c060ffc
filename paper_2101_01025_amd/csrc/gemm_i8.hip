// Grouped product kernel on INT8 MFMA (gfx950 v_mfma_i32_32x32x32_i8).
//
// Computes, for every task of a table, C = X * phi(Z) mod p on square tiles:
// the general products P3 = A22 phi(S4), P4 = S1 phi(S2) of every recursion
// level and the base-case products Low(X phi(X)) (Algorithm 1, Section 3) in
// ONE launch.  A task with syrk = 1 only has tiles on or below the diagonal
// and writes row >= col.
//
// Exactness: operands are balanced int8 limbs of residues, accumulation is in
// int32 and exact (the planner bounds K * max|x| * max|y| below 2^31 for each
// accumulator); with two limbs x = 256 hi + lo the tile keeps three
// accumulators hh, (hl + lh), ll and recombines 65536 hh + 256 mid + ll
// exactly before the reduction mod p.
// Complex operands (F_p[i], phi = conjugate transpose) use planes re, im and
// -re:  Re(X Z^H) = Xr Zr^T + Xi Zi^T,  Im(X Z^H) = Xi Zr^T + (-Xr) Zi^T, i.e.
// two K-segments that share the B operand (Zr, then Zi) and two A roles.
//
// Data movement: global -> registers (a ring of PF k-tiles in flight) -> LDS
// (double buffer, XOR-swizzled 16-byte segments so that the ds_read_b128 of
// consecutive rows hits distinct banks) -> MFMA.  Which tile a workgroup
// computes comes from a host-built schedule indexed by blockIdx: tiles are
// grouped into L2-friendly blocks and the blocks are dealt to the 8 XCDs
// (workgroup b runs on XCD b mod 8) so that each XCD's L2 serves a compact set
// of operand panels and every XCD gets the same amount of work.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "ffa_internal.h"

namespace ffa {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// LDS byte offset of 16-byte segment seg of row r in a tile with KT-byte rows.
template <int KT>
__device__ __forceinline__ int swz(int r, int seg)
{
    constexpr int NSEG = KT / 16;
    constexpr int RPB = 256 / KT;  // rows per 256-byte bank row
    return r * KT + ((seg ^ ((r / RPB) & (NSEG - 1))) << 4);
}

// Canonical residue of an int32 for any odd p < 2^16 (|x| < 2^31 - 2^16).
__device__ __forceinline__ int32_t mod_i32(int32_t x, int32_t p, float inv_p)
{
    int32_t q = (int32_t)floorf((float)x * inv_p);
    int32_t r = (int32_t)((uint32_t)x - (uint32_t)q * (uint32_t)p);
    q = (int32_t)floorf((float)r * inv_p);
    r -= q * p;
    r += (r < 0) ? p : 0;
    r -= (r >= p) ? p : 0;
    return r;
}

// Canonical residue of an int32 for p < 2^8 with full-rate 24-bit arithmetic:
// x = hi 2^16 + lo, v = hi (2^16 mod p) + lo has |v| < 2^24 (exact in fp32), one
// fp32 quotient within one of v / p, then a correction.  c16 = 2^16 mod p.
__device__ __forceinline__ int32_t mod_small_p(int32_t x, int32_t p, int32_t c16, float inv_p)
{
    const int32_t hi = x >> 16, lo = x & 0xffff;
    const int32_t v = __mul24(hi, c16) + lo;
    const int32_t q = (int32_t)floorf((float)v * inv_p);
    int32_t r = v - __mul24(q, p);
    r += (r < 0) ? p : 0;
    r -= (r >= p) ? p : 0;
    return r;
}

template <int NL, int CPLX, int BT, int WGM, int WGN, int KT, int PF>
__global__ void __launch_bounds__(WGM* WGN * 64)
    gemm_i8(Bases bases, const GemmTask* __restrict__ tasks, const TileEnt* __restrict__ sched,
            FieldParams fp)
{
    constexpr int NT = WGM * WGN * 64;
    constexpr int NROLE = CPLX ? 2 : 1;
    constexpr int NSEG = CPLX ? 2 : 1;
    constexpr int NA = NROLE * NL;  // A sub-tiles per stage
    constexpr int NB = NL;          // B sub-tiles per stage
    constexpr int WM = BT / WGM, WN = BT / WGN;
    constexpr int FM = WM / 32, FN = WN / 32;
    constexpr int NACC = NL == 1 ? 1 : 3;
    constexpr int TILE = BT * KT;
    constexpr int STAGE = (NA + NB) * TILE;
    constexpr int SPR = KT / 16;  // 16-byte segments per row
    constexpr int ACH = NA * TILE / 16 / NT;
    constexpr int BCH = NB * TILE / 16 / NT;
    static_assert(NA * TILE % (16 * NT) == 0 && NB * TILE % (16 * NT) == 0, "chunking");
    static_assert(FM >= 1 && FN >= 1, "wave tile");

    extern __shared__ __attribute__((aligned(16))) char lds[];

    const TileEnt ent = sched[blockIdx.x];
    if (ent.x < 0) return;  // padding entry of the XCD-balanced schedule
    const GemmTask& T = tasks[ent.x];
    const int row0 = (ent.y & 0xffff) * BT, col0 = (ent.y >> 16) * BT;
    const int M = T.M, N = T.N, K = T.K;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave / WGN) * WM, wn0 = (wave % WGN) * WN;

    // ---- operand panels as buffer resources: every load is (constant per-thread
    // offset, stage offset in a scalar register).  Rows past the matrix are clamped
    // to its last row; the resource extent covers exactly the rows of this tile.
    constexpr int NSUB = (CPLX ? 3 : 1) * NL;  // carrier sub-planes an operand may touch
    const int rows_a = min(BT, M - row0), rows_b = min(BT, N - col0);
    const char* abase = bases.p[T.x.buf] + T.x.off + (int64_t)row0 * T.x.ld;
    const char* bbase = bases.p[T.z.buf] + T.z.off + (int64_t)col0 * T.z.ld;
    const int ext_a = (int)((NSUB - 1) * T.x.ps + (int64_t)rows_a * T.x.ld);
    const int ext_b = (int)((NSUB - 1) * T.z.ps + (int64_t)rows_b * T.z.ld);
    const __amdgpu_buffer_rsrc_t rsa = __builtin_amdgcn_make_buffer_rsrc((void*)abase, (short)0, ext_a, 0x00020000);
    const __amdgpu_buffer_rsrc_t rsb = __builtin_amdgcn_make_buffer_rsrc((void*)bbase, (short)0, ext_b, 0x00020000);
    int aoff[ACH], boff[BCH], alds[ACH], blds[BCH];
#pragma unroll
    for (int i = 0; i < ACH; ++i) {
        const int c = tid + i * NT;
        const int sub = c / (BT * SPR), r = (c / SPR) % BT, s = c % SPR;
        aoff[i] = (int)(sub * T.x.ps + (int64_t)min(r, rows_a - 1) * T.x.ld) + s * 16;
        alds[i] = sub * TILE + swz<KT>(r, s);
    }
#pragma unroll
    for (int i = 0; i < BCH; ++i) {
        const int c = tid + i * NT;
        const int sub = c / (BT * SPR), r = (c / SPR) % BT, s = c % SPR;
        boff[i] = (int)(sub * T.z.ps + (int64_t)min(r, rows_b - 1) * T.z.ld) + s * 16;
        blds[i] = (NA + sub) * TILE + swz<KT>(r, s);
    }
    // Complex: A sub-tile index sub = role * NL + limb reads plane role (segment 0) and
    // plane role + 1 (segment 1); B reads plane 0 then plane 1.
    const int nkc = K / KT;
    const int nst = NSEG * nkc;
    const int seg_a = (int)(NL * T.x.ps), seg_b = (int)(NL * T.z.ps);

    v4i ra[PF][ACH], rb[PF][BCH];
    auto gload = [&](int st, v4i* a, v4i* b) {
        const int seg = st >= nkc ? 1 : 0;
        const int kc = st - seg * nkc;
        const int oa = seg * seg_a + kc * KT, ob = seg * seg_b + kc * KT;
#pragma unroll
        for (int i = 0; i < ACH; ++i) a[i] = __builtin_amdgcn_raw_buffer_load_b128(rsa, aoff[i], oa, 0);
#pragma unroll
        for (int i = 0; i < BCH; ++i) b[i] = __builtin_amdgcn_raw_buffer_load_b128(rsb, boff[i], ob, 0);
    };
    auto sstore = [&](int buf, const v4i* a, const v4i* b) {
        char* base = lds + buf * STAGE;
#pragma unroll
        for (int i = 0; i < ACH; ++i) *reinterpret_cast<v4i*>(base + alds[i]) = a[i];
#pragma unroll
        for (int i = 0; i < BCH; ++i) *reinterpret_cast<v4i*>(base + blds[i]) = b[i];
    };

    v16i acc[NROLE][NACC][FM][FN];
#pragma unroll
    for (int r = 0; r < NROLE; ++r)
#pragma unroll
        for (int a = 0; a < NACC; ++a)
#pragma unroll
            for (int m = 0; m < FM; ++m)
#pragma unroll
                for (int n = 0; n < FN; ++n)
#pragma unroll
                    for (int v = 0; v < 16; ++v) acc[r][a][m][n][v] = 0;

    const int lrow = lane & 31, lseg = lane >> 5;
    // fragment reads of k-step ks (32 bytes of K) from an LDS stage
    auto load_frags = [&](const char* base, int ks, v4i (*af)[FM], v4i (*bf)[FN]) {
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
            for (int m = 0; m < FM; ++m)
                af[a][m] = *reinterpret_cast<const v4i*>(
                    base + a * TILE + swz<KT>(wm0 + m * 32 + lrow, ks * 2 + lseg));
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int n = 0; n < FN; ++n)
                bf[b][n] = *reinterpret_cast<const v4i*>(
                    base + (NA + b) * TILE + swz<KT>(wn0 + n * 32 + lrow, ks * 2 + lseg));
    };
    auto mfmas = [&](v4i (*af)[FM], v4i (*bf)[FN]) {
        if (NL == 1) {
#pragma unroll
            for (int r = 0; r < NROLE; ++r)
#pragma unroll
                for (int m = 0; m < FM; ++m)
#pragma unroll
                    for (int n = 0; n < FN; ++n)
                        acc[r][0][m][n] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                            af[r][m], bf[0][n], acc[r][0][m][n], 0, 0, 0);
        } else {
            // limb products (hi,hi) -> 0, (hi,lo) and (lo,hi) -> 1, (lo,lo) -> 2, ordered
            // so that consecutive MFMAs do not share an accumulator
#pragma unroll
            for (int pr = 0; pr < 4; ++pr) {
                const int la = pr >> 1, lb = pr & 1;
                const int ai = (pr == 0) ? 0 : (pr == 3 ? 2 : 1);
#pragma unroll
                for (int r = 0; r < NROLE; ++r)
#pragma unroll
                    for (int m = 0; m < FM; ++m)
#pragma unroll
                        for (int n = 0; n < FN; ++n)
                            acc[r][ai][m][n] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                af[r * NL + la][m], bf[lb][n], acc[r][ai][m][n], 0, 0, 0);
            }
        }
    };
    // the fragments of k-step ks + 1 are read while the MFMAs of k-step ks run
    constexpr int NKS = KT / 32;
    auto compute = [&](int buf) {
        const char* base = lds + buf * STAGE;
        v4i af[2][NA][FM], bf[2][NB][FN];
        load_frags(base, 0, af[0], bf[0]);
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
            if (ks + 1 < NKS) load_frags(base, ks + 1, af[(ks + 1) & 1], bf[(ks + 1) & 1]);
            mfmas(af[ks & 1], bf[ks & 1]);
        }
    };

    // ---- pipeline: PF k-tiles in flight in registers, two LDS buffers
#pragma unroll
    for (int u = 0; u < PF; ++u)
        if (u < nst) gload(u, ra[u], rb[u]);
    if (nst > 0) sstore(0, ra[0], rb[0]);
    __syncthreads();
    for (int st0 = 0; st0 < nst; st0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int st = st0 + u;
            if (st < nst) {
                // register slot u held stage st (already in LDS): refill it with stage st + PF
                if (st + PF < nst) gload(st + PF, ra[u], rb[u]);
                compute(st & 1);
                if (st + 1 < nst) sstore((st + 1) & 1, ra[(u + 1) % PF], rb[(u + 1) % PF]);
                __syncthreads();
            }
        }
    }

    // ---- epilogue: exact recombination, reduction mod p, store.  The output format is
    // switched on once, outside the fully unrolled fragment loops.
    // Output layout of the 32x32 MFMA: lane -> column (lane & 31), register v -> row
    // 8 (v / 4) + 4 (lane / 32) + v % 4 of the fragment.
    const int p = fp.p;
    const float inv_pf = (float)fp.inv_p;
    const int32_t c16 = (int32_t)(65536 % p);
    const int i0 = row0 + wm0 + 4 * (lane >> 5), j0 = col0 + wn0 + (lane & 31);
    const bool syrk = T.syrk != 0;
    const int64_t ldc = T.c.ld;
    // interior tiles (inside the matrix and strictly below the diagonal) need no checks
    const bool interior = row0 + BT <= M && col0 + BT <= N && (!syrk || row0 >= col0 + BT);
    auto epilogue = [&](auto tag) {
        using OT = decltype(tag);
#pragma unroll
        for (int r = 0; r < NROLE; ++r) {
            OT* cp = reinterpret_cast<OT*>(r == 0 ? bases.p[T.c.buf] + T.c.off
                                                  : bases.p[T.c.buf2] + T.c.off2);
#pragma unroll
            for (int m = 0; m < FM; ++m)
#pragma unroll
                for (int n = 0; n < FN; ++n)
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        int32_t res;
                        if (NL == 1) {
                            res = p < 256 ? mod_small_p(acc[r][0][m][n][v], p, c16, inv_pf)
                                          : mod_i32(acc[r][0][m][n][v], p, inv_pf);
                        } else {
                            const double val = 65536.0 * (double)acc[r][0][m][n][v] +
                                               256.0 * (double)acc[r][NACC - 2][m][n][v] +
                                               (double)acc[r][NACC - 1][m][n][v];
                            res = mod_canon(val, p, fp.inv_p);
                        }
                        const int i = i0 + m * 32 + 8 * (v >> 2) + (v & 3);
                        const int j = j0 + n * 32;
                        if (interior || (i < M && j < N && (!syrk || i >= j)))
                            cp[(int64_t)i * ldc + j] = (OT)res;
                        // keep the scheduler from hoisting the reads of every accumulator
                        if ((v & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                    }
        }
    };
    switch (T.c.dt) {
    case DT_U8: epilogue(uint8_t{}); break;
    case DT_U16: epilogue(uint16_t{}); break;
    case DT_I32: epilogue(int32_t{}); break;
    case DT_I64: epilogue(int64_t{}); break;
    case DT_F64: epilogue(double{}); break;
    default: break;
    }
}

// ---- configurations ---------------------------------------------------------
// id -> (limbs, complex, tile edge, wave grid, k-tile bytes, prefetch depth).
// Accumulator registers per lane: NROLE * NACC * (BT/WGM/32) * (BT/WGN/32) * 16.
struct CfgInfo {
    int nl, cplx, bt, kt, nthreads, lds;
};

#define FFA_I8_CONFIGS(X)                 \
    X(0, 1, 0, 256, 2, 2, 128, 2)         \
    X(1, 1, 0, 256, 2, 4, 64, 2)          \
    X(2, 1, 0, 128, 2, 2, 128, 2)         \
    X(3, 2, 0, 128, 2, 2, 128, 2)         \
    X(4, 1, 1, 128, 2, 2, 128, 2)         \
    X(5, 2, 1, 128, 2, 4, 64, 1)          \
    X(6, 2, 0, 128, 2, 2, 64, 2)          \
    X(7, 1, 0, 256, 2, 2, 64, 2)          \
    X(8, 2, 1, 64, 2, 2, 128, 2)          \
    X(9, 2, 0, 128, 2, 2, 128, 1)         \
    X(10, 1, 0, 256, 2, 4, 128, 2)        \
    X(11, 1, 0, 256, 2, 4, 64, 3)         \
    X(12, 1, 0, 256, 4, 2, 64, 2)

static CfgInfo cfg_info(int id)
{
#define FFA_INFO(ID, NL, CP, BT, WM, WN, KT, PF) \
    if (id == ID) return CfgInfo{NL, CP, BT, KT, WM * WN * 64, 2 * ((CP ? 2 : 1) * NL + NL) * BT * KT};
    FFA_I8_CONFIGS(FFA_INFO)
#undef FFA_INFO
    return CfgInfo{0, 0, 0, 0, 0, 0};
}

int gemm_i8_config_tile(int cfg) { return cfg_info(cfg).bt; }
int gemm_i8_config_ktile(int cfg) { return cfg_info(cfg).kt; }

int gemm_i8_config_valid(int cfg, int nl, int cplx)
{
    const CfgInfo ci = cfg_info(cfg);
    return ci.bt > 0 && ci.nl == nl && ci.cplx == cplx;
}

int gemm_i8_default_config(int nl, int cplx, int64_t max_dim)
{
    if (cplx) return nl == 1 ? 4 : 8;
    if (nl == 2) return 9;
    return max_dim >= 2048 ? 10 : 2;
}

template <int NL, int CPLX, int BT, int WGM, int WGN, int KT, int PF>
static int launch_cfg(const GemmTask* d_tasks, const TileEnt* d_sched, int nblocks, const Bases& b,
                      const FieldParams& fp, hipStream_t s)
{
    constexpr int NA = (CPLX ? 2 : 1) * NL, NB = NL;
    constexpr int lds_bytes = 2 * (NA + NB) * BT * KT;
    auto kern = gemm_i8<NL, CPLX, BT, WGM, WGN, KT, PF>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) return (int)e;
        attr_set = true;
    }
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(WGM * WGN * 64), lds_bytes, s, b, d_tasks,
                       d_sched, fp);
    return (int)hipGetLastError();
}

int launch_gemm_i8(int cfg, const GemmTask* d_tasks, const TileEnt* d_sched, int nblocks,
                   const Bases& b, const FieldParams& fp, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (nblocks <= 0) return 0;
#define FFA_LAUNCH(ID, NL, CP, BT, WM, WN, KT, PF) \
    if (cfg == ID) return launch_cfg<NL, CP, BT, WM, WN, KT, PF>(d_tasks, d_sched, nblocks, b, fp, s);
    FFA_I8_CONFIGS(FFA_LAUNCH)
#undef FFA_LAUNCH
    return (int)hipErrorInvalidValue;
}

}  // namespace ffa
