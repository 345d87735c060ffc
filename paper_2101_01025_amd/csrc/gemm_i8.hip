// Grouped product kernel on INT8 MFMA (gfx950 v_mfma_i32_32x32x32_i8).
//
// Computes, for every task of a table, C = X * phi(Z) mod p on square tiles:
// the general products P3 = A22 phi(S4), P4 = S1 phi(S2) of every recursion
// level and the base-case products Low(X phi(X)) (Algorithm 1, Section 3) in
// ONE launch.  A task with syrk = 1 only enumerates tiles on or below the
// diagonal and writes row >= col.
//
// Exactness: operands are balanced int8 limbs of residues, accumulation is in
// int32 and exact (the planner bounds K * max|x| * max|y| below 2^31 for each
// accumulator); with two limbs x = 256 hi + lo the tile keeps three
// accumulators hh, (hl + lh), ll and recombines 65536 hh + 256 mid + ll exactly
// in fp64 before the reduction mod p.
// Complex operands (F_p[i], phi = conjugate transpose) use planes re, im and
// -re:  Re(X Z^H) = Xr Zr^T + Xi Zi^T,  Im(X Z^H) = Xi Zr^T + (-Xr) Zi^T, i.e.
// two K-segments that share the B operand (Zr, then Zi) and two A roles.
//
// Data movement: global -> registers (prefetch of the next k-tile while the
// current one is multiplied) -> LDS (double buffer, XOR-swizzled 16-byte
// segments so that the ds_read_b128 of 32 consecutive rows is conflict free)
// -> MFMA.  Workgroups are remapped so that consecutive tiles run on the same
// XCD (round-robin dispatch over the 8 XCDs, each with its own L2).
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "ffa_internal.h"

namespace ffa {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int KT8 = 64;  // bytes of K per pipeline stage

__device__ __forceinline__ int swz(int row, int seg)
{
    return row * KT8 + ((seg ^ ((row >> 2) & 3)) << 4);
}

__device__ __forceinline__ int xcd_remap(int b, int G)
{
    const int xcd = b & 7, loc = b >> 3, per = G >> 3, rem = G & 7;
    return (xcd < rem) ? xcd * (per + 1) + loc : rem * (per + 1) + (xcd - rem) * per + loc;
}

__device__ __forceinline__ void tri_decode(int t, int& ti, int& tj)
{
    int r = (int)((sqrtf(8.f * (float)t + 1.f) - 1.f) * 0.5f);
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    while (r * (r + 1) / 2 > t) --r;
    ti = r;
    tj = t - r * (r + 1) / 2;
}

template <int NL, int CPLX, int BT, int WGM, int WGN>
__global__ void __launch_bounds__(WGM* WGN * 64)
    gemm_i8(Bases bases, const GemmTask* __restrict__ tasks, int ntasks, FieldParams fp)
{
    constexpr int NT = WGM * WGN * 64;
    constexpr int NROLE = CPLX ? 2 : 1;
    constexpr int NSEG = CPLX ? 2 : 1;
    constexpr int NA = NROLE * NL;  // A sub-tiles per stage
    constexpr int NB = NL;          // B sub-tiles per stage
    constexpr int WM = BT / WGM, WN = BT / WGN;
    constexpr int FM = WM / 32, FN = WN / 32;
    constexpr int NACC = NL == 1 ? 1 : 3;
    constexpr int TILE = BT * KT8;
    constexpr int STAGE = (NA + NB) * TILE;
    constexpr int ACH = NA * TILE / 16 / NT;
    constexpr int BCH = NB * TILE / 16 / NT;
    static_assert(NA * TILE % (16 * NT) == 0 && NB * TILE % (16 * NT) == 0, "chunking");
    static_assert(FM >= 1 && FN >= 1, "wave tile");

    extern __shared__ __attribute__((aligned(16))) char lds[];

    // ---- which tile of which task
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tasks[mid].tile_begin <= lid) lo = mid;
        else hi = mid - 1;
    }
    const GemmTask T = tasks[lo];
    const int t = lid - T.tile_begin;
    int ti, tj;
    if (T.syrk) tri_decode(t, ti, tj);
    else {
        ti = t / T.tiles_n;
        tj = t - ti * T.tiles_n;
    }
    const int row0 = ti * BT, col0 = tj * BT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave / WGN) * WM, wn0 = (wave % WGN) * WN;

    // ---- per-thread global source pointers (segment 0, k = 0)
    const char* aptr[ACH];
    const char* bptr[BCH];
    int alds[ACH], blds[BCH];
#pragma unroll
    for (int i = 0; i < ACH; ++i) {
        const int c = tid + i * NT;
        const int sub = c / (BT * 4), r = (c >> 2) % BT, s = c & 3;
        const int role = sub / NL, limb = sub % NL;
        const int grow = min(row0 + r, T.M - 1);
        aptr[i] = bases.p[T.x.buf] + T.x.off + (int64_t)(role * NL + limb) * T.x.ps +
                  (int64_t)grow * T.x.ld + s * 16;
        alds[i] = sub * TILE + swz(r, s);
    }
#pragma unroll
    for (int i = 0; i < BCH; ++i) {
        const int c = tid + i * NT;
        const int sub = c / (BT * 4), r = (c >> 2) % BT, s = c & 3;
        const int grow = min(col0 + r, T.N - 1);
        bptr[i] = bases.p[T.z.buf] + T.z.off + (int64_t)sub * T.z.ps + (int64_t)grow * T.z.ld +
                  s * 16;
        blds[i] = (NA + sub) * TILE + swz(r, s);
    }
    const int nkc = T.K / KT8;
    const int nst = NSEG * nkc;
    const int64_t seg_a = (int64_t)NL * T.x.ps, seg_b = (int64_t)NL * T.z.ps;

    v4i ra[ACH], rb[BCH];
    auto gload = [&](int st) {
        const int seg = st / nkc, kc = st - seg * nkc;
        const int64_t oa = seg * seg_a + (int64_t)kc * KT8;
        const int64_t ob = seg * seg_b + (int64_t)kc * KT8;
#pragma unroll
        for (int i = 0; i < ACH; ++i) ra[i] = *reinterpret_cast<const v4i*>(aptr[i] + oa);
#pragma unroll
        for (int i = 0; i < BCH; ++i) rb[i] = *reinterpret_cast<const v4i*>(bptr[i] + ob);
    };
    auto sstore = [&](int buf) {
        char* base = lds + buf * STAGE;
#pragma unroll
        for (int i = 0; i < ACH; ++i) *reinterpret_cast<v4i*>(base + alds[i]) = ra[i];
#pragma unroll
        for (int i = 0; i < BCH; ++i) *reinterpret_cast<v4i*>(base + blds[i]) = rb[i];
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

    if (nst > 0) {
        gload(0);
        sstore(0);
    }
    __syncthreads();
    const int lrow = lane & 31, lseg = lane >> 5;
    for (int st = 0; st < nst; ++st) {
        const int buf = st & 1;
        if (st + 1 < nst) gload(st + 1);
        const char* base = lds + buf * STAGE;
#pragma unroll
        for (int ks = 0; ks < KT8 / 32; ++ks) {
            v4i af[NA][FM], bf[NB][FN];
#pragma unroll
            for (int a = 0; a < NA; ++a)
#pragma unroll
                for (int m = 0; m < FM; ++m)
                    af[a][m] = *reinterpret_cast<const v4i*>(
                        base + a * TILE + swz(wm0 + m * 32 + lrow, ks * 2 + lseg));
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int n = 0; n < FN; ++n)
                    bf[b][n] = *reinterpret_cast<const v4i*>(
                        base + (NA + b) * TILE + swz(wn0 + n * 32 + lrow, ks * 2 + lseg));
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
                // limb products: (hi,hi) -> 0, (hi,lo) and (lo,hi) -> 1, (lo,lo) -> 2;
                // ordered so that consecutive MFMAs do not share an accumulator
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
        }
        if (st + 1 < nst) sstore(buf ^ 1);
        __syncthreads();
    }

    // ---- epilogue: exact recombination, reduction mod p, store
    const int p = fp.p;
    const double inv_p = fp.inv_p;
#pragma unroll
    for (int r = 0; r < NROLE; ++r) {
        char* cbase = (r == 0) ? bases.p[T.c.buf] + T.c.off : bases.p[T.c.buf2] + T.c.off2;
#pragma unroll
        for (int m = 0; m < FM; ++m)
#pragma unroll
            for (int n = 0; n < FN; ++n)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int i = row0 + wm0 + m * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                    const int j = col0 + wn0 + n * 32 + (lane & 31);
                    if (i < T.M && j < T.N && (!T.syrk || i >= j)) {
                        double val;
                        if (NL == 1) val = (double)acc[r][0][m][n][v];
                        else
                            val = 65536.0 * (double)acc[r][0][m][n][v] +
                                  256.0 * (double)acc[r][1][m][n][v] + (double)acc[r][2][m][n][v];
                        store_res(cbase, T.c.dt, (int64_t)i * T.c.ld + j, mod_canon(val, p, inv_p));
                    }
                }
    }
}

// ---- configurations --------------------------------------------------------
// (limbs, complex) -> tile edge BT and wave grid; accumulator registers per lane
// are NROLE * NACC * (BT/WGM/32) * (BT/WGN/32) * 16.
#define CFG_R1 1, 0, 256, 2, 4   // 128 acc regs, 8 waves
#define CFG_R2 2, 0, 128, 2, 2   // 192 acc regs, 4 waves
#define CFG_C1 1, 1, 128, 2, 2   // 128 acc regs, 4 waves
#define CFG_C2 2, 1, 128, 2, 4   // 192 acc regs, 8 waves

template <int NL, int CPLX, int BT, int WGM, int WGN>
static int launch_cfg(const GemmTask* d_tasks, int ntasks, int total_tiles, const Bases& b,
                      const FieldParams& fp, hipStream_t s)
{
    constexpr int NA = (CPLX ? 2 : 1) * NL, NB = NL;
    constexpr int lds_bytes = 2 * (NA + NB) * BT * KT8;
    auto kern = gemm_i8<NL, CPLX, BT, WGM, WGN>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) return (int)e;
        attr_set = true;
    }
    hipLaunchKernelGGL(kern, dim3(total_tiles), dim3(WGM * WGN * 64), lds_bytes, s, b, d_tasks,
                       ntasks, fp);
    return (int)hipGetLastError();
}

int gemm_tile_i8(int nl, int cplx)
{
    if (nl == 1 && !cplx) return 256;
    return 128;
}

int launch_gemm_i8(const GemmTask* d_tasks, int ntasks, int total_tiles, const Bases& b,
                   const FieldParams& fp, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (ntasks <= 0 || total_tiles <= 0) return 0;
    if (fp.nl == 1 && !fp.cplx) return launch_cfg<CFG_R1>(d_tasks, ntasks, total_tiles, b, fp, s);
    if (fp.nl == 2 && !fp.cplx) return launch_cfg<CFG_R2>(d_tasks, ntasks, total_tiles, b, fp, s);
    if (fp.nl == 1) return launch_cfg<CFG_C1>(d_tasks, ntasks, total_tiles, b, fp, s);
    return launch_cfg<CFG_C2>(d_tasks, ntasks, total_tiles, b, fp, s);
}

}  // namespace ffa
