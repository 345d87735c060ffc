// Grouped product kernel on INT8 MFMA (gfx950 v_mfma_i32_32x32x32_i8 or
// v_mfma_i32_16x16x64_i8).
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
// Raw operands: when the products read the caller's canonical uint16 residues
// directly (no recursion, two limbs), each 16-byte load brings 8 residues c
// and the limbs are formed between the registers and LDS in offset binary:
// r = c - D with D = 32896 = 128 * 257 has limbs (c >> 8) - 128 and
// (c & 255) - 128, i.e. the two bytes of c with their top bit flipped.  With
// s_i = sum_t c_it (row sums over the padded K, taken on the same loads),
//   sum_t c_it c_jt = sum_t r_it r_jt + D (s_i + s_j) - K D^2,
// exact in the fp64 epilogue.  Columns at or past the valid width enter as c = 0
// (a chunk past them is not read; the part of the row's last chunk past them is
// zeroed after the load).
//
// Data movement: global -> registers (a ring of PF k-tiles in flight) -> LDS
// (double buffer, XOR-swizzled 16-byte segments so that the ds_read_b128 of
// consecutive rows hits distinct banks) -> MFMA.  Configurations with PF = 0
// load global -> LDS directly (buffer loads that write LDS, each thread reading
// the segment that the swizzle puts in its slot): no ring registers, and the
// next k-tile is in flight while the current one is multiplied; PF < 0 does the
// same into -PF buffers with the loads spread between the k-steps.  Which tile a
// workgroup computes comes from a host-built schedule: tiles are grouped into
// L2-friendly blocks and the blocks are dealt to the 8 XCDs (workgroup b runs on
// XCD b mod 8) so that each XCD's L2 serves a compact set of operand panels and
// every XCD gets the same amount of work.  Workgroup b computes entry b, or, in
// a persistent launch, the entries of its XCD taken from a queue counter.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "device_common.h"
#include "ffa_internal.h"
#include "gemm_i8_configs.h"

namespace ffa {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// LDS byte offset of 16-byte segment seg of row r in a tile with KT-byte rows.
// The XOR is its own inverse: the segment stored at physical slot s of row r is
// swz_seg(r, s).
template <int KT>
__device__ __forceinline__ int swz_seg(int r, int seg)
{
    constexpr int NSEG = KT / 16;
    constexpr int RPB = 256 / KT;  // rows per 256-byte bank row
    return seg ^ ((r / RPB) & (NSEG - 1));
}

template <int KT>
__device__ __forceinline__ int swz(int r, int seg)
{
    return r * KT + (swz_seg<KT>(r, seg) << 4);
}

// Canonical residue of an int32 x (|x| < 2^31) for p < 2^8, in full-rate 32-bit
// and 24-bit operations:
//   v = (x >> 16) (2^16 mod p) + (x & 0xffff) + off, off = ceil(2^23 / p) p,
// so 0 <= v < 2^24 is exact in fp32; q = floor(v inv_lo) with inv_lo a little
// below 1/p is the quotient or one less, so r = v - q p lies in [0, 2p) and one
// unsigned minimum finishes.
__device__ __forceinline__ int32_t mod_small_p(int32_t x, int32_t p, int32_t c16, int32_t off, float inv_lo)
{
    // (the mask tells the compiler that the product fits its 24-bit multiplier)
    const int32_t v = (x >> 16) * (c16 & 0xff) + (x & 0xffff) + off;
    const int32_t q = (int32_t)floorf((float)v * inv_lo);
    const uint32_t r = (uint32_t)mad24_s(q, -p, v);
    return (int32_t)min(r, r - (uint32_t)p);
}

// Canonical residue of an int32 x with |x| < 2^22 p (p < 2^8) in six full-rate
// operations: y = x / p is formed in fp32 and rounded to the nearest integer by
// adding 1.5 * 2^23 in the same fused multiply-add (whose result then has an
// ulp of 1).  The computed y is within |y| 2^-23 < 1/2 of x / p, so q differs
// from x / p by less than 1 and r = x - q p lies in (-p, p); one unsigned
// minimum makes it canonical.
__device__ __forceinline__ int32_t mod_fast_p(int32_t x, int32_t p, float inv_p)
{
    constexpr float MAGIC = 12582912.0f;  // 1.5 * 2^23
    const float t = __builtin_fmaf((float)x, inv_p, MAGIC);
    const int32_t q = __float_as_int(t) - __float_as_int(MAGIC);
    const int32_t r = mad24_s(q, -p, x);
    return (int32_t)min((uint32_t)r, (uint32_t)(r + p));
}

// Offset-binary limbs of 8 uint16 values: high limbs into hi (8 bytes), low
// limbs into lo, element e at byte e.
__device__ __forceinline__ void split_u16x8(v4i v, int2& hi, int2& lo)
{
    const uint32_t x0 = (uint32_t)v[0] ^ 0x80808080u, x1 = (uint32_t)v[1] ^ 0x80808080u;
    const uint32_t x2 = (uint32_t)v[2] ^ 0x80808080u, x3 = (uint32_t)v[3] ^ 0x80808080u;
    // v_perm_b32 selects bytes of the pair {second operand: bytes 0..3, first: 4..7}
    hi.x = (int)__builtin_amdgcn_perm(x1, x0, 0x07050301u);
    hi.y = (int)__builtin_amdgcn_perm(x3, x2, 0x07050301u);
    lo.x = (int)__builtin_amdgcn_perm(x1, x0, 0x06040200u);
    lo.y = (int)__builtin_amdgcn_perm(x3, x2, 0x06040200u);
}

// 16 bytes per lane from a buffer straight into LDS: lane l's bytes land at
// dst + 16 l, dst being wave-uniform.  The completion counts as a vector memory
// load (vmcnt).  (A separate function: the address-space cast inside a kernel
// template keeps the host pass from instantiating it.)
__device__ __forceinline__ void lds_load16(__amdgpu_buffer_rsrc_t rs, char* dst, int voff, int soff)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)dst, 16, voff, soff, 0,
                                             0);
}

// One INT8 MFMA of shape MS: 32x32 blocks with 32 bytes of K, or 16x16 blocks
// with 64 bytes of K (16 bytes per lane either way).  A block's result in a lane:
// MS = 32: row lane % 32, columns 8 (v / 4) + 4 (lane / 32) + v % 4 of register v;
// MS = 16: row lane % 16, columns 4 (lane / 16) + v.
template <int MS, typename ACC>
__device__ __forceinline__ ACC mfma_i8(v4i b, v4i a, ACC c)
{
    if constexpr (MS == 32) return __builtin_amdgcn_mfma_i32_32x32x32_i8(b, a, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_i32_16x16x64_i8(b, a, c, 0, 0, 0);
}

// s_waitcnt vmcnt(N) alone (expcnt and lgkmcnt at their maxima: not waited for).
template <int N>
__device__ __forceinline__ void wait_vm()
{
    static_assert(N >= 0 && N < 64, "vmcnt field");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// A workgroup barrier without a memory fence: the waits that it needs are explicit
// (a fence would also wait for the operand loads that are meant to stay in flight).
// Nothing is moved across it, by the compiler or its scheduler.
__device__ __forceinline__ void phase_barrier()
{
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_barrier" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// acc + the sum of the 8 uint16 values of a chunk.
__device__ __forceinline__ uint32_t sum_u16x8(v4i v, uint32_t acc)
{
    const u16x2 one = {1, 1};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        // through a scalar: a bit_cast of the vector element itself read element 0
        const uint32_t w = (uint32_t)v[j];
        acc = __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, w), one, acc, false);
    }
    return acc;
}

// One tile of the grouped product launch: entry e of the schedule.
template <int NL, int CPLX, int BT, int WGM, int WGN, int KT, int PF, int SRC, int MS, int OPT>
__device__ __forceinline__ void gemm_i8_tile(const Bases& bases, const GemmTask* __restrict__ tasks,
                                             const TileEnt* __restrict__ sched, const FieldParams& fp,
                                             char* lds, int e)
{
    constexpr bool RAW = SRC == SRC_RAW_U16;
    static_assert(!RAW || (NL == 2 && !CPLX), "raw uint16 operands feed two limbs of a real field");
    // PF = 0: operands go from global memory straight into LDS (no register ring),
    // two buffers, the next k-tile's loads issued at the start of an iteration.
    // PF < 0: the same loads into -PF buffers, k-tile st - PF - 1 loaded while
    // k-tile st is multiplied, its loads spread over the k-steps.
    constexpr bool DMA = PF <= 0;
    constexpr bool RING = PF < 0;
    constexpr int NBUFS = RING ? -PF : 2;
    constexpr int PFR = DMA ? 1 : PF;
    static_assert(!(DMA && RAW), "raw operands are split into limbs in registers");
    constexpr int NT = WGM * WGN * 64;
    constexpr int NTL = NT;  // threads that load operands
    static_assert(!RING || NBUFS >= 2, "ring: at least two buffers");
    constexpr int NROLE = CPLX ? 2 : 1;
    constexpr int NSEG = CPLX ? 2 : 1;
    constexpr int NA = NROLE * NL;  // A sub-tiles per stage
    constexpr int NB = NL;          // B sub-tiles per stage
    constexpr int WM = BT / WGM, WN = BT / WGN;
    // MFMA shape: MS = 32 (v_mfma_i32_32x32x32_i8, a k-step of 32 bytes) or 16
    // (v_mfma_i32_16x16x64_i8, a k-step of 64 bytes); FM x FN blocks of MS x MS per wave
    static_assert(MS == 32 || MS == 16, "MFMA shape");
    constexpr int FM = WM / MS, FN = WN / MS;
    constexpr int NREG = MS == 32 ? 16 : 4;  // accumulator registers per block
    constexpr int SPK = 64 / MS;             // 16-byte segments of a row per k-step
    static_assert(KT % (16 * SPK) == 0, "k-tile of whole k-steps");
    constexpr int NACC = NL == 1 ? 1 : 3;
    constexpr int TILE = BT * KT;
    constexpr int STAGE = (NA + NB) * TILE;
    constexpr int SPR = KT / 16;  // 16-byte segments per carrier row
    constexpr int RPR = KT / 8;   // 16-byte raw chunks (8 residues) per row
    constexpr int ACH = NA * TILE / 16 / NTL;
    constexpr int BCH = NB * TILE / 16 / NTL;
    static_assert(NA * TILE % (16 * NTL) == 0 && NB * TILE % (16 * NTL) == 0, "chunking");
    static_assert(FM >= 1 && FN >= 1, "wave tile");

    const TileEnt ent = sched[e];
    if (ent.x < 0) return;  // padding entry of the XCD-balanced schedule
    const GemmTask& T = tasks[ent.x];
    if (T.wait > 0) {
        // operands produced beside this launch: wait until they are all written
        if (threadIdx.x == 0)
            wait_counter(bases.p[BUF_WS] + T.wait_off, T.wait, reinterpret_cast<int32_t*>(bases.p[BUF_ERR]) + 1);
        __syncthreads();
    }
    const int row0 = (ent.y & 0xffff) * BT, col0 = (ent.y >> 16) * BT;
    const int M = T.M, N = T.N, K = T.K;
    // (the thread index passes through an empty asm statement so that the compiler
    // does not hoist the per-thread offsets derived from it out of a persistent
    // launch's loop over tiles, where they would stay live and spill)
    // (the mask gives the compiler the index's range back: LDS addresses derived from
    // it are then known to be non-negative, so that constant parts of them go into
    // the instructions' offset fields instead of registers; option bit 5 leaves it
    // out for the configurations whose allocation grows with it)
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    if (!(OPT & 32)) tid &= NT - 1;
    const int lane = tid & 63, wave = tid >> 6;
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
    int acol[RAW ? ACH : 1], bcol[RAW ? BCH : 1];  // raw: first column of the chunk in a k-tile
    uint32_t asum[RAW ? ACH : 1], bsum[RAW ? BCH : 1];  // raw: partial row sums of the chunks
#pragma unroll
    for (int i = 0; i < (RAW ? ACH : 1); ++i) asum[i] = 0;
#pragma unroll
    for (int i = 0; i < (RAW ? BCH : 1); ++i) bsum[i] = 0;
#pragma unroll
    for (int i = 0; i < ACH; ++i) {
        const int c = tid + i * NTL;
        if (RAW) {
            // (row, chunk) -> hi limb at sub-tile 0, lo limb at sub-tile 1, 8 bytes each
            const int r = c / RPR, s = c % RPR;
            aoff[i] = min(r, rows_a - 1) * T.x.ld + s * 16;
            alds[i] = swz<KT>(r, s >> 1) + (s & 1) * 8;
            acol[i] = s * 8;
        } else {
            const int sub = c / (BT * SPR), r = (c / SPR) % BT, s = c % SPR;
            // direct loads put lane l's 16 bytes at LDS slot c: that thread reads the
            // segment which the swizzle places there
            const int gs = DMA ? swz_seg<KT>(r, s) : s;
            aoff[i] = (int)(sub * T.x.ps + (int64_t)min(r, rows_a - 1) * T.x.ld) + gs * 16;
            alds[i] = sub * TILE + swz<KT>(r, s);
        }
    }
#pragma unroll
    for (int i = 0; i < BCH; ++i) {
        const int c = tid + i * NTL;
        if (RAW) {
            const int r = c / RPR, s = c % RPR;
            boff[i] = min(r, rows_b - 1) * T.z.ld + s * 16;
            blds[i] = NA * TILE + swz<KT>(r, s >> 1) + (s & 1) * 8;
            bcol[i] = s * 8;
        } else {
            const int sub = c / (BT * SPR), r = (c / SPR) % BT, s = c % SPR;
            const int gs = DMA ? swz_seg<KT>(r, s) : s;
            boff[i] = (int)(sub * T.z.ps + (int64_t)min(r, rows_b - 1) * T.z.ld) + gs * 16;
            blds[i] = (NA + sub) * TILE + swz<KT>(r, s);
        }
    }
    // Complex: A sub-tile index sub = role * NL + limb reads plane role (segment 0) and
    // plane role + 1 (segment 1); B reads plane 0 then plane 1.
    const int nkc = K / KT;
    const int nst = NSEG * nkc;
    const int seg_a = (int)(NL * T.x.ps), seg_b = (int)(NL * T.z.ps);

    v4i ra[PFR][ACH], rb[PFR][BCH];
    const int kvalid = T.kvalid;
    // Register-ring loads are issued without branches (the same instructions for every
    // stage, so that each wait covers only the stage it needs): a load that has nothing
    // to read (a stage past the last, a raw chunk past the valid columns) gets an offset
    // past the resource's extent, which the buffer range check turns into zeros
    // without a memory access.
    constexpr int OOR = (int)0x80000000u;
    auto gload = [&](int st, v4i* a, v4i* b) {
        if (RAW) {
            // a chunk that holds valid columns is read whole (16-byte aligned rows: it
            // stays in its row); sstore zeroes the columns past the valid ones
            const int kb = st * KT;
#pragma unroll
            for (int i = 0; i < ACH; ++i)
                a[i] = __builtin_amdgcn_raw_buffer_load_b128(rsa, kvalid - kb - acol[i] > 0 ? aoff[i] + 2 * kb : OOR, 0, 0);
#pragma unroll
            for (int i = 0; i < BCH; ++i)
                b[i] = __builtin_amdgcn_raw_buffer_load_b128(rsb, kvalid - kb - bcol[i] > 0 ? boff[i] + 2 * kb : OOR, 0, 0);
            return;
        }
        const int seg = st >= nkc ? 1 : 0;
        const int kc = st - seg * nkc;
        const int oa = seg * seg_a + kc * KT, ob = seg * seg_b + kc * KT;
        if (DMA) {
            // chunk c = tid + i * NTL lands at LDS byte 16 c of the stage: the wave's 64
            // lanes fill 1 KiB from the wave-uniform base given here
            char* base = lds + (st % NBUFS) * STAGE + wave * 1024;
#pragma unroll
            for (int i = 0; i < ACH; ++i) lds_load16(rsa, base + i * NTL * 16, aoff[i], oa);
#pragma unroll
            for (int i = 0; i < BCH; ++i) lds_load16(rsb, base + NA * TILE + i * NTL * 16, boff[i], ob);
            return;
        }
        const bool live = st < nst;
#pragma unroll
        for (int i = 0; i < ACH; ++i) a[i] = __builtin_amdgcn_raw_buffer_load_b128(rsa, live ? aoff[i] : OOR, live ? oa : 0, 0);
#pragma unroll
        for (int i = 0; i < BCH; ++i) b[i] = __builtin_amdgcn_raw_buffer_load_b128(rsb, live ? boff[i] : OOR, live ? ob : 0, 0);
    };
    // one direct load of stage st: chunk q of A (q < ACH) or q - ACH of B
    auto gload_one = [&](int st, int q) {
        const int seg = st >= nkc ? 1 : 0;
        const int kc = st - seg * nkc;
        char* base = lds + (st % NBUFS) * STAGE + wave * 1024;
        if (q < ACH) lds_load16(rsa, base + q * NTL * 16, aoff[q], seg * seg_a + kc * KT);
        else lds_load16(rsb, base + NA * TILE + (q - ACH) * NTL * 16, boff[q - ACH], seg * seg_b + kc * KT);
    };
    // raw chunk of 8 uint16 columns with lim valid ones: the others zeroed
    auto keep_valid = [&](v4i v, int lim) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t m = lim >= 2 * j + 2 ? 0xffffffffu : (lim == 2 * j + 1 ? 0x0000ffffu : 0u);
            v[j] = (int)((uint32_t)v[j] & m);
        }
        return v;
    };
    auto sstore = [&](int buf, int st, const v4i* a, const v4i* b) {
        char* base = lds + buf * STAGE;
        if (RAW) {
            // the stage holds columns past the valid ones when it reaches kvalid
            const int kb = st * KT;
            const bool edge = kb + KT > kvalid;
#pragma unroll
            for (int i = 0; i < ACH; ++i) {
                int2 hi, lo;
                const v4i av = edge ? keep_valid(a[i], kvalid - kb - acol[i]) : a[i];
                split_u16x8(av, hi, lo);
                asum[i] = sum_u16x8(av, asum[i]);
                *reinterpret_cast<int2*>(base + alds[i]) = hi;
                *reinterpret_cast<int2*>(base + alds[i] + TILE) = lo;
            }
#pragma unroll
            for (int i = 0; i < BCH; ++i) {
                int2 hi, lo;
                const v4i bv = edge ? keep_valid(b[i], kvalid - kb - bcol[i]) : b[i];
                split_u16x8(bv, hi, lo);
                bsum[i] = sum_u16x8(bv, bsum[i]);
                *reinterpret_cast<int2*>(base + blds[i]) = hi;
                *reinterpret_cast<int2*>(base + blds[i] + TILE) = lo;
            }
            return;
        }
#pragma unroll
        for (int i = 0; i < ACH; ++i) *reinterpret_cast<v4i*>(base + alds[i]) = a[i];
#pragma unroll
        for (int i = 0; i < BCH; ++i) *reinterpret_cast<v4i*>(base + blds[i]) = b[i];
    };

    using acc_t = std::conditional_t<MS == 32, v16i, v4i>;
    acc_t acc[NROLE][NACC][FM][FN];
#pragma unroll
    for (int r = 0; r < NROLE; ++r)
#pragma unroll
        for (int a = 0; a < NACC; ++a)
#pragma unroll
            for (int m = 0; m < FM; ++m)
#pragma unroll
                for (int n = 0; n < FN; ++n)
#pragma unroll
                    for (int v = 0; v < NREG; ++v) acc[r][a][m][n][v] = 0;

    // lane -> row lane % MS of a block, 16-byte segment lane / MS of the k-step
    const int lrow = lane % MS, lseg = lane / MS;
    // fragment reads of k-step ks (16 SPK bytes of K) from an LDS stage
    auto load_frags = [&](const char* base, int ks, v4i (*af)[FM], v4i (*bf)[FN]) {
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
            for (int m = 0; m < FM; ++m)
                af[a][m] = *reinterpret_cast<const v4i*>(
                    base + a * TILE + swz<KT>(wm0 + m * MS + lrow, ks * SPK + lseg));
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int n = 0; n < FN; ++n)
                bf[b][n] = *reinterpret_cast<const v4i*>(
                    base + (NA + b) * TILE + swz<KT>(wn0 + n * MS + lrow, ks * SPK + lseg));
    };
    auto mfmas = [&](v4i (*af)[FM], v4i (*bf)[FN]) {
        if (NL == 1) {
#pragma unroll
            for (int r = 0; r < NROLE; ++r)
#pragma unroll
                for (int m = 0; m < FM; ++m)
#pragma unroll
                    for (int n = 0; n < FN; ++n)
                        acc[r][0][m][n] = mfma_i8<MS>(bf[0][n], af[r][m], acc[r][0][m][n]);
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
                            acc[r][ai][m][n] = mfma_i8<MS>(bf[lb][n], af[r * NL + la][m], acc[r][ai][m][n]);
            }
        }
    };
    // the fragments of k-step ks + 1 are read while the MFMAs of k-step ks run;
    // hook(ks) runs after the MFMAs of k-step ks are issued
    constexpr int NKS = KT / (16 * SPK);
    // option bit 4: the last k-step's MFMAs after the k-tile's barrier (direct loads,
    // an even number of k-steps, so that they and the next k-tile's first fragments
    // use different halves of the fragment double buffer)
    constexpr bool DEFER = (OPT & 16) != 0;
    static_assert(!DEFER || (DMA && !RING && NKS % 2 == 0), "deferred MFMAs: direct loads, even k-steps");
    // Where stage st + 1 is written to LDS: before compute(st) when it was loaded at
    // least one iteration earlier (PF >= 2), else halfway through compute(st) (its
    // loads are issued at the start of the iteration).  Measured against writing it
    // after compute(st): 1.86 vs 1.93 ms (one limb, 256-tiles, PF = 2) and 7.11 vs
    // 7.26 ms (two limbs, PF = 1) for the products at n = k = 16384.
    constexpr int SPOS = PF >= 2 ? 2 : 1;
    constexpr int HK = SPOS == 1 && !DMA ? (NKS >= 2 ? NKS / 2 - 1 : 0) : -1;
    // The compiler's MFMA / LDS-read interleaving strategy 0 for the two-limb products
    // read from carrier planes through registers (6.40 vs 6.82 ms of products at
    // n = k = 16384).  One limb (its 128 accumulator registers) and raw operands
    // would spill with it; with direct loads it made the one-limb kernel slower
    // (1.82 vs 1.75 ms) and changed nothing with two limbs.
    constexpr bool IGLP = NL == 2 && !RAW && !DMA;
    auto compute = [&](int buf, auto hook) {
        const char* base = lds + buf * STAGE;
        v4i af[2][NA][FM], bf[2][NB][FN];
        load_frags(base, 0, af[0], bf[0]);
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
            if (ks + 1 < NKS) load_frags(base, ks + 1, af[(ks + 1) & 1], bf[(ks + 1) & 1]);
            mfmas(af[ks & 1], bf[ks & 1]);
            hook(ks);
        }
        if (IGLP) __builtin_amdgcn_iglp_opt(0);
    };

    // ---- pipeline: PF k-tiles in flight in registers, two LDS buffers.  Stage
    // st + 1 goes to the buffer that compute(st - 1) read, which the barrier ending
    // iteration st - 1 released, so it may be written while compute(st) runs.
    // Direct loads: stage st + 1 is loaded into that buffer while compute(st) runs;
    // the barrier ending iteration st waits for the loads (vmcnt) before any wave
    // reads the stage.
    if (RING) {
        // k-tiles 0 .. NBUFS - 2 are loaded before the loop; during iteration st the
        // loads of k-tile st + NBUFS - 1 (into the buffer of k-tile st - 1, released by
        // the barrier that ended iteration st - 1) follow the MFMAs of the k-steps, a
        // few after each; the iteration ends with a wait for k-tile st + 1 (the loads
        // issued after it stay in flight) and a barrier.
        constexpr int LPB = ACH + BCH;
        // with two buffers the loads issued in an iteration are waited for at its end:
        // they follow the first half of the k-steps only
        constexpr int NKW = NBUFS == 2 ? (NKS + 1) / 2 : NKS;
        constexpr int LPK = (LPB + NKW - 1) / NKW;  // loads after each of the first NKW k-steps
        for (int u = 0; u < min(NBUFS - 1, nst); ++u) gload(u, ra[0], rb[0]);
        if (nst - 1 >= NBUFS - 2) wait_vm<LPB * (NBUFS - 2)>();
        else wait_vm<0>();
        phase_barrier();
        for (int st = 0; st < nst; ++st) {
            const int ld = st + NBUFS - 1;
            compute(st % NBUFS, [&](int ks) {
                if (ld < nst) {
#pragma unroll
                    for (int q = ks * LPK; q < min(LPB, (ks + 1) * LPK); ++q) gload_one(ld, q);  // none past NKW
                }
            });
            if (st + 1 < nst) {
                if (nst - 2 - st >= NBUFS - 2) wait_vm<LPB * (NBUFS - 2)>();
                else wait_vm<0>();
            }
            phase_barrier();
        }
    } else if (DMA && DEFER) {
        // The MFMAs of each k-tile's last k-step (their fragments already in registers)
        // are issued after the barrier that ends the k-tile, while the next k-tile's
        // first fragments are read: the two waves of a SIMD leave the barrier together,
        // and without this both would wait for those reads before their next MFMA.
        // The loads of k-tile st + 2 are issued right after that barrier (their buffer's
        // last reads are behind it), ahead of the deferred MFMAs.
        v4i af[2][NA][FM], bf[2][NB][FN];
        if (nst > 0) gload(0, ra[0], rb[0]);
        wait_vm<0>();
        __syncthreads();
        if (nst > 1) gload(1, ra[0], rb[0]);
        if (nst > 0) load_frags(lds, 0, af[0], bf[0]);
        for (int st = 0; st < nst; ++st) {
            const char* base = lds + (st & 1) * STAGE;
#pragma unroll
            for (int ks = 0; ks < NKS - 1; ++ks) {
                load_frags(base, ks + 1, af[(ks + 1) & 1], bf[(ks + 1) & 1]);
                mfmas(af[ks & 1], bf[ks & 1]);
            }
            wait_vm<0>();  // k-tile st + 1 is in LDS
            __syncthreads();
            __builtin_amdgcn_sched_barrier(0);
            if (st + 2 < nst) gload(st + 2, ra[0], rb[0]);
            if (st + 1 < nst) load_frags(lds + ((st + 1) & 1) * STAGE, 0, af[0], bf[0]);
            mfmas(af[(NKS - 1) & 1], bf[(NKS - 1) & 1]);
            __builtin_amdgcn_sched_barrier(0);
        }
    } else if (DMA) {
        // (the waits for the direct loads are explicit: the barrier's fence need not
        // cover loads that write LDS)
        if (nst > 0) gload(0, ra[0], rb[0]);
        wait_vm<0>();
        __syncthreads();
        for (int st = 0; st < nst; ++st) {
            if (st + 1 < nst) gload(st + 1, ra[0], rb[0]);
            compute(st & 1, [](int) {});
            wait_vm<0>();
            __syncthreads();
        }
    }
    if (!DMA) {
        // register slot u holds stage st with st % PF == u.  The main loop runs whole
        // groups of PF stages, each refilling its slot with the stage PF ahead (nothing
        // past the last stage is read); the stages left over follow without loads.
#pragma unroll
        for (int u = 0; u < PFR; ++u) gload(u, ra[u], rb[u]);
        if (nst > 0) sstore(0, 0, ra[0], rb[0]);
        __syncthreads();
        auto step = [&](int st, int u, bool refill) __attribute__((always_inline)) {
            auto next = [&] {
                if (st + 1 < nst) sstore((st + 1) & 1, st + 1, ra[(u + 1) % PFR], rb[(u + 1) % PFR]);
            };
            if (SPOS == 2) next();
            if (refill) gload(st + PFR, ra[u], rb[u]);
            compute(st & 1, [&](int ks) {
                if (ks == HK) next();
            });
            __syncthreads();
        };
        int st0 = 0;
        for (; st0 + PFR <= nst; st0 += PFR) {
#pragma unroll
            for (int u = 0; u < PFR; ++u) step(st0 + u, u, true);
        }
#pragma unroll
        for (int u = 0; u < PFR - 1; ++u)
            if (st0 + u < nst) step(st0 + u, u, false);
    }

    // ---- raw operands: row sums of the tile's A rows and B rows into LDS (the
    // stage buffers are free after the last barrier of the loop).  The RPR
    // consecutive threads that loaded one row's chunks reduce across lanes.
    constexpr int RSUM_BYTES = RAW ? 2 * BT * 4 : 0;  // at the end of LDS, clear of the staging below
    const uint32_t* rsum_a = reinterpret_cast<const uint32_t*>(lds + NBUFS * STAGE - RSUM_BYTES);
    const uint32_t* rsum_b = rsum_a + BT;
    if (RAW) {
        static_assert(RPR <= 64 && NT % RPR == 0, "row chunks within a wave");
        uint32_t* rs = reinterpret_cast<uint32_t*>(lds + NBUFS * STAGE - RSUM_BYTES);
#pragma unroll
        for (int i = 0; i < ACH; ++i) {
            uint32_t v = asum[i];
#pragma unroll
            for (int o = RPR / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o);
            const int c = tid + i * NT;
            if (c % RPR == 0) rs[c / RPR] = v;
        }
#pragma unroll
        for (int i = 0; i < BCH; ++i) {
            uint32_t v = bsum[i];
#pragma unroll
            for (int o = RPR / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o);
            const int c = tid + i * NT;
            if (c % RPR == 0) rs[BT + c / RPR] = v;
        }
        __syncthreads();
    }
    constexpr double RAW_D = 32896.0;
    const double raw_kdd = RAW_D * RAW_D * (double)K;

    // ---- epilogue: exact recombination, reduction mod p, store.
    // The MFMAs take (B fragment, A fragment), so a 32x32 accumulator holds its
    // block transposed: lane -> row (lane & 31), register v -> column
    // 8 (v / 4) + 4 (lane / 32) + v % 4; four consecutive registers are four
    // consecutive columns of one row of C.
    const int p = fp.p;
    const int32_t c16 = (int32_t)(65536 % p);
    const int32_t moff = ((1 << 23) / p + 1) * p;                 // makes v non-negative
    const float inv_lo = (float)(fp.inv_p * (1.0 - 1.0 / 4194304.0));  // below 1/p
    const bool syrk = T.syrk != 0;
    const int ldc = T.c.ld;
    const int rows_c = min(BT, M - row0), cols_c = min(BT, N - col0);
    // one limb: the six-operation reduction where every accumulator stays below
    // 2^22 p in magnitude (K ((p-1)/2)^2 below it: the planner's products up to
    // K = 67000 at p = 251), else the exact 24-bit folding
    const bool fast = NL == 1 && (int64_t)K * fp.half * fp.half < ((int64_t)p << 22);
    // tile row and column of accumulator register v of block (m, n) in this lane
    auto row_of = [&](int m) { return wm0 + m * MS + lane % MS; };
    auto col_of = [&](int n, int v) {
        return MS == 32 ? wn0 + n * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3) : wn0 + n * 16 + 4 * (lane >> 4) + v;
    };
    const float inv_p32 = (float)fp.inv_p;
    auto residue_in = [&](auto fast_tag, int r, int m, int n, int v) __attribute__((always_inline)) -> int32_t {
        if (NL == 1) {
            if (decltype(fast_tag)::value) return mod_fast_p(acc[r][0][m][n][v], p, inv_p32);
            return mod_small_p(acc[r][0][m][n][v], p, c16, moff, inv_lo);
        }
        double val = 65536.0 * (double)acc[r][0][m][n][v] + 256.0 * (double)acc[r][NACC - 2][m][n][v] +
                     (double)acc[r][NACC - 1][m][n][v];
        if (RAW) {
            const int li = row_of(m);
            const int lj = col_of(n, v);
            val += RAW_D * ((double)rsum_a[li] + (double)rsum_b[lj]) - raw_kdd;
        }
        return mod_canon(val, p, fp.inv_p);
    };
    // Staged store: the tile's residues go to LDS in the output format (rows of
    // BT elements, 16-byte segments XOR-swizzled by row), then every thread
    // writes whole 16-byte segments of C rows.  Segments that cross the matrix
    // edge or the diagonal of a base case are written element by element.  Needs
    // a 16-byte aligned tile origin and row stride, and 32-bit tile offsets.
    auto epilogue = [&](auto tag, auto fast_tag) __attribute__((always_inline)) {
        using OT = decltype(tag);
        auto residue = [&](int r, int m, int n, int v) __attribute__((always_inline)) {
            return residue_in(fast_tag, r, m, n, v);
        };
        constexpr int ES = (int)sizeof(OT);
        constexpr int RB = BT * ES;   // bytes per staged row
        constexpr int NSR = RB / 16;  // segments per row
        constexpr int EPS = 16 / ES;  // elements per segment
        constexpr bool CAN_STAGE = BT * RB <= NBUFS * STAGE - RSUM_BYTES;
#pragma unroll
        for (int r = 0; r < NROLE; ++r) {
            char* cb = (r == 0 ? bases.p[T.c.buf] + T.c.off : bases.p[T.c.buf2] + T.c.off2) +
                       ((int64_t)row0 * ldc + col0) * ES;
            const bool staged = CAN_STAGE && ((((uintptr_t)cb) | (uintptr_t)(ldc * ES)) & 15) == 0 &&
                                (int64_t)BT * ldc * ES < (1ll << 31);
            if (staged) {
                if (r > 0) __syncthreads();  // the previous role's reads of LDS are done
#pragma unroll
                for (int m = 0; m < FM; ++m)
#pragma unroll
                    for (int n = 0; n < FN; ++n)
#pragma unroll
                        for (int q = 0; q < NREG / 4; ++q) {
                            OT vals[4];
#pragma unroll
                            for (int e = 0; e < 4; ++e) vals[e] = (OT)residue(r, m, n, 4 * q + e);
                            const int li = row_of(m);
                            const int byte = col_of(n, 4 * q) * ES;
#pragma unroll
                            for (int h = 0; h < (4 * ES + 15) / 16; ++h) {
                                // 4 * ES bytes: part of one segment, or whole segments (ES = 8)
                                const int bb = byte + 16 * h;
                                char* dst = lds + li * RB + (((bb >> 4) ^ (li & (NSR - 1))) << 4) + (bb & 15);
                                if (ES == 1) *reinterpret_cast<uint32_t*>(dst) = *reinterpret_cast<const uint32_t*>(vals);
                                else if (ES == 2) *reinterpret_cast<uint2*>(dst) = *reinterpret_cast<const uint2*>(vals);
                                else *reinterpret_cast<int4*>(dst) = reinterpret_cast<const int4*>(vals)[h];
                            }
                            if (q == NREG / 4 - 1) __builtin_amdgcn_sched_barrier(0);
                        }
                __syncthreads();
                const int ext = (int)((int64_t)(rows_c - 1) * ldc * ES + (int64_t)cols_c * ES);
                const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc((void*)cb, (short)0, ext, 0x00020000);
                constexpr int NCH = BT * NSR;
                static_assert(NCH % NT == 0, "store chunks");
#pragma unroll
                for (int it = 0; it < NCH / NT; ++it) {
                    const int c = tid + it * NT;
                    const int rr = c / NSR, sg = c % NSR;
                    if (rr >= rows_c) continue;
                    const v4i val = *reinterpret_cast<const v4i*>(lds + rr * RB + ((sg ^ (rr & (NSR - 1))) << 4));
                    const int off = rr * ldc * ES + sg * 16;
                    // valid columns of the segment: inside the matrix, and on or below the diagonal
                    int nv = cols_c - sg * EPS;
                    if (syrk) nv = min(nv, row0 + rr - (col0 + sg * EPS) + 1);
                    if (nv >= EPS) {
                        __builtin_amdgcn_raw_buffer_store_b128(val, rc, off, 0, 0);
                    } else if (nv > 0) {
                        const OT* el = reinterpret_cast<const OT*>(&val);
#pragma unroll
                        for (int e = 0; e < EPS; ++e)
                            if (e < nv) *reinterpret_cast<OT*>(cb + off + e * ES) = el[e];
                    }
                }
            } else {
                OT* cp = reinterpret_cast<OT*>(cb);
#pragma unroll
                for (int m = 0; m < FM; ++m)
#pragma unroll
                    for (int n = 0; n < FN; ++n)
#pragma unroll
                        for (int v = 0; v < NREG; ++v) {
                            const int li = row_of(m);
                            const int lj = col_of(n, v);
                            const int32_t res = residue(r, m, n, v);
                            if (li < rows_c && lj < cols_c && (!syrk || row0 + li >= col0 + lj))
                                cp[(int64_t)li * ldc + lj] = (OT)res;
                            if ((v & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                        }
            }
        }
    };
    // (the faster reduction only for byte residues, the format of every product of a
    // one-limb recursion, so that the epilogue exists once more, not five times)
    if (fast && T.c.dt == DT_U8) {
        epilogue(uint8_t{}, std::true_type{});
        return;
    }
    switch (T.c.dt) {
    case DT_U8: epilogue(uint8_t{}, std::false_type{}); break;
    case DT_U16: epilogue(uint16_t{}, std::false_type{}); break;
    case DT_I32: epilogue(int32_t{}, std::false_type{}); break;
    case DT_I64: epilogue(int64_t{}, std::false_type{}); break;
    case DT_F64: epilogue(double{}, std::false_type{}); break;
    default: break;
    }
}

// The grouped product launch.  fp.nent == 0: workgroup b computes schedule entry b.
// fp.nent > 0 (persistent): a grid of at most the resident workgroups; workgroup b
// takes the entries of its XCD (x = b mod 8; entries x, x + 8, ... were dealt to it by
// the host) in order from that XCD's queue counter in the workspace (zeroed before
// the launch), grabbing the next one while it computes the current one, until the
// queue passes fp.nent.  Every workgroup ends once its queue is drained.
template <int NL, int CPLX, int BT, int WGM, int WGN, int KT, int PF, int SRC, int MS, int OPT>
__global__ void __launch_bounds__(WGM* WGN * 64, (OPT & 15) > 0 ? (OPT & 15) : 1)
    gemm_i8(Bases bases, const GemmTask* __restrict__ tasks, const TileEnt* __restrict__ sched,
            FieldParams fp)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    __shared__ int s_next;
    const bool persist = fp.nent > 0;
    const int x = blockIdx.x & 7;
    int* q = persist ? reinterpret_cast<int*>(bases.p[BUF_WS] + fp.queue_off) + x : nullptr;
    int e = blockIdx.x;
    if (persist) {
        if (threadIdx.x == 0) s_next = atomicAdd(q, 1) * 8 + x;
        __syncthreads();
        e = s_next;
    }
    const int nent = persist ? fp.nent : (int)gridDim.x;
    while (e < nent) {
        int nx = 0;
        if (persist && threadIdx.x == 0) nx = atomicAdd(q, 1) * 8 + x;
        gemm_i8_tile<NL, CPLX, BT, WGM, WGN, KT, PF, SRC, MS, OPT>(bases, tasks, sched, fp, lds, e);
        if (!persist) break;
        __syncthreads();  // the tile's last reads of LDS are done
        if (threadIdx.x == 0) s_next = nx;
        __syncthreads();
        e = s_next;
    }
}

template <int NL, int CPLX, int BT, int WGM, int WGN, int KT, int PF, int SRC, int MS, int OPT>
static int launch_cfg(const GemmTask* d_tasks, const TileEnt* d_sched, int nblocks, const Bases& b,
                      const FieldParams& fp, hipStream_t s)
{
    constexpr int NA = (CPLX ? 2 : 1) * NL, NB = NL;
    constexpr int lds_bytes = (PF < 0 ? -PF : 2) * (NA + NB) * BT * KT;
    auto kern = gemm_i8<NL, CPLX, BT, WGM, WGN, KT, PF, SRC, MS, OPT>;
    // the LDS limit is raised once per device the kernel runs on
    static uint64_t attr_devices = 0;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    const uint64_t bit = 1ull << (dev & 63);
    if (!(attr_devices & bit)) {
        e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) return (int)e;
        attr_devices |= bit;
    }
    int grid = nblocks;
    if (fp.nent > 0) {
        // persistent: at most the workgroups that fit the device at once, a multiple of 8
        static int resident[64] = {0};
        int& r = resident[dev & 63];
        if (r == 0) {
            int per_cu = 0, cus = 0;
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, WGM * WGN * 64, lds_bytes);
            if (e != hipSuccess) return (int)e;
            e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            if (e != hipSuccess) return (int)e;
            r = std::max(8, std::max(per_cu, 1) * cus / 8 * 8);
        }
        grid = std::min(grid, r);
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(WGM * WGN * 64), lds_bytes, s, b, d_tasks,
                       d_sched, fp);
    return (int)hipGetLastError();
}

// Raw uint16 operands exist only for the two-limb real configurations that load
// through registers.
template <int NL, int CPLX, int BT, int WGM, int WGN, int KT, int PF, int MS, int OPT>
static int launch_src(int src, const GemmTask* d_tasks, const TileEnt* d_sched, int nblocks,
                      const Bases& b, const FieldParams& fp, hipStream_t s)
{
    if (src == SRC_CARRIER)
        return launch_cfg<NL, CPLX, BT, WGM, WGN, KT, PF, SRC_CARRIER, MS, OPT>(d_tasks, d_sched, nblocks, b, fp, s);
    if constexpr (NL == 2 && CPLX == 0 && PF > 0) {
        if (src == SRC_RAW_U16)
            return launch_cfg<NL, CPLX, BT, WGM, WGN, KT, PF, SRC_RAW_U16, MS, OPT>(d_tasks, d_sched, nblocks, b, fp, s);
    }
    return (int)hipErrorInvalidValue;
}

// The entry points of one translation unit that instantiates the kernel for the
// configurations of LIST (the kernel is instantiated in several units, compiled in
// parallel); both return FFA_I8_NOT_HERE for a configuration the unit does not hold.

#define FFA_I8_PART(PART, LIST)                                                                        \
    int gemm_i8_launch_##PART(int cfg, int src, const GemmTask* d_tasks, const TileEnt* d_sched,      \
                              int nblocks, const Bases& b, const FieldParams& fp, hipStream_t s)       \
    {                                                                                                  \
        LIST(FFA_I8_PART_LAUNCH)                                                                       \
        (void)src; (void)d_tasks; (void)d_sched; (void)nblocks; (void)b; (void)fp; (void)s;            \
        return FFA_I8_NOT_HERE;                                                                        \
    }                                                                                                  \
    int gemm_i8_regs_##PART(int cfg, int* vgprs)                                                       \
    {                                                                                                  \
        LIST(FFA_I8_PART_REGS)                                                                         \
        (void)vgprs;                                                                                   \
        return FFA_I8_NOT_HERE;                                                                        \
    }

#define FFA_I8_PART_LAUNCH(ID, NL, CP, BT, WM, WN, KT, PF, MS, OPT) \
    if (cfg == ID) return launch_src<NL, CP, BT, WM, WN, KT, PF, MS, OPT>(src, d_tasks, d_sched, nblocks, b, fp, s);

#define FFA_I8_PART_REGS(ID, NL, CP, BT, WM, WN, KT, PF, MS, OPT)                                   \
    if (cfg == ID) {                                                                                \
        hipFuncAttributes a{};                                                                      \
        const hipError_t e =                                                                        \
            hipFuncGetAttributes(&a, (const void*)gemm_i8<NL, CP, BT, WM, WN, KT, PF, SRC_CARRIER, MS, OPT>); \
        if (e != hipSuccess) return (int)e;                                                         \
        *vgprs = a.numRegs;                                                                         \
        return 0;                                                                                   \
    }

}  // namespace ffa
