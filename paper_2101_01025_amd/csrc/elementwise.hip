// HBM-bound kernels of the recursion (Algorithm 1, Section 3):
//   * conditioning: caller's residues -> carrier planes (zero padded);
//   * pre-additions: S1 = (A21 - A11) Y, S2 = A22 - A21 Y, S3 = S1 - A22,
//     S4 = S3 + A12, fused in one pass per recursion level;
//   * post-additions: U1 = P1 + P5, U3 = P1 + P2, Up(U1) = phi(Low(U1)),
//     U2 = U1 + P4, U4 = U2 + P3, U5 = Low(U2) + Low(phi(P4)), fused in one
//     pass per recursion level, transposed reads staged through LDS.
// Every value is reduced mod p where it is produced.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.h"
#include "ffa_internal.h"

namespace ffa {

// ============================================================================
// conditioning
// ============================================================================

__device__ __forceinline__ bool read_input(const char* base, int dt, int64_t idx, int32_t p,
                                           int32_t half, int32_t& v)
{
    switch (dt) {
    case DT_I8C: {
        int32_t x = reinterpret_cast<const int8_t*>(base)[idx];
        v = x < 0 ? x + p : x;
        return x >= -half && x <= half;
    }
    case DT_U8: v = reinterpret_cast<const uint8_t*>(base)[idx]; return v < p;
    case DT_U16: v = reinterpret_cast<const uint16_t*>(base)[idx]; return v < p;
    case DT_I32: v = reinterpret_cast<const int32_t*>(base)[idx]; return v >= 0 && v < p;
    case DT_I64: {
        int64_t x = reinterpret_cast<const int64_t*>(base)[idx];
        v = (int32_t)x;
        return x >= 0 && x < p;
    }
    case DT_F64: {
        double x = reinterpret_cast<const double*>(base)[idx];
        v = (int32_t)x;
        return x >= 0.0 && x < (double)p && (double)v == x;
    }
    }
    v = 0;
    return false;
}

// One thread converts VEC consecutive columns of one row.
template <int NL, int CPLX>
__global__ void __launch_bounds__(256) condition_i8(const CondTask* tasks, Bases b, FieldParams fp,
                                                    int32_t* err)
{
    constexpr int VEC = 16;
    const CondTask& t = tasks[blockIdx.y];
    const int gpr = t.kpad / VEC;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)t.npad * gpr) return;
    const int r = (int)(idx / gpr), c0 = (int)(idx % gpr) * VEC;
    const int p = fp.p;
    constexpr int NPL = CPLX ? 3 : 1;
    alignas(16) int8_t out[NPL][NL][VEC];
    bool bad = false;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        const int c = c0 + e;
        int32_t vr = 0, vi = 0;
        if (r < t.n && c < t.k) {
            const int64_t off = (int64_t)r * t.lda + c;
            bad |= !read_input(b.p[t.buf_re] + t.off_re, t.dt_in, off, p, fp.half, vr);
            if (CPLX) bad |= !read_input(b.p[t.buf_im] + t.off_im, t.dt_in, off, p, fp.half, vi);
        }
        int32_t vals[3] = {vr, vi, neg_mod(vr, p)};
#pragma unroll
        for (int q = 0; q < NPL; ++q) {
            if (NL == 1) {
                out[q][0][e] = (int8_t)(vals[q] > fp.half ? vals[q] - p : vals[q]);
            } else {
                int8_t hi, lo;
                split2(rep2(vals[q], p), hi, lo);
                out[q][0][e] = hi;
                out[q][NL - 1][e] = lo;
            }
        }
    }
    if (bad) err[0] = 1;
    char* ob = b.p[t.out.buf] + t.out.off + (int64_t)r * t.out.ld + c0;
#pragma unroll
    for (int q = 0; q < NPL; ++q)
#pragma unroll
        for (int l = 0; l < NL; ++l)
            *reinterpret_cast<int4*>(ob + (int64_t)(q * NL + l) * t.out.ps) =
                *reinterpret_cast<const int4*>(out[q][l]);
}

__global__ void __launch_bounds__(256) condition_f64(const CondTask* tasks, Bases b, FieldParams fp,
                                                     int32_t* err)
{
    const CondTask& t = tasks[blockIdx.y];
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)t.npad * t.kpad) return;
    const int r = (int)(idx / t.kpad), c = (int)(idx % t.kpad);
    int32_t v = 0;
    bool bad = false;
    if (r < t.n && c < t.k)
        bad = !read_input(b.p[t.buf_re] + t.off_re, t.dt_in, (int64_t)r * t.lda + c, fp.p,
                          fp.half, v);
    if (bad) err[0] = 1;
    double* ob = reinterpret_cast<double*>(b.p[t.out.buf] + t.out.off);
    ob[(int64_t)r * t.out.ld + c] = (double)(v > fp.half ? v - fp.p : v);
}

// ============================================================================
// pre-additions with the skew-unitary Y
// ============================================================================

// Value of one element of a carrier plane group (NL limbs).
template <int NL>
__device__ __forceinline__ int32_t car_val(const int8_t* hi, const int8_t* lo, int e)
{
    return NL == 1 ? (int32_t)hi[e] : 256 * (int32_t)hi[e] + (int32_t)lo[e];
}

// Reduce an exact integer to the carrier representative of its residue.  One
// limb (p < 256): every intermediate is below 2^20 and int32 / fp32 arithmetic is
// exact; two limbs: products reach 2^32 and are formed in fp64 (exact below 2^53).
template <int NL>
struct PreArith {
    typedef typename std::conditional<NL == 1, int32_t, double>::type T;
};

template <int NL>
__device__ __forceinline__ int32_t to_rep(typename PreArith<NL>::T v, const FieldParams& fp)
{
    if (NL == 1) return mod_centred_small((int32_t)v, fp.p, (float)fp.inv_p);
    return rep2(mod_canon((double)v, fp.p, fp.inv_p), fp.p);
}

template <int NL>
__device__ __forceinline__ void put_rep(int32_t r, int8_t* hi, int8_t* lo, int e)
{
    if (NL == 1) {
        hi[e] = (int8_t)r;
    } else {
        int8_t h, l;
        split2(r, h, l);
        hi[e] = h;
        lo[e] = l;
    }
}

// Each thread handles VEC columns c.. of the left column half of a block and
// the matching columns c + w/2 of the right half (the block-structured Y mixes
// exactly these two).
template <int NL, int CPLX, int VEC>
__global__ void __launch_bounds__(256) preadd_i8(const PreaddTask* tasks, Bases b, FieldParams fp)
{
    const PreaddTask& T = tasks[blockIdx.y];
    const int h = T.h, w = T.w, hw = w / 2;
    const int gpr = hw / VEC;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= h * gpr) return;
    const int r = idx / gpr, c = (idx % gpr) * VEC;
    constexpr int NPI = CPLX ? 2 : 1;  // planes read (re, im)
    constexpr int NPO = CPLX ? 3 : 1;  // planes written (re, im, -re)
    typedef int8_t vec_t[VEC];

    // load A11, A12, A21, A22 (index blk = 2*row_half + col_half), left/right column halves
    alignas(16) vec_t in[4][2][NPI][NL];
    const char* abase = b.p[T.a.buf] + T.a.off;
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) {
        const int rr = (blk >> 1) * h + r;
        const int cc = (blk & 1) * w + c;
#pragma unroll
        for (int half = 0; half < 2; ++half)
#pragma unroll
            for (int q = 0; q < NPI; ++q)
#pragma unroll
                for (int l = 0; l < NL; ++l) {
                    const char* src = abase + (int64_t)(q * NL + l) * T.a.ps +
                                      (int64_t)rr * T.a.ld + cc + half * hw;
                    if (VEC == 16)
                        *reinterpret_cast<int4*>(in[blk][half][q][l]) =
                            *reinterpret_cast<const int4*>(src);
                    else
                        *reinterpret_cast<int2*>(in[blk][half][q][l]) =
                            *reinterpret_cast<const int2*>(src);
                }
    }
    alignas(16) vec_t out[4][2][NPO][NL];
    const int32_t p = fp.p;
    typedef typename PreArith<NL>::T AT;
    const AT ya = (AT)fp.ya, yb = (AT)fp.yb;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        // x[blk][half][plane]
        int32_t x[4][2][2];
#pragma unroll
        for (int blk = 0; blk < 4; ++blk)
#pragma unroll
            for (int half = 0; half < 2; ++half)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    x[blk][half][q] = (q < NPI) ? car_val<NL>(in[blk][half][q][0],
                                                               in[blk][half][q][NL - 1], e)
                                                : 0;
        int32_t s[4][2][2];  // S1..S4, half, plane
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            AT d[2], a21y[2];  // (A21 - A11) Y and A21 Y on this half
            if (fp.ykind == Y_BLOCKS) {
                // [X_L | X_R] Y = [a X_L - b X_R | b X_L + a X_R]
                const AT dl = x[2][0][0] - x[0][0][0], dr = x[2][1][0] - x[0][1][0];
                const AT el = x[2][0][0], er = x[2][1][0];
                d[0] = half == 0 ? ya * dl - yb * dr : yb * dl + ya * dr;
                a21y[0] = half == 0 ? ya * el - yb * er : yb * el + ya * er;
                d[1] = a21y[1] = 0;
            } else if (fp.ykind == Y_GAUSS) {
                // (u + iv)(a + ib) = (au - bv) + i(bu + av)
                const AT du = x[2][half][0] - x[0][half][0];
                const AT dv = x[2][half][1] - x[0][half][1];
                const AT eu = x[2][half][0], ev = x[2][half][1];
                d[0] = ya * du - yb * dv;
                d[1] = yb * du + ya * dv;
                a21y[0] = ya * eu - yb * ev;
                a21y[1] = yb * eu + ya * ev;
            } else {
                d[0] = ya * (AT)(x[2][half][0] - x[0][half][0]);
                a21y[0] = ya * (AT)x[2][half][0];
                d[1] = a21y[1] = 0;
            }
#pragma unroll
            for (int q = 0; q < NPI; ++q) {
                const int32_t s1 = to_rep<NL>(d[q], fp);
                const int32_t s2 = to_rep<NL>((AT)x[3][half][q] - a21y[q], fp);
                const int32_t s3 = to_rep<NL>((AT)(s1 - x[3][half][q]), fp);
                const int32_t s4 = to_rep<NL>((AT)(s3 + x[1][half][q]), fp);
                s[0][half][q] = s1;
                s[1][half][q] = s2;
                s[2][half][q] = s3;
                s[3][half][q] = s4;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int half = 0; half < 2; ++half) {
#pragma unroll
                for (int q = 0; q < NPI; ++q)
                    put_rep<NL>(s[j][half][q], out[j][half][q][0], out[j][half][q][NL - 1], e);
                if (CPLX) {
                    // the "-re" plane used by the imaginary part of complex products
                    int32_t v = s[j][half][0];
                    int32_t nv = NL == 1 ? -v : rep2(neg_mod(v < 0 ? v + p : v, p), p);
                    put_rep<NL>(nv, out[j][half][NPO - 1][0], out[j][half][NPO - 1][NL - 1], e);
                }
            }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        char* sbase = b.p[T.s[j].buf] + T.s[j].off + (int64_t)r * T.s[j].ld + c;
#pragma unroll
        for (int half = 0; half < 2; ++half)
#pragma unroll
            for (int q = 0; q < NPO; ++q)
#pragma unroll
                for (int l = 0; l < NL; ++l) {
                    char* dst = sbase + (int64_t)(q * NL + l) * T.s[j].ps + half * hw;
                    if (VEC == 16)
                        *reinterpret_cast<int4*>(dst) =
                            *reinterpret_cast<const int4*>(out[j][half][q][l]);
                    else
                        *reinterpret_cast<int2*>(dst) =
                            *reinterpret_cast<const int2*>(out[j][half][q][l]);
                }
    }
}

// fp64 carrier (real only): centred residues held as doubles.
__global__ void __launch_bounds__(256) preadd_f64(const PreaddTask* tasks, Bases b,
                                                  FieldParams fp)
{
    const PreaddTask& T = tasks[blockIdx.y];
    const int h = T.h, w = T.w, hw = w / 2;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= h * hw) return;
    const int r = idx / hw, c = idx % hw;
    const double* A = reinterpret_cast<const double*>(b.p[T.a.buf] + T.a.off);
    double x[4][2];
#pragma unroll
    for (int blk = 0; blk < 4; ++blk)
#pragma unroll
        for (int half = 0; half < 2; ++half)
            x[blk][half] = A[(int64_t)((blk >> 1) * h + r) * T.a.ld + (blk & 1) * w + c + half * hw];
    const double ya = fp.ya, yb = fp.yb, p = fp.p;
    auto cen = [&](double v) {
        int32_t cc = mod_canon(v, fp.p, fp.inv_p);
        return (double)(cc > fp.half ? cc - fp.p : cc);
    };
    (void)p;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        double d, a21y;
        if (fp.ykind == Y_BLOCKS) {
            const double dl = x[2][0] - x[0][0], dr = x[2][1] - x[0][1];
            d = half == 0 ? ya * dl - yb * dr : yb * dl + ya * dr;
            a21y = half == 0 ? ya * x[2][0] - yb * x[2][1] : yb * x[2][0] + ya * x[2][1];
        } else {
            d = ya * (x[2][half] - x[0][half]);
            a21y = ya * x[2][half];
        }
        const double s1 = cen(d);
        const double s2 = cen(x[3][half] - a21y);
        const double s3 = cen(s1 - x[3][half]);
        const double s4 = cen(s3 + x[1][half]);
        const double sv[4] = {s1, s2, s3, s4};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double* S = reinterpret_cast<double*>(b.p[T.s[j].buf] + T.s[j].off);
            S[(int64_t)r * T.s[j].ld + c + half * hw] = sv[j];
        }
    }
}

// ============================================================================
// post-additions
// ============================================================================

template <typename RT>
__device__ __forceinline__ void load_row16(const char* base, int ld, int row, int col, int32_t* v)
{
    const RT* src = reinterpret_cast<const RT*>(base) + (int64_t)row * ld + col;
    if (sizeof(RT) == 1) {
        int4 q = *reinterpret_cast<const int4*>(src);
        const uint8_t* u = reinterpret_cast<const uint8_t*>(&q);
#pragma unroll
        for (int e = 0; e < 16; ++e) v[e] = u[e];
    } else if (sizeof(RT) == 2) {
        int4 q[2];
        q[0] = reinterpret_cast<const int4*>(src)[0];
        q[1] = reinterpret_cast<const int4*>(src)[1];
        const uint16_t* u = reinterpret_cast<const uint16_t*>(q);
#pragma unroll
        for (int e = 0; e < 16; ++e) v[e] = u[e];
    } else {
        int4 q[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) q[i] = reinterpret_cast<const int4*>(src)[i];
        const int32_t* u = reinterpret_cast<const int32_t*>(q);
#pragma unroll
        for (int e = 0; e < 16; ++e) v[e] = u[e];
    }
}

// Stores 16 consecutive elements of a row: one or more 16-byte vector stores
// when all are wanted and the address is aligned, element stores otherwise.
template <typename OT>
__device__ __forceinline__ void store_row16(char* base, int64_t idx, const int32_t* v, int nwant)
{
    OT* dst = reinterpret_cast<OT*>(base) + idx;
    if (nwant >= 16 && ((uintptr_t)dst & 15) == 0) {
        alignas(16) OT tmp[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) tmp[e] = (OT)v[e];
#pragma unroll
        for (int q = 0; q < (int)(16 * sizeof(OT) / 16); ++q)
            reinterpret_cast<int4*>(dst)[q] = reinterpret_cast<const int4*>(tmp)[q];
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e)
            if (e < nwant) dst[e] = (OT)v[e];
    }
}

// Lower tile pairs (R, C), R >= C, of 64 x 64 tiles of the h x h blocks; one
// workgroup of 256 threads per pair; thread = (row tr, 16-column group).  All
// loads and stores move 16 consecutive elements of a row.
template <typename RT, typename OT, int CPLX>
__global__ void __launch_bounds__(256) postadd(const PostaddTask* tasks, Bases b, FieldParams fp)
{
    constexpr int TS = 64;
    constexpr int NP = CPLX ? 2 : 1;
    __shared__ int32_t u1s[NP][TS][TS + 1];
    __shared__ int32_t p4s[NP][TS][TS + 1];

    const PostaddTask& T = tasks[blockIdx.y];
    const int h = T.h, nt = (h + TS - 1) / TS;
    const int t = blockIdx.x;
    int R = (int)((sqrtf(8.f * t + 1.f) - 1.f) * 0.5f);
    while ((R + 1) * (R + 2) / 2 <= t) ++R;
    while (R * (R + 1) / 2 > t) --R;
    const int C = t - R * (R + 1) / 2;
    if (R >= nt) return;
    const int p = fp.p;
    const int tr = threadIdx.x >> 2, tc = (threadIdx.x & 3) * 16;
    const bool diag = (R == C);

    const int gi = R * TS + tr;          // row (within the h x h block) of tile (R, C)
    const int gj0 = C * TS + tc;         // first column of this thread in tile (R, C)
    const int mi = C * TS + tr;          // row of the mirrored tile (C, R)
    const int mj0 = R * TS + tc;

    auto plane = [&](const ResRef& rr, int q) -> const char* {
        return q == 0 ? b.p[rr.buf] + rr.off : b.p[rr.buf2] + rr.off2;
    };
    int32_t P1[NP][16], P2[NP][16], P3[NP][16], P4[NP][16], P5[NP][16];
    int32_t Q3[NP][16], Q4[NP][16];  // tiles (C, R) of P3 and P4
#pragma unroll
    for (int q = 0; q < NP; ++q) {
#pragma unroll
        for (int e = 0; e < 16; ++e)
            P1[q][e] = P2[q][e] = P3[q][e] = P4[q][e] = P5[q][e] = Q3[q][e] = Q4[q][e] = 0;
        if (gi < h && gj0 < h) {
            load_row16<RT>(plane(T.p[0], q), T.p[0].ld, gi, gj0, P1[q]);
            load_row16<RT>(plane(T.p[1], q), T.p[1].ld, gi, gj0, P2[q]);
            load_row16<RT>(plane(T.p[2], q), T.p[2].ld, gi, gj0, P3[q]);
            load_row16<RT>(plane(T.p[3], q), T.p[3].ld, gi, gj0, P4[q]);
            load_row16<RT>(plane(T.p[4], q), T.p[4].ld, gi, gj0, P5[q]);
        }
        if (!diag && mi < h && mj0 < h) {
            load_row16<RT>(plane(T.p[2], q), T.p[2].ld, mi, mj0, Q3[q]);
            load_row16<RT>(plane(T.p[3], q), T.p[3].ld, mi, mj0, Q4[q]);
        }
    }
    // U1 = P1 + P5 on tile (R, C); stage U1 and the tile whose transpose is needed
    int32_t U1[NP][16];
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            U1[q][e] = add_mod(P1[q][e], P5[q][e], p);
            u1s[q][tr][tc + e] = U1[q][e];
            p4s[q][tr][tc + e] = diag ? P4[q][e] : Q4[q][e];
        }
    __syncthreads();

    // the node's C: C11 at (0,0), C21 at (h,0), C22 at (h,h); rows/cols >= nvalid not written
    const int nv = T.nvalid;
    const int64_t ldc = T.c.ld;
    char* cpl[2] = {b.p[T.c.buf] + T.c.off, b.p[T.c.buf2] + T.c.off2};
    // conjugation of the imaginary plane under phi
    auto conjv = [&](int q, int32_t v) { return q == 1 ? neg_mod(v, p) : v; };
    // number of the 16 columns starting at col that are inside [0, lim)
    auto cnt = [](int col, int lim) { return max(0, min(16, lim - col)); };

    if (gi < h) {
        const int wantC = cnt(gj0, min(h, nv));            // C11 columns
        const int wantH = cnt(h + gj0, nv);                // C21 / C22 columns (offset h)
        const int lowlen = diag ? min(16, max(0, tr - tc + 1)) : 16;  // entries with col <= row
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            int32_t c11[16], c21[16], c22[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int lc = tc + e;
                // phi(Low(U1)) above the diagonal of the diagonal tile; P4^phi at (gi, gj)
                int32_t u1full = U1[q][e];
                if (diag && lc > tr) u1full = conjv(q, u1s[q][lc][tr]);
                const int32_t p4t = conjv(q, p4s[q][lc][tr]);
                const int32_t u2 = add_mod(u1full, P4[q][e], p);
                c21[e] = add_mod(u2, P3[q][e], p);     // U4 = U2 + P3
                c11[e] = add_mod(P1[q][e], P2[q][e], p);  // U3 = P1 + P2
                c22[e] = add_mod(u2, p4t, p);          // U5 = U2 + phi(P4)
            }
            if (gi < nv) store_row16<OT>(cpl[q], (int64_t)gi * ldc + gj0, c11, min(wantC, lowlen));
            if (h + gi < nv) {
                store_row16<OT>(cpl[q], (int64_t)(h + gi) * ldc + gj0, c21, wantC);
                store_row16<OT>(cpl[q], (int64_t)(h + gi) * ldc + h + gj0, c22, min(wantH, lowlen));
            }
        }
    }
    if (!diag && mi < h && h + mi < nv) {
        // tile (C, R) of C21: U1 there is phi of the staged lower tile (R, C)
        const int want = cnt(mj0, min(h, nv));
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            int32_t c21[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int32_t u1 = conjv(q, u1s[q][tc + e][tr]);
                c21[e] = add_mod(add_mod(u1, Q4[q][e], p), Q3[q][e], p);
            }
            store_row16<OT>(cpl[q], (int64_t)(h + mi) * ldc + mj0, c21, want);
        }
    }
}

// ============================================================================
// launch wrappers
// ============================================================================

__global__ void zero_flag(int32_t* f) { f[0] = 0; }

int launch_zero_flag(int32_t* d_flag, void* stream)
{
    hipLaunchKernelGGL(zero_flag, dim3(1), dim3(1), 0, (hipStream_t)stream, d_flag);
    return (int)hipGetLastError();
}

int launch_condition(const CondTask* d_tasks, int ntasks, int max_blocks, const Bases& b,
                     const FieldParams& fp, int carrier, int32_t* d_err, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (ntasks <= 0 || max_blocks <= 0) return 0;
    dim3 g(max_blocks, ntasks);
    if (carrier == CAR_F64)
        hipLaunchKernelGGL(condition_f64, g, dim3(256), 0, s, d_tasks, b, fp, d_err);
    else if (fp.nl == 1 && !fp.cplx)
        hipLaunchKernelGGL((condition_i8<1, 0>), g, dim3(256), 0, s, d_tasks, b, fp, d_err);
    else if (fp.nl == 2 && !fp.cplx)
        hipLaunchKernelGGL((condition_i8<2, 0>), g, dim3(256), 0, s, d_tasks, b, fp, d_err);
    else if (fp.nl == 1)
        hipLaunchKernelGGL((condition_i8<1, 1>), g, dim3(256), 0, s, d_tasks, b, fp, d_err);
    else
        hipLaunchKernelGGL((condition_i8<2, 1>), g, dim3(256), 0, s, d_tasks, b, fp, d_err);
    return (int)hipGetLastError();
}

int launch_preadd(const PreaddTask* d_tasks, int ntasks, int h, int w, const Bases& b,
                  const FieldParams& fp, int carrier, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (ntasks <= 0 || h <= 0 || w <= 0) return 0;
    if (carrier == CAR_F64) {
        const int64_t total = (int64_t)h * (w / 2);
        hipLaunchKernelGGL(preadd_f64, dim3((unsigned)((total + 255) / 256), ntasks), dim3(256), 0,
                           s, d_tasks, b, fp);
    } else if (!fp.cplx) {
        const int64_t total = (int64_t)h * (w / 2 / 16);
        dim3 g((unsigned)((total + 255) / 256), ntasks);
        if (fp.nl == 1) hipLaunchKernelGGL((preadd_i8<1, 0, 16>), g, dim3(256), 0, s, d_tasks, b, fp);
        else hipLaunchKernelGGL((preadd_i8<2, 0, 16>), g, dim3(256), 0, s, d_tasks, b, fp);
    } else {
        const int64_t total = (int64_t)h * (w / 2 / 8);
        dim3 g((unsigned)((total + 255) / 256), ntasks);
        if (fp.nl == 1) hipLaunchKernelGGL((preadd_i8<1, 1, 8>), g, dim3(256), 0, s, d_tasks, b, fp);
        else hipLaunchKernelGGL((preadd_i8<2, 1, 8>), g, dim3(256), 0, s, d_tasks, b, fp);
    }
    return (int)hipGetLastError();
}

template <typename RT, int CPLX>
static void launch_post_rt(dim3 g, hipStream_t s, const PostaddTask* d_tasks, const Bases& b,
                           const FieldParams& fp, int out_dt)
{
    switch (out_dt) {
    case DT_U8: hipLaunchKernelGGL((postadd<RT, uint8_t, CPLX>), g, dim3(256), 0, s, d_tasks, b, fp); break;
    case DT_U16: hipLaunchKernelGGL((postadd<RT, uint16_t, CPLX>), g, dim3(256), 0, s, d_tasks, b, fp); break;
    case DT_I32: hipLaunchKernelGGL((postadd<RT, int32_t, CPLX>), g, dim3(256), 0, s, d_tasks, b, fp); break;
    case DT_I64: hipLaunchKernelGGL((postadd<RT, int64_t, CPLX>), g, dim3(256), 0, s, d_tasks, b, fp); break;
    case DT_F64: hipLaunchKernelGGL((postadd<RT, double, CPLX>), g, dim3(256), 0, s, d_tasks, b, fp); break;
    default: break;
    }
}

int launch_postadd(const PostaddTask* d_tasks, int ntasks, int h, int out_dt, const Bases& b,
                   const FieldParams& fp, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (ntasks <= 0 || h <= 0) return 0;
    const int nt = (h + 63) / 64;
    dim3 g(nt * (nt + 1) / 2, ntasks);
    if (fp.p < 256) {
        if (fp.cplx) launch_post_rt<uint8_t, 1>(g, s, d_tasks, b, fp, out_dt);
        else launch_post_rt<uint8_t, 0>(g, s, d_tasks, b, fp, out_dt);
    } else if (fp.p < 65536) {
        if (fp.cplx) launch_post_rt<uint16_t, 1>(g, s, d_tasks, b, fp, out_dt);
        else launch_post_rt<uint16_t, 0>(g, s, d_tasks, b, fp, out_dt);
    } else {
        if (fp.cplx) launch_post_rt<int32_t, 1>(g, s, d_tasks, b, fp, out_dt);
        else launch_post_rt<int32_t, 0>(g, s, d_tasks, b, fp, out_dt);
    }
    return (int)hipGetLastError();
}

}  // namespace ffa
