// HBM-bound kernels of the recursion (Algorithm 1, Section 3):
//   * conditioning: caller's residues -> carrier planes (zero padded);
//   * pre-additions: S1 = (A21 - A11) Y, S2 = A22 - A21 Y, S3 = S1 - A22,
//     S4 = S3 + A12, fused in one pass per recursion level;
//   * post-additions: U1 = P1 + P5, U3 = P1 + P2, Up(U1) = phi(Low(U1)),
//     U2 = U1 + P4, U4 = U2 + P3, U5 = Low(U2) + Low(phi(P4)), fused in one
//     pass per recursion level, transposed reads staged through LDS.
// Every value is reduced mod p where it is produced.
#include <hip/hip_runtime.h>

#include <algorithm>

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

// Loads 16 consecutive input elements of a row as canonical residues; vector
// loads when the 16 are inside the row and aligned.  Returns false if an entry
// is outside its residue range.
template <typename IT>
__device__ __forceinline__ bool load_input16(const char* base, int64_t idx, int valid, int32_t p,
                                             int32_t half, bool centred, int32_t* v)
{
    const IT* src = reinterpret_cast<const IT*>(base) + idx;
    alignas(16) IT raw[16];
    if (valid >= 16 && ((uintptr_t)src & 15) == 0) {
#pragma unroll
        for (int q = 0; q < (int)(16 * sizeof(IT) / 16); ++q)
            reinterpret_cast<int4*>(raw)[q] = reinterpret_cast<const int4*>(src)[q];
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) raw[e] = e < valid ? src[e] : (IT)0;
    }
    bool ok = true;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        if (centred) {
            const int32_t x = (int32_t)raw[e];
            ok &= (x >= -half) & (x <= half);
            v[e] = x < 0 ? x + p : x;
        } else {
            const double xd = (double)raw[e];
            const int32_t x = (int32_t)raw[e];
            ok &= (xd >= 0.0) & (xd < (double)p) & ((double)x == xd);
            v[e] = x;
        }
    }
    return ok;
}

// The task owning block blk of a one-dimensional grid (tasks in order of blk0).
__device__ __forceinline__ int cond_task_of(const CondTask* tasks, int ntasks, int blk)
{
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tasks[mid].blk0 <= blk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// One thread converts 16 consecutive columns of one row into every carrier
// sub-plane (limbs of re, and of im and -re for F_p[i]).
template <typename IT, int NL, int CPLX>
__global__ void __launch_bounds__(256) condition_i8(const CondTask* tasks, int ntasks, Bases b,
                                                    FieldParams fp, int32_t* err)
{
    constexpr int VEC = 16;
    const CondTask& t = tasks[cond_task_of(tasks, ntasks, (int)blockIdx.x)];
    const int gpr = t.kpad / VEC;
    const int64_t idx = (int64_t)((int)blockIdx.x - t.blk0) * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)t.npad * gpr) return;
    const int r = (int)(idx / gpr), c0 = (int)(idx % gpr) * VEC;
    const int p = fp.p;
    const bool centred = t.dt_in == DT_I8C;
    constexpr int NPL = CPLX ? 4 : 1;  // re, im, -re, re + im (the last for the 2M base case)
    const int npl = CPLX ? fp.npo : 1;
    int32_t vr[16], vi[16];
    bool ok = true;
    const int valid = (r < t.n) ? max(0, min(VEC, t.k - c0)) : 0;
    const int64_t off = (int64_t)r * t.lda + c0;
    if (valid > 0) {
        ok &= load_input16<IT>(b.p[t.buf_re] + t.off_re, off, valid, p, fp.half, centred, vr);
        if (CPLX) ok &= load_input16<IT>(b.p[t.buf_im] + t.off_im, off, valid, p, fp.half, centred, vi);
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) vr[e] = vi[e] = 0;
    }
    if (!ok) err[0] = 1;
    alignas(16) int8_t out[NPL][NL][VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        const int32_t vals[4] = {vr[e], CPLX ? vi[e] : 0, neg_mod(vr[e], p), add_mod(vr[e], CPLX ? vi[e] : 0, p)};
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
    char* ob = b.p[t.out.buf] + t.out.off + (int64_t)r * t.out.ld + c0;
#pragma unroll
    for (int q = 0; q < NPL; ++q)
#pragma unroll
        for (int l = 0; l < NL; ++l)
            if (q < npl && !((t.skip >> q) & 1))
                *reinterpret_cast<int4*>(ob + (int64_t)(q * NL + l) * t.out.ps) =
                    *reinterpret_cast<const int4*>(out[q][l]);
}

// ST: storage of the fp64 carrier (double, or float for integers below 2^24)
template <typename ST>
__global__ void __launch_bounds__(256) condition_f64(const CondTask* tasks, int ntasks, Bases b,
                                                     FieldParams fp, int32_t* err)
{
    // four consecutive columns per thread (kpad is a multiple of the k-tile)
    constexpr int V = 4;
    const CondTask& t = tasks[cond_task_of(tasks, ntasks, (int)blockIdx.x)];
    const int gpr = t.kpad / V;
    const int64_t idx = (int64_t)((int)blockIdx.x - t.blk0) * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)t.npad * gpr) return;
    const int r = (int)(idx / gpr), c0 = (int)(idx % gpr) * V;
    alignas(16) ST out[V];
    bool bad = false;
#pragma unroll
    for (int e = 0; e < V; ++e) {
        const int c = c0 + e;
        int32_t v = 0;
        if (r < t.n && c < t.k)
            bad |= !read_input(b.p[t.buf_re] + t.off_re, t.dt_in, (int64_t)r * t.lda + c, fp.p, fp.half, v);
        out[e] = (ST)(v > fp.half ? v - fp.p : v);
    }
    if (bad) err[0] = 1;
    ST* ob = reinterpret_cast<ST*>(b.p[t.out.buf] + t.out.off) + (int64_t)r * t.out.ld + c0;
    if (sizeof(ST) == 4) {
        *reinterpret_cast<int4*>(ob) = *reinterpret_cast<const int4*>(out);
    } else {
        reinterpret_cast<int4*>(ob)[0] = reinterpret_cast<const int4*>(out)[0];
        reinterpret_cast<int4*>(ob)[1] = reinterpret_cast<const int4*>(out)[1];
    }
}

// ============================================================================
// pre-additions with the skew-unitary Y
// ============================================================================

// Canonical residue of one element of a carrier plane group (NL limbs).
template <int NL>
__device__ __forceinline__ int32_t car_canon(const int8_t* hi, const int8_t* lo, int e, int32_t p)
{
    const int32_t r = NL == 1 ? (int32_t)hi[e] : 256 * (int32_t)hi[e] + (int32_t)lo[e];
    return r < 0 ? r + p : r;
}

// Writes the carrier encoding of a canonical residue.
template <int NL>
__device__ __forceinline__ void put_canon(int32_t c, int32_t p, int32_t half, int8_t* hi, int8_t* lo,
                                          int e)
{
    if (NL == 1) {
        hi[e] = (int8_t)(c > half ? c - p : c);
    } else {
        int8_t h, l;
        split2(rep2(c, p), h, l);
        hi[e] = h;
        lo[e] = l;
    }
}

// Each thread handles VEC columns c.. of the left column half of a block and
// the matching columns c + w/2 of the right half (the block-structured Y mixes
// exactly these two).  All arithmetic is on canonical residues in 32-bit
// integers: products of two residues stay below 2^32 for p < 2^16.
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
    constexpr int NPO = CPLX ? 4 : 1;  // planes written (re, im, -re; re + im for S3 in the 2M mode)
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
    const float ip = (float)fp.inv_p;
    const int32_t ya = fp.ya, yb = fp.yb, nyb = neg_mod(fp.yb, p);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        int32_t x[4][2][2];  // [block][half][plane], canonical
#pragma unroll
        for (int blk = 0; blk < 4; ++blk)
#pragma unroll
            for (int half = 0; half < 2; ++half)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    x[blk][half][q] =
                        (q < NPI) ? car_canon<NL>(in[blk][half][q][0], in[blk][half][q][NL - 1], e, p) : 0;
        int32_t s[4][2][2];  // S1..S4, half, plane
        int32_t d[2][2], g[2][2];  // (A21 - A11) Y and A21 Y, per half and plane
        if (NL == 1) {
            // p < 256: every combination below is an exact int32 below 2^17 in magnitude;
            // one centred reduction per value
            auto cen = [&](int32_t v) {
                const int32_t m = mod_centred_small(v, p, ip);
                return m < 0 ? m + p : m;
            };
            if (fp.ykind == Y_BLOCKS) {
                const int32_t dl = x[2][0][0] - x[0][0][0], dr = x[2][1][0] - x[0][1][0];
                const int32_t el = x[2][0][0], er = x[2][1][0];
                d[0][0] = cen(ya * dl - yb * dr);
                d[1][0] = cen(yb * dl + ya * dr);
                g[0][0] = cen(ya * el - yb * er);
                g[1][0] = cen(yb * el + ya * er);
                d[0][1] = d[1][1] = g[0][1] = g[1][1] = 0;
            } else {
#pragma unroll
                for (int half = 0; half < 2; ++half) {
                    if (fp.ykind == Y_GAUSS) {
                        const int32_t du = x[2][half][0] - x[0][half][0];
                        const int32_t dv = x[2][half][1] - x[0][half][1];
                        const int32_t eu = x[2][half][0], ev = x[2][half][1];
                        d[half][0] = cen(ya * du - yb * dv);
                        d[half][1] = cen(yb * du + ya * dv);
                        g[half][0] = cen(ya * eu - yb * ev);
                        g[half][1] = cen(yb * eu + ya * ev);
                    } else {
                        d[half][0] = cen(ya * (x[2][half][0] - x[0][half][0]));
                        g[half][0] = cen(ya * x[2][half][0]);
                        d[half][1] = g[half][1] = 0;
                    }
                }
            }
        } else if (fp.ykind == Y_BLOCKS) {
            // [X_L | X_R] Y = [a X_L - b X_R | b X_L + a X_R]
            const int32_t dl = sub_mod(x[2][0][0], x[0][0][0], p), dr = sub_mod(x[2][1][0], x[0][1][0], p);
            const int32_t el = x[2][0][0], er = x[2][1][0];
            d[0][0] = add_mod(mul_mod(ya, dl, p, ip), mul_mod(nyb, dr, p, ip), p);
            d[1][0] = add_mod(mul_mod(yb, dl, p, ip), mul_mod(ya, dr, p, ip), p);
            g[0][0] = add_mod(mul_mod(ya, el, p, ip), mul_mod(nyb, er, p, ip), p);
            g[1][0] = add_mod(mul_mod(yb, el, p, ip), mul_mod(ya, er, p, ip), p);
            d[0][1] = d[1][1] = g[0][1] = g[1][1] = 0;
        } else {
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                if (fp.ykind == Y_GAUSS) {
                    // (u + iv)(a + ib) = (au - bv) + i(bu + av)
                    const int32_t du = sub_mod(x[2][half][0], x[0][half][0], p);
                    const int32_t dv = sub_mod(x[2][half][1], x[0][half][1], p);
                    const int32_t eu = x[2][half][0], ev = x[2][half][1];
                    d[half][0] = add_mod(mul_mod(ya, du, p, ip), mul_mod(nyb, dv, p, ip), p);
                    d[half][1] = add_mod(mul_mod(yb, du, p, ip), mul_mod(ya, dv, p, ip), p);
                    g[half][0] = add_mod(mul_mod(ya, eu, p, ip), mul_mod(nyb, ev, p, ip), p);
                    g[half][1] = add_mod(mul_mod(yb, eu, p, ip), mul_mod(ya, ev, p, ip), p);
                } else {
                    d[half][0] = mul_mod(ya, sub_mod(x[2][half][0], x[0][half][0], p), p, ip);
                    g[half][0] = mul_mod(ya, x[2][half][0], p, ip);
                    d[half][1] = g[half][1] = 0;
                }
            }
        }
#pragma unroll
        for (int half = 0; half < 2; ++half)
#pragma unroll
            for (int q = 0; q < NPI; ++q) {
                const int32_t s1 = d[half][q];
                const int32_t s2 = sub_mod(x[3][half][q], g[half][q], p);
                const int32_t s3 = sub_mod(s1, x[3][half][q], p);
                const int32_t s4 = add_mod(s3, x[1][half][q], p);
                s[0][half][q] = s1;
                s[1][half][q] = s2;
                s[2][half][q] = s3;
                s[3][half][q] = s4;
            }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int half = 0; half < 2; ++half) {
#pragma unroll
                for (int q = 0; q < NPI; ++q)
                    put_canon<NL>(s[j][half][q], p, fp.half, out[j][half][q][0], out[j][half][q][NL - 1], e);
                // the "-re" plane used by the imaginary part of complex products, and
                // re + im, which the 2M base case squares
                if (CPLX) {
                    put_canon<NL>(neg_mod(s[j][half][0], p), p, fp.half, out[j][half][2][0],
                                  out[j][half][2][NL - 1], e);
                    put_canon<NL>(add_mod(s[j][half][0], s[j][half][NPI - 1], p), p, fp.half,
                                  out[j][half][NPO - 1][0], out[j][half][NPO - 1][NL - 1], e);
                }
            }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        char* sbase = b.p[T.s[j].buf] + T.s[j].off + (int64_t)r * T.s[j].ld + c;
        const int nplanes = !CPLX ? 1 : (j == 2 ? fp.npo : 3);
#pragma unroll
        for (int half = 0; half < 2; ++half)
#pragma unroll
            for (int q = 0; q < NPO; ++q)
#pragma unroll
                for (int l = 0; l < NL; ++l) {
                    if (q >= nplanes) continue;
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

// One limb over F_p (p < 2^8), real field: the carrier and every S hold centred
// residues in [-(p-1)/2, (p-1)/2], and the pre-additions stay in that form
// throughout (no canonical round trip).  Each S is reduced once: a sum that
// contains a product by a coefficient of Y with an fp32 quotient
// (mod_centred_small), a short sum of residues with cen_short.  The element
// pairs (left column c, right column c + w/2) are those the block-structured Y
// mixes; with the scalar Y the two halves are independent.
typedef int nt4 __attribute__((ext_vector_type(4)));

template <int YK, int VEC, bool NT = false>
__device__ __forceinline__ void preadd_c1_item(const PreaddTask& T, const Bases& b, const FieldParams& fp,
                                               int r, int c)
{
    const int h = T.h, w = T.w, hw = w / 2;
    typedef int8_t vec_t[VEC];
    // A11, A12, A21, A22 (blk = 2 * row half + column half), left / right column halves
    alignas(16) vec_t in[4][2];
    const char* abase = b.p[T.a.buf] + T.a.off;
#pragma unroll
    for (int blk = 0; blk < 4; ++blk)
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const char* src = abase + (int64_t)((blk >> 1) * h + r) * T.a.ld + (blk & 1) * w + c + half * hw;
            if (NT) *reinterpret_cast<nt4*>(in[blk][half]) = __builtin_nontemporal_load(reinterpret_cast<const nt4*>(src));
            else if (VEC == 16) *reinterpret_cast<int4*>(in[blk][half]) = *reinterpret_cast<const int4*>(src);
            else *reinterpret_cast<int2*>(in[blk][half]) = *reinterpret_cast<const int2*>(src);
        }
    const int32_t p = fp.p, r20 = fp.r20;
    const float ip = (float)fp.inv_p;
    // Y's coefficients as centred residues (|a|, |b| <= (p-1)/2)
    const int32_t ca = fp.ya > fp.half ? fp.ya - p : fp.ya;
    const int32_t cb = fp.yb > fp.half ? fp.yb - p : fp.yb;
    alignas(16) vec_t out[4][2];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        int32_t x[4][2];
#pragma unroll
        for (int blk = 0; blk < 4; ++blk)
#pragma unroll
            for (int half = 0; half < 2; ++half) x[blk][half] = in[blk][half][e];
        int32_t s1[2], s2[2];
        if (YK == Y_BLOCKS) {
            // [X_L | X_R] Y = [a X_L - b X_R | b X_L + a X_R];  |.| <= 4 ((p-1)/2)^2 < 2^16
            const int32_t dl = x[2][0] - x[0][0], dr = x[2][1] - x[0][1];
            s1[0] = mod_centred_small(__mul24(ca, dl) - __mul24(cb, dr), p, ip);
            s1[1] = mod_centred_small(__mul24(cb, dl) + __mul24(ca, dr), p, ip);
            s2[0] = mod_centred_small(x[3][0] - __mul24(ca, x[2][0]) + __mul24(cb, x[2][1]), p, ip);
            s2[1] = mod_centred_small(x[3][1] - __mul24(cb, x[2][0]) - __mul24(ca, x[2][1]), p, ip);
        } else {
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                s1[half] = mod_centred_small(__mul24(ca, x[2][half] - x[0][half]), p, ip);
                s2[half] = mod_centred_small(x[3][half] - __mul24(ca, x[2][half]), p, ip);
            }
        }
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int32_t t = s1[half] - x[3][half];  // S3 before reduction, |t| <= p - 1
            out[0][half][e] = (int8_t)s1[half];
            out[1][half][e] = (int8_t)s2[half];
            out[2][half][e] = (int8_t)cen_short(t, p, r20);                  // S3 = S1 - A22
            out[3][half][e] = (int8_t)cen_short(t + x[1][half], p, r20);     // S4 = S3 + A12
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        char* sbase = b.p[T.s[j].buf] + T.s[j].off + (int64_t)r * T.s[j].ld + c;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            char* dst = sbase + half * hw;
            if (NT) __builtin_nontemporal_store(*reinterpret_cast<const nt4*>(out[j][half]), reinterpret_cast<nt4*>(dst));
            else if (VEC == 16) *reinterpret_cast<int4*>(dst) = *reinterpret_cast<const int4*>(out[j][half]);
            else *reinterpret_cast<int2*>(dst) = *reinterpret_cast<const int2*>(out[j][half]);
        }
    }
}

template <int YK, int VEC>
__global__ void __launch_bounds__(256) preadd_c1(const PreaddTask* tasks, Bases b, FieldParams fp)
{
    const PreaddTask& T = tasks[blockIdx.y];
    const int gpr = T.w / 2 / VEC;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= T.h * gpr) return;
    preadd_c1_item<YK, VEC>(T, b, fp, idx / gpr, (idx % gpr) * VEC);
}

// The same on a fixed grid that loops over the work, for running beside the
// product launch: each workgroup, once every one of its threads' S values is
// stored, raises the workspace counter by one with release ordering at device
// scope (its stores are written back from this XCD's L2 before the counter
// moves), so that product tiles waiting for the counter read complete S blocks.
// Its loads and stores are non-temporal: the streamed blocks then displace less
// of the operand panels that the product tiles beside it keep in L2 (measured:
// 1.847 vs 1.860 ms per call at 16384^2, p = 251).
template <int YK>
__global__ void __launch_bounds__(256) preadd_c1_signal(const PreaddTask* tasks, Bases b, FieldParams fp,
                                                        int64_t counter_off)
{
    constexpr int VEC = 16;
    const PreaddTask& T = tasks[blockIdx.y];
    const int gpr = T.w / 2 / VEC;
    const int total = T.h * gpr;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x)
        preadd_c1_item<YK, VEC, true>(T, b, fp, idx / gpr, (idx % gpr) * VEC);
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(reinterpret_cast<int32_t*>(b.p[BUF_WS] + counter_off), 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void zero_words(Bases b, int64_t off, int words)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < words) reinterpret_cast<int32_t*>(b.p[BUF_WS] + off)[i] = 0;
}

// fp64 carrier (real only): centred residues held as doubles.
template <typename ST>
__global__ void __launch_bounds__(256) preadd_f64(const PreaddTask* tasks, Bases b,
                                                  FieldParams fp)
{
    const PreaddTask& T = tasks[blockIdx.y];
    const int h = T.h, w = T.w, hw = w / 2;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= h * hw) return;
    const int r = idx / hw, c = idx % hw;
    const ST* A = reinterpret_cast<const ST*>(b.p[T.a.buf] + T.a.off);
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
            ST* S = reinterpret_cast<ST*>(b.p[T.s[j].buf] + T.s[j].off);
            S[(int64_t)r * T.s[j].ld + c + half * hw] = (ST)sv[j];
        }
    }
}

// ============================================================================
// post-additions
// ============================================================================

// Stores V consecutive elements of a row: vector stores when all are wanted
// and the address is aligned, element stores otherwise.
template <typename OT, int V>
__device__ __forceinline__ void store_rowv(char* base, int64_t idx, const int32_t* v, int nwant)
{
    OT* dst = reinterpret_cast<OT*>(base) + idx;
    constexpr int BYTES = V * (int)sizeof(OT);
    if (nwant >= V && ((uintptr_t)dst & (BYTES >= 16 ? 15 : BYTES - 1)) == 0) {
        alignas(16) OT tmp[V];
#pragma unroll
        for (int e = 0; e < V; ++e) tmp[e] = (OT)v[e];
        if (BYTES >= 16) {
#pragma unroll
            for (int q = 0; q < BYTES / 16; ++q)
                reinterpret_cast<int4*>(dst)[q] = reinterpret_cast<const int4*>(tmp)[q];
        } else if (BYTES == 8) {
            *reinterpret_cast<int2*>(dst) = *reinterpret_cast<const int2*>(tmp);
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) dst[e] = tmp[e];
        }
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e)
            if (e < nwant) dst[e] = (OT)v[e];
    }
}

// v <- alpha v + beta C_old mod p on the first n of V consecutive entries of a row
// of the caller's C (the SYRK update form of Section 7; beta = 0 does not read C).
// alpha v and beta C_old are below 2^52 for p < 2^26, so the sum is exact in fp64.
template <typename OT, int V>
__device__ __forceinline__ void update_rowv(const char* base, int64_t idx, int32_t* v, int n,
                                            const FieldParams& fp)
{
    const OT* src = reinterpret_cast<const OT*>(base) + idx;
#pragma unroll
    for (int e = 0; e < V; ++e)
        if (e < n) {
            double val = (double)fp.alpha * (double)v[e];
            if (fp.beta) val += (double)fp.beta * (double)src[e];
            v[e] = mod_canon(val, fp.p, fp.inv_p);
        }
}

// V consecutive residues of a row, kept packed as loaded (V * sizeof(RT) bytes).
template <typename RT, int V>
struct RowV {
    static constexpr int BYTES = V * (int)sizeof(RT);
    static constexpr int NQ = BYTES >= 16 ? BYTES / 16 : 1;
    int4 q[NQ];
    __device__ __forceinline__ void load(const char* base, int ld, int row, int col)
    {
        const RT* src = reinterpret_cast<const RT*>(base) + (int64_t)row * ld + col;
        if (BYTES >= 16) {
#pragma unroll
            for (int i = 0; i < NQ; ++i) q[i] = reinterpret_cast<const int4*>(src)[i];
        } else {
            const int2 v = *reinterpret_cast<const int2*>(src);
            q[0] = int4{v.x, v.y, 0, 0};
        }
    }
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int i = 0; i < NQ; ++i) q[i] = int4{0, 0, 0, 0};
    }
    __device__ __forceinline__ int32_t operator[](int e) const
    {
        return (int32_t)reinterpret_cast<const RT*>(q)[e];
    }
};

// Workgroup w of a launch runs on XCD w mod 8.  Renumbers the grid so that each
// XCD takes one contiguous range of work items: neighbouring items then share
// that XCD's L2 (a bijection of [0, total)).
__device__ __forceinline__ int xcd_contiguous(int lin, int total)
{
    const int q = total >> 3, r = total & 7;
    const int xcd = lin & 7, slot = lin >> 3;
    return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

// Lower tile pairs (R, C), R >= C, of 64 x 64 tiles of the h x h blocks; one
// workgroup of 512 threads per pair; thread = (row tr, 8-column group).  All
// loads and stores move 8 consecutive elements of a row; loaded rows stay
// packed in registers.  Tiles are renumbered per XCD so that the tiles
// sharing cache lines (narrow residues fill half a line per tile row) are
// read through one L2.
template <typename RT, typename OT, int CPLX>
__global__ void __launch_bounds__(512) postadd(const PostaddTask* tasks, Bases b, FieldParams fp)
{
    constexpr int TS = 64, V = 8;
    constexpr int NP = CPLX ? 2 : 1;
    __shared__ int32_t u1s[NP][TS][TS + 1];
    __shared__ int32_t p4s[NP][TS][TS + 1];

    const int gx = (int)gridDim.x;
    const int logical = xcd_contiguous((int)(blockIdx.y * gx + blockIdx.x), gx * (int)gridDim.y);
    const PostaddTask& T = tasks[logical / gx];
    const int h = T.h, nt = (h + TS - 1) / TS;
    const int t = logical % gx;
    int R = (int)((sqrtf(8.f * t + 1.f) - 1.f) * 0.5f);
    while ((R + 1) * (R + 2) / 2 <= t) ++R;
    while (R * (R + 1) / 2 > t) --R;
    const int C = t - R * (R + 1) / 2;
    if (R >= nt) return;
    const int p = fp.p;
    const int tr = threadIdx.x >> 3, tc = (threadIdx.x & 7) * V;
    const bool diag = (R == C);

    const int gi = R * TS + tr;          // row (within the h x h block) of tile (R, C)
    const int gj0 = C * TS + tc;         // first column of this thread in tile (R, C)
    const int mi = C * TS + tr;          // row of the mirrored tile (C, R)
    const int mj0 = R * TS + tc;

    auto plane = [&](const ResRef& rr, int q) -> const char* {
        return q == 0 ? b.p[rr.buf] + rr.off : b.p[rr.buf2] + rr.off2;
    };
    RowV<RT, V> P1[NP], P2[NP], P3[NP], P4[NP], P5[NP], Q3[NP], Q4[NP];  // Q: tiles (C, R)
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        if (gi < h && gj0 < h) {
            P1[q].load(plane(T.p[0], q), T.p[0].ld, gi, gj0);
            P2[q].load(plane(T.p[1], q), T.p[1].ld, gi, gj0);
            P3[q].load(plane(T.p[2], q), T.p[2].ld, gi, gj0);
            P4[q].load(plane(T.p[3], q), T.p[3].ld, gi, gj0);
            P5[q].load(plane(T.p[4], q), T.p[4].ld, gi, gj0);
        } else {
            P1[q].zero(); P2[q].zero(); P3[q].zero(); P4[q].zero(); P5[q].zero();
        }
        if (!diag && mi < h && mj0 < h) {
            Q3[q].load(plane(T.p[2], q), T.p[2].ld, mi, mj0);
            Q4[q].load(plane(T.p[3], q), T.p[3].ld, mi, mj0);
        } else {
            Q3[q].zero(); Q4[q].zero();
        }
    }
    // U1 = P1 + P5 on tile (R, C); stage U1 and the tile whose transpose is needed
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int e = 0; e < V; ++e) {
            u1s[q][tr][tc + e] = add_mod(P1[q][e], P5[q][e], p);
            p4s[q][tr][tc + e] = diag ? P4[q][e] : Q4[q][e];
        }
    __syncthreads();

    // the node's C: C11 at (0,0), C21 at (h,0), C22 at (h,h); rows/cols >= nvalid not written
    const int nv = T.nvalid;
    const int64_t ldc = T.c.ld;
    char* cpl[2] = {b.p[T.c.buf] + T.c.off, b.p[T.c.buf2] + T.c.off2};
    // conjugation of the imaginary plane under phi
    auto conjv = [&](int q, int32_t v) { return q == 1 ? neg_mod(v, p) : v; };
    // number of the V columns starting at col that are inside [0, lim)
    auto cnt = [](int col, int lim) { return max(0, min(V, lim - col)); };

    if (gi < h) {
        const int wantC = cnt(gj0, min(h, nv));            // C11 columns
        const int wantH = cnt(h + gj0, nv);                // C21 / C22 columns (offset h)
        const int lowlen = diag ? min(V, max(0, tr - tc + 1)) : V;  // entries with col <= row
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            int32_t c11[V], c21[V], c22[V];
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int lc = tc + e;
                // phi(Low(U1)) above the diagonal of the diagonal tile; P4^phi at (gi, gj)
                int32_t u1full = add_mod(P1[q][e], P5[q][e], p);
                if (diag && lc > tr) u1full = conjv(q, u1s[q][lc][tr]);
                const int32_t p4t = conjv(q, p4s[q][lc][tr]);
                const int32_t u2 = add_mod(u1full, P4[q][e], p);
                c21[e] = add_mod(u2, P3[q][e], p);        // U4 = U2 + P3
                c11[e] = add_mod(P1[q][e], P2[q][e], p);  // U3 = P1 + P2
                c22[e] = add_mod(u2, p4t, p);             // U5 = U2 + phi(P4)
            }
            if (T.upd) {
                // the top level of an update call: alpha U + beta C as the results are stored
                if (gi < nv) update_rowv<OT, V>(cpl[q], (int64_t)gi * ldc + gj0, c11, min(wantC, lowlen), fp);
                if (h + gi < nv) {
                    update_rowv<OT, V>(cpl[q], (int64_t)(h + gi) * ldc + gj0, c21, wantC, fp);
                    update_rowv<OT, V>(cpl[q], (int64_t)(h + gi) * ldc + h + gj0, c22, min(wantH, lowlen), fp);
                }
            }
            if (gi < nv) store_rowv<OT, V>(cpl[q], (int64_t)gi * ldc + gj0, c11, min(wantC, lowlen));
            if (h + gi < nv) {
                store_rowv<OT, V>(cpl[q], (int64_t)(h + gi) * ldc + gj0, c21, wantC);
                store_rowv<OT, V>(cpl[q], (int64_t)(h + gi) * ldc + h + gj0, c22, min(wantH, lowlen));
            }
        }
    }
    if (!diag && mi < h && h + mi < nv) {
        // tile (C, R) of C21: U1 there is phi of the staged lower tile (R, C)
        const int want = cnt(mj0, min(h, nv));
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            int32_t c21[V];
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int32_t u1 = conjv(q, u1s[q][tc + e][tr]);
                c21[e] = add_mod(add_mod(u1, Q4[q][e], p), Q3[q][e], p);
            }
            if (T.upd) update_rowv<OT, V>(cpl[q], (int64_t)(h + mi) * ldc + mj0, c21, want, fp);
            store_rowv<OT, V>(cpl[q], (int64_t)(h + mi) * ldc + mj0, c21, want);
        }
    }
}

// ============================================================================
// Strassen-Winograd operand sums and result combination
// ============================================================================

// One thread: VEC columns of one row of the h x w half-blocks; the 8 operand
// blocks are read as carriers (canonical residues), the 8 sums written back.
template <int NL, int VEC>
__global__ void __launch_bounds__(256) wino_pre(const WinoPreTask* tasks, Bases b, FieldParams fp)
{
    const WinoPreTask& T = tasks[blockIdx.y];
    const int h = T.h, w = T.w, gpr = w / VEC;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= h * gpr) return;
    const int r = idx / gpr, c = (idx % gpr) * VEC;
    const int32_t p = fp.p;
    typedef int8_t vec_t[VEC];
    // [operand (x, z)][block (11, 12, 21, 22)][limb]
    alignas(16) vec_t in[2][4][NL];
#pragma unroll
    for (int o = 0; o < 2; ++o) {
        const CarRef& a = o == 0 ? T.x : T.z;
        const char* base = b.p[a.buf] + a.off;
#pragma unroll
        for (int blk = 0; blk < 4; ++blk)
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                const char* src = base + (int64_t)l * a.ps + (int64_t)((blk >> 1) * h + r) * a.ld +
                                  (blk & 1) * w + c;
                *reinterpret_cast<int4*>(in[o][blk][l]) = *reinterpret_cast<const int4*>(src);
            }
    }
    alignas(16) vec_t out[2][4][NL];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        int32_t x[4], z[4];
#pragma unroll
        for (int blk = 0; blk < 4; ++blk) {
            x[blk] = car_canon<NL>(in[0][blk][0], in[0][blk][NL - 1], e, p);
            z[blk] = car_canon<NL>(in[1][blk][0], in[1][blk][NL - 1], e, p);
        }
        int32_t s[4], t[4];
        s[0] = add_mod(x[2], x[3], p);  // S1 = X21 + X22
        s[1] = sub_mod(s[0], x[0], p);  // S2 = S1 - X11
        s[2] = sub_mod(x[0], x[2], p);  // S3 = X11 - X21
        s[3] = sub_mod(x[1], s[1], p);  // S4 = X12 - S2
        t[0] = sub_mod(z[2], z[0], p);  // T1 = Z21 - Z11
        t[1] = sub_mod(z[3], t[0], p);  // T2 = Z22 - T1
        t[2] = sub_mod(z[3], z[2], p);  // T3 = Z22 - Z21
        t[3] = sub_mod(t[1], z[1], p);  // T4 = T2 - Z12
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            put_canon<NL>(s[j], p, fp.half, out[0][j][0], out[0][j][NL - 1], e);
            put_canon<NL>(t[j], p, fp.half, out[1][j][0], out[1][j][NL - 1], e);
        }
    }
#pragma unroll
    for (int o = 0; o < 2; ++o)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const CarRef& d = o == 0 ? T.s[j] : T.t[j];
#pragma unroll
            for (int l = 0; l < NL; ++l)
                *reinterpret_cast<int4*>(b.p[d.buf] + d.off + (int64_t)l * d.ps + (int64_t)r * d.ld + c) =
                    *reinterpret_cast<const int4*>(out[o][j][l]);
        }
}

// fp64 carrier: centred residues held as doubles, 4 consecutive columns per thread
// (w is a multiple of the 16-column k-tile, rows are 32-byte aligned).
template <typename ST>
__global__ void __launch_bounds__(256) wino_pre_f64(const WinoPreTask* tasks, Bases b, FieldParams fp)
{
    constexpr int V = 4;
    constexpr int NQ = V * (int)sizeof(ST) / 16;  // 16-byte moves per V elements
    const WinoPreTask& T = tasks[blockIdx.y];
    const int h = T.h, w = T.w, gpr = w / V;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)h * gpr) return;
    const int r = (int)(idx / gpr), c = (int)(idx % gpr) * V;
    const int32_t p = fp.p;
    auto ld = [&](const CarRef& a, int blk, int32_t* v) {
        const ST* src = reinterpret_cast<const ST*>(b.p[a.buf] + a.off) +
                        (int64_t)((blk >> 1) * h + r) * a.ld + (blk & 1) * w + c;
        alignas(16) ST t[V];
#pragma unroll
        for (int q = 0; q < NQ; ++q) reinterpret_cast<int4*>(t)[q] = reinterpret_cast<const int4*>(src)[q];
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const int32_t iv = (int32_t)t[e];
            v[e] = iv < 0 ? iv + p : iv;
        }
    };
    auto st = [&](const CarRef& d, const int32_t* v) {
        alignas(16) ST t[V];
#pragma unroll
        for (int e = 0; e < V; ++e) t[e] = (ST)(v[e] > fp.half ? v[e] - p : v[e]);
        ST* dst = reinterpret_cast<ST*>(b.p[d.buf] + d.off) + (int64_t)r * d.ld + c;
#pragma unroll
        for (int q = 0; q < NQ; ++q) reinterpret_cast<int4*>(dst)[q] = reinterpret_cast<const int4*>(t)[q];
    };
    int32_t x[4][V], z[4][V];
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) {
        ld(T.x, blk, x[blk]);
        ld(T.z, blk, z[blk]);
    }
    int32_t s[4][V], t[4][V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
        s[0][e] = add_mod(x[2][e], x[3][e], p);
        s[1][e] = sub_mod(s[0][e], x[0][e], p);
        s[2][e] = sub_mod(x[0][e], x[2][e], p);
        s[3][e] = sub_mod(x[1][e], s[1][e], p);
        t[0][e] = sub_mod(z[2][e], z[0][e], p);
        t[1][e] = sub_mod(z[3][e], t[0][e], p);
        t[2][e] = sub_mod(z[3][e], z[2][e], p);
        t[3][e] = sub_mod(t[1][e], z[1][e], p);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        st(T.s[j], s[j]);
        st(T.t[j], t[j]);
    }
}

// One thread: 8 consecutive columns of one row of the h x h results, vector
// loads of the seven products; the four blocks of C (vector stores where aligned).
template <typename RT>
__global__ void __launch_bounds__(256) wino_post(const WinoPostTask* tasks, Bases b, FieldParams fp)
{
    constexpr int V = 8;
    const WinoPostTask& T = tasks[blockIdx.y];
    const int h = T.h, gpr = (h + V - 1) / V;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= h * gpr) return;
    const int r = idx / gpr, c0 = (idx % gpr) * V;
    const int32_t p = fp.p;
    // residue rows are padded to a multiple of 64 elements: whole groups are inside them
    RowV<RT, V> R[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) R[q].load(b.p[T.r[q].buf] + T.r[q].off, T.r[q].ld, r, c0);
    int32_t c11[V], c12[V], c21[V], c22[V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
        const int32_t u2 = add_mod(R[0][e], R[5][e], p), u3 = add_mod(u2, R[6][e], p);
        const int32_t u4 = add_mod(u2, R[4][e], p);
        c11[e] = add_mod(R[0][e], R[1][e], p);  // C11 = R1 + R2
        c12[e] = add_mod(u4, R[2][e], p);       // C12 = U4 + R3
        c21[e] = sub_mod(u3, R[3][e], p);       // C21 = U3 - R4
        c22[e] = add_mod(u3, R[4][e], p);       // C22 = U3 + R5
    }
    const int want = min(V, h - c0);
    char* cb = b.p[T.c.buf] + T.c.off;
    const int64_t ldc = T.c.ld;
    store_rowv<RT, V>(cb, (int64_t)r * ldc + c0, c11, want);
    store_rowv<RT, V>(cb, (int64_t)r * ldc + h + c0, c12, want);
    store_rowv<RT, V>(cb, (int64_t)(h + r) * ldc + c0, c21, want);
    store_rowv<RT, V>(cb, (int64_t)(h + r) * ldc + h + c0, c22, want);
}

// ============================================================================
// transposed conditioning and the final update C <- alpha X + beta C
// ============================================================================

// Canonical residue of one caller element (range-checked).
template <typename IT>
__device__ __forceinline__ int32_t canon_in(IT raw, int32_t p, int32_t half, bool centred, bool& ok)
{
    if (centred) {
        const int32_t x = (int32_t)raw;
        ok &= (x >= -half) & (x <= half);
        return x < 0 ? x + p : x;
    }
    const double xd = (double)raw;
    const int32_t x = (int32_t)raw;
    ok &= (xd >= 0.0) & (xd < (double)p) & ((double)x == xd);
    return x;
}

// Carrier tile of 64 x 64 from the transpose of the caller's k x n matrix: the
// block of A rows C0.. (carrier columns) and A columns R0.. (carrier rows) is
// read row by row into LDS and written out transposed, 16 carrier columns per
// thread.  Carrier: NL int8 limbs (F64C = 0) or centred doubles (F64C = 1).
template <typename IT, int NL, int F64C>
__global__ void __launch_bounds__(256) condition_t(const CondTask* tasks, Bases b, FieldParams fp,
                                                   int32_t* err)
{
    __shared__ int32_t tile[64][65];
    const CondTask& t = tasks[blockIdx.y];
    const int tcols = (t.kpad + 63) / 64;
    const int ntile = ((t.npad + 63) / 64) * tcols;
    if ((int)blockIdx.x >= ntile) return;
    const int R0 = ((int)blockIdx.x / tcols) * 64, C0 = ((int)blockIdx.x % tcols) * 64;
    const IT* A = reinterpret_cast<const IT*>(b.p[t.buf_re] + t.off_re);
    const int p = fp.p, half = fp.half;
    const bool centred = t.dt_in == DT_I8C;
    const int tid = threadIdx.x;
    bool ok = true;
    {
        const int ar = tid >> 2, ac = (tid & 3) * 16;
        const int arow = C0 + ar;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int acol = R0 + ac + e;
            int32_t v = 0;
            if (arow < t.k && acol < t.n) v = canon_in<IT>(A[(int64_t)arow * t.lda + acol], p, half, centred, ok);
            tile[ar][ac + e] = v;
        }
    }
    if (!ok) err[0] = 1;
    __syncthreads();
    const int cr = tid >> 2, cc = (tid & 3) * 16;
    const int crow = R0 + cr, ccol = C0 + cc;
    if (crow >= t.npad || ccol >= t.kpad) return;
    char* ob = b.p[t.out.buf] + t.out.off;
    if (F64C) {
        alignas(16) double out[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int32_t v = tile[cc + e][cr];
            out[e] = (double)(v > half ? v - p : v);
        }
        double* dst = reinterpret_cast<double*>(ob) + (int64_t)crow * t.out.ld + ccol;
#pragma unroll
        for (int q = 0; q < 8; ++q) reinterpret_cast<int4*>(dst)[q] = reinterpret_cast<const int4*>(out)[q];
    } else {
        alignas(16) int8_t out[NL][16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int32_t v = tile[cc + e][cr];
            if (NL == 1) {
                out[0][e] = (int8_t)(v > half ? v - p : v);
            } else {
                int8_t hi, lo;
                split2(rep2(v, p), hi, lo);
                out[0][e] = hi;
                out[NL - 1][e] = lo;
            }
        }
#pragma unroll
        for (int l = 0; l < NL; ++l)
            *reinterpret_cast<int4*>(ob + (int64_t)l * t.out.ps + (int64_t)crow * t.out.ld + ccol) =
                *reinterpret_cast<const int4*>(out[l]);
    }
}

// 2M base case: tile (R, C), R >= C, of 64 x 64 of a leaf's lower triangle, one
// workgroup of 256 threads (row tr, 16 columns), 16-element vector loads and
// stores; the mirrored tile of H is read transposed through LDS.
template <typename RT, typename OT>
__global__ void __launch_bounds__(256) herk2m_combine(const Herk2mTask* tasks, Bases b, FieldParams fp)
{
    constexpr int TS = 64, V = 16;
    __shared__ int32_t ht[TS][TS + 1];
    const Herk2mTask& T = tasks[blockIdx.y];
    const int n = T.n, nt = (n + TS - 1) / TS;
    const int t = blockIdx.x;
    int R = (int)((sqrtf(8.f * t + 1.f) - 1.f) * 0.5f);
    while ((R + 1) * (R + 2) / 2 <= t) ++R;
    while (R * (R + 1) / 2 > t) --R;
    const int C = t - R * (R + 1) / 2;
    if (R >= nt) return;
    const int p = fp.p;
    const int tr = threadIdx.x >> 2, tc = (threadIdx.x & 3) * V;
    const char* gb = b.p[T.g.buf] + T.g.off;
    const char* hb = b.p[T.h.buf] + T.h.off;
    const char* h2b = b.p[T.h2.buf] + T.h2.off;  // second half of H over K (split)
    const bool split = T.split != 0;
    // H on the mirrored tile (C, R): row C*TS + tr, columns R*TS + tc ..; the
    // residue matrices have ld a multiple of 64, so whole 16-element groups are in
    // bounds of the allocation (entries past n are never used)
    {
        const int mi = C * TS + tr;
        RowV<RT, V> hm, hm2;
        if (mi < n) {
            hm.load(hb, T.h.ld, mi, R * TS + tc);
            if (split) hm2.load(h2b, T.h2.ld, mi, R * TS + tc);
            else hm2.zero();
        } else {
            hm.zero();
            hm2.zero();
        }
#pragma unroll
        for (int e = 0; e < V; ++e) ht[tr][tc + e] = split ? add_mod(hm[e], hm2[e], p) : hm[e];
    }
    __syncthreads();
    const int i = R * TS + tr, j0 = C * TS + tc;
    const int lim = min(n, T.nvalid);
    if (i >= lim || j0 > i) return;
    RowV<RT, V> g, h, h2;
    g.load(gb, T.g.ld, i, j0);
    h.load(hb, T.h.ld, i, j0);
    if (split) h2.load(h2b, T.h2.ld, i, j0);
    else h2.zero();
    int32_t re[V], im[V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
        const int32_t hji = ht[tc + e][tr];  // H[j][i]
        const int32_t hij = split ? add_mod(h[e], h2[e], p) : h[e];
        re[e] = sub_mod(sub_mod(g[e], hij, p), hji, p);  // Re = G - H - H^T
        im[e] = sub_mod(hji, hij, p);                    // Im = H^T - H
    }
    const int want = min(V, min(lim, i + 1) - j0);  // columns j <= i inside the leaf
    char* ore = b.p[T.out.buf] + T.out.off;
    char* oim = b.p[T.out.buf2] + T.out.off2;
    store_rowv<OT, V>(ore, (int64_t)i * T.out.ld + j0, re, want);
    store_rowv<OT, V>(oim, (int64_t)i * T.out.ld + j0, im, want);
}

// C <- alpha X + beta C on the lower triangle; one thread per 8 columns of a row.
template <typename RT, typename OT>
__global__ void __launch_bounds__(256) update_c(const UpdateTask* tasks, Bases b, FieldParams fp)
{
    const UpdateTask& t = tasks[blockIdx.y];
    const int n = t.n, gpr = (n + 7) / 8;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)n * gpr) return;
    const int i = (int)(idx / gpr), j0 = (int)(idx % gpr) * 8;
    if (j0 > i) return;
    const RT* x = reinterpret_cast<const RT*>(b.p[t.x.buf] + t.x.off) + (int64_t)i * t.x.ld;
    OT* c = reinterpret_cast<OT*>(b.p[t.c.buf] + t.c.off) + (int64_t)i * t.c.ld;
    const int p = fp.p;
    const double al = (double)fp.alpha, be = (double)fp.beta;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int j = j0 + e;
        if (j > i) break;
        // alpha x + beta c < 2^53 for p < 2^26: exact in fp64
        // beta = 0: C is not read (it may hold anything)
        const double cv = fp.beta ? be * (double)(int64_t)c[j] : 0.0;
        const double v = al * (double)(int64_t)x[j] + cv;
        c[j] = (OT)mod_canon(v, p, fp.inv_p);
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

template <typename IT>
static void launch_cond_typed(dim3 g, hipStream_t s, const CondTask* d_tasks, int ntasks, const Bases& b,
                              const FieldParams& fp, int32_t* d_err)
{
    if (fp.nl == 1 && !fp.cplx)
        hipLaunchKernelGGL((condition_i8<IT, 1, 0>), g, dim3(256), 0, s, d_tasks, ntasks, b, fp, d_err);
    else if (fp.nl == 2 && !fp.cplx)
        hipLaunchKernelGGL((condition_i8<IT, 2, 0>), g, dim3(256), 0, s, d_tasks, ntasks, b, fp, d_err);
    else if (fp.nl == 1)
        hipLaunchKernelGGL((condition_i8<IT, 1, 1>), g, dim3(256), 0, s, d_tasks, ntasks, b, fp, d_err);
    else
        hipLaunchKernelGGL((condition_i8<IT, 2, 1>), g, dim3(256), 0, s, d_tasks, ntasks, b, fp, d_err);
}

int launch_condition(const CondTask* d_tasks, int ntasks, int nblocks, int dt_in, const Bases& b,
                     const FieldParams& fp, int carrier, int32_t* d_err, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (ntasks <= 0 || nblocks <= 0) return 0;
    const dim3 g(nblocks);
    if (carrier == CAR_F64) {
        if (fp.st32) hipLaunchKernelGGL(condition_f64<float>, g, dim3(256), 0, s, d_tasks, ntasks, b, fp, d_err);
        else hipLaunchKernelGGL(condition_f64<double>, g, dim3(256), 0, s, d_tasks, ntasks, b, fp, d_err);
    } else {
        switch (dt_in) {
        case DT_I8C: launch_cond_typed<int8_t>(g, s, d_tasks, ntasks, b, fp, d_err); break;
        case DT_U8: launch_cond_typed<uint8_t>(g, s, d_tasks, ntasks, b, fp, d_err); break;
        case DT_U16: launch_cond_typed<uint16_t>(g, s, d_tasks, ntasks, b, fp, d_err); break;
        case DT_I32: launch_cond_typed<int32_t>(g, s, d_tasks, ntasks, b, fp, d_err); break;
        case DT_I64: launch_cond_typed<int64_t>(g, s, d_tasks, ntasks, b, fp, d_err); break;
        case DT_F64: launch_cond_typed<double>(g, s, d_tasks, ntasks, b, fp, d_err); break;
        default: return (int)hipErrorInvalidValue;
        }
    }
    return (int)hipGetLastError();
}

int launch_preadd_signal(const PreaddTask* d_tasks, int ntasks, int h, int w, const Bases& b,
                         const FieldParams& fp, int blocks, int64_t counter_off, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (ntasks <= 0 || h <= 0 || w <= 0 || (w / 2) % 16 || fp.nl != 1 || fp.cplx) return (int)hipErrorInvalidValue;
    const dim3 g((unsigned)blocks, ntasks);
    if (fp.ykind == Y_BLOCKS)
        hipLaunchKernelGGL((preadd_c1_signal<Y_BLOCKS>), g, dim3(256), 0, s, d_tasks, b, fp, counter_off);
    else
        hipLaunchKernelGGL((preadd_c1_signal<Y_SCALAR>), g, dim3(256), 0, s, d_tasks, b, fp, counter_off);
    return (int)hipGetLastError();
}

int launch_zero_words(const Bases& b, int64_t off, int words, void* stream)
{
    if (words <= 0) return 0;
    hipLaunchKernelGGL(zero_words, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, (hipStream_t)stream, b,
                       off, words);
    return (int)hipGetLastError();
}

int preadd_signal_regs(int* vgprs, int* threads)
{
    hipFuncAttributes a{};
    hipError_t e = hipFuncGetAttributes(&a, (const void*)preadd_c1_signal<Y_BLOCKS>);
    if (e != hipSuccess) return (int)e;
    hipFuncAttributes a2{};
    e = hipFuncGetAttributes(&a2, (const void*)preadd_c1_signal<Y_SCALAR>);
    if (e != hipSuccess) return (int)e;
    *vgprs = std::max(a.numRegs, a2.numRegs);
    *threads = 256;
    return 0;
}

int launch_preadd(const PreaddTask* d_tasks, int ntasks, int h, int w, const Bases& b,
                  const FieldParams& fp, int carrier, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (ntasks <= 0 || h <= 0 || w <= 0) return 0;
    if (carrier == CAR_F64) {
        const int64_t total = (int64_t)h * (w / 2);
        const dim3 g((unsigned)((total + 255) / 256), ntasks);
        if (fp.st32) hipLaunchKernelGGL(preadd_f64<float>, g, dim3(256), 0, s, d_tasks, b, fp);
        else hipLaunchKernelGGL(preadd_f64<double>, g, dim3(256), 0, s, d_tasks, b, fp);
    } else if (!fp.cplx) {
        if (fp.nl == 1) {
            // one limb: centred arithmetic throughout; 16 columns per thread when every
            // half-row holds whole 16-byte groups (w / 2 is a multiple of the k-tile)
            const bool v16 = (w / 2) % 16 == 0;
            const int vec = v16 ? 16 : 8;
            const dim3 g((unsigned)(((int64_t)h * (w / 2 / vec) + 255) / 256), ntasks);
            if (fp.ykind == Y_BLOCKS) {
                if (v16) hipLaunchKernelGGL((preadd_c1<Y_BLOCKS, 16>), g, dim3(256), 0, s, d_tasks, b, fp);
                else hipLaunchKernelGGL((preadd_c1<Y_BLOCKS, 8>), g, dim3(256), 0, s, d_tasks, b, fp);
            } else {
                if (v16) hipLaunchKernelGGL((preadd_c1<Y_SCALAR, 16>), g, dim3(256), 0, s, d_tasks, b, fp);
                else hipLaunchKernelGGL((preadd_c1<Y_SCALAR, 8>), g, dim3(256), 0, s, d_tasks, b, fp);
            }
        } else {
            const int64_t t8 = (int64_t)h * (w / 2 / 8);
            hipLaunchKernelGGL((preadd_i8<2, 0, 8>), dim3((unsigned)((t8 + 255) / 256), ntasks),
                               dim3(256), 0, s, d_tasks, b, fp);
        }
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
    case DT_U8: hipLaunchKernelGGL((postadd<RT, uint8_t, CPLX>), g, dim3(512), 0, s, d_tasks, b, fp); break;
    case DT_U16: hipLaunchKernelGGL((postadd<RT, uint16_t, CPLX>), g, dim3(512), 0, s, d_tasks, b, fp); break;
    case DT_I32: hipLaunchKernelGGL((postadd<RT, int32_t, CPLX>), g, dim3(512), 0, s, d_tasks, b, fp); break;
    case DT_I64: hipLaunchKernelGGL((postadd<RT, int64_t, CPLX>), g, dim3(512), 0, s, d_tasks, b, fp); break;
    case DT_F64: hipLaunchKernelGGL((postadd<RT, double, CPLX>), g, dim3(512), 0, s, d_tasks, b, fp); break;
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

template <typename IT>
static void launch_cond_t_typed(dim3 g, hipStream_t s, const CondTask* d_tasks, const Bases& b,
                                const FieldParams& fp, int carrier, int32_t* d_err)
{
    if (carrier == CAR_F64)
        hipLaunchKernelGGL((condition_t<IT, 1, 1>), g, dim3(256), 0, s, d_tasks, b, fp, d_err);
    else if (fp.nl == 1)
        hipLaunchKernelGGL((condition_t<IT, 1, 0>), g, dim3(256), 0, s, d_tasks, b, fp, d_err);
    else
        hipLaunchKernelGGL((condition_t<IT, 2, 0>), g, dim3(256), 0, s, d_tasks, b, fp, d_err);
}

int launch_condition_trans(const CondTask* d_tasks, int ntasks, int max_tiles, int dt_in, const Bases& b,
                           const FieldParams& fp, int carrier, int32_t* d_err, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (ntasks <= 0 || max_tiles <= 0) return 0;
    if (fp.cplx) return (int)hipErrorInvalidValue;
    const dim3 g(max_tiles, ntasks);
    switch (dt_in) {
    case DT_I8C: launch_cond_t_typed<int8_t>(g, s, d_tasks, b, fp, carrier, d_err); break;
    case DT_U8: launch_cond_t_typed<uint8_t>(g, s, d_tasks, b, fp, carrier, d_err); break;
    case DT_U16: launch_cond_t_typed<uint16_t>(g, s, d_tasks, b, fp, carrier, d_err); break;
    case DT_I32: launch_cond_t_typed<int32_t>(g, s, d_tasks, b, fp, carrier, d_err); break;
    case DT_I64: launch_cond_t_typed<int64_t>(g, s, d_tasks, b, fp, carrier, d_err); break;
    case DT_F64: launch_cond_t_typed<double>(g, s, d_tasks, b, fp, carrier, d_err); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

int launch_wino_pre(const WinoPreTask* d_tasks, int ntasks, int max_h, int max_w, const Bases& b,
                    const FieldParams& fp, int carrier, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (ntasks <= 0 || max_h <= 0 || max_w <= 0) return 0;
    if (carrier == CAR_F64) {
        const int64_t total = (int64_t)max_h * (max_w / 4);
        const dim3 g((unsigned)((total + 255) / 256), ntasks);
        if (fp.st32) hipLaunchKernelGGL(wino_pre_f64<float>, g, dim3(256), 0, s, d_tasks, b, fp);
        else hipLaunchKernelGGL(wino_pre_f64<double>, g, dim3(256), 0, s, d_tasks, b, fp);
    } else {
        const int64_t total = (int64_t)max_h * (max_w / 16);
        const dim3 g((unsigned)((total + 255) / 256), ntasks);
        if (fp.nl == 1) hipLaunchKernelGGL((wino_pre<1, 16>), g, dim3(256), 0, s, d_tasks, b, fp);
        else hipLaunchKernelGGL((wino_pre<2, 16>), g, dim3(256), 0, s, d_tasks, b, fp);
    }
    return (int)hipGetLastError();
}

int launch_wino_post(const WinoPostTask* d_tasks, int ntasks, int max_h, const Bases& b,
                     const FieldParams& fp, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (ntasks <= 0 || max_h <= 0) return 0;
    const int64_t total = (int64_t)max_h * ((max_h + 7) / 8);
    const dim3 g((unsigned)((total + 255) / 256), ntasks);
    if (fp.p < 256) hipLaunchKernelGGL((wino_post<uint8_t>), g, dim3(256), 0, s, d_tasks, b, fp);
    else if (fp.p < 65536) hipLaunchKernelGGL((wino_post<uint16_t>), g, dim3(256), 0, s, d_tasks, b, fp);
    else hipLaunchKernelGGL((wino_post<int32_t>), g, dim3(256), 0, s, d_tasks, b, fp);
    return (int)hipGetLastError();
}

template <typename RT>
static int launch_herk2m_rt(dim3 g, hipStream_t s, const Herk2mTask* d, int out_dt, const Bases& b,
                            const FieldParams& fp)
{
    switch (out_dt) {
    case DT_U8: hipLaunchKernelGGL((herk2m_combine<RT, uint8_t>), g, dim3(256), 0, s, d, b, fp); break;
    case DT_U16: hipLaunchKernelGGL((herk2m_combine<RT, uint16_t>), g, dim3(256), 0, s, d, b, fp); break;
    case DT_I32: hipLaunchKernelGGL((herk2m_combine<RT, int32_t>), g, dim3(256), 0, s, d, b, fp); break;
    case DT_I64: hipLaunchKernelGGL((herk2m_combine<RT, int64_t>), g, dim3(256), 0, s, d, b, fp); break;
    case DT_F64: hipLaunchKernelGGL((herk2m_combine<RT, double>), g, dim3(256), 0, s, d, b, fp); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

int launch_herk2m(const Herk2mTask* d_tasks, int ntasks, int max_n, int res_dt, int out_dt,
                  const Bases& b, const FieldParams& fp, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (ntasks <= 0 || max_n <= 0) return 0;
    const int nt = (max_n + 63) / 64;
    const dim3 g((unsigned)(nt * (nt + 1) / 2), ntasks);
    switch (res_dt) {
    case DT_U8: return launch_herk2m_rt<uint8_t>(g, s, d_tasks, out_dt, b, fp);
    case DT_U16: return launch_herk2m_rt<uint16_t>(g, s, d_tasks, out_dt, b, fp);
    case DT_I32: return launch_herk2m_rt<int32_t>(g, s, d_tasks, out_dt, b, fp);
    default: return (int)hipErrorInvalidValue;
    }
}

// Sum of the K-pieces of split product tiles: blockIdx.y picks the task, and the
// workgroups of its row stride over the tile in 16-byte chunks of consecutive
// columns (element by element where the output rows are not 16-byte aligned or
// the width is not a multiple of a chunk).  Pieces and output share the element
// format T (canonical residues, exact in every format); piece rows are 16-byte
// aligned by construction.
template <typename T>
__global__ void __launch_bounds__(256) tail_sum(const TailTask* tasks, Bases b, FieldParams fp)
{
    constexpr int E = 16 / (int)sizeof(T);
    const TailTask& t = tasks[blockIdx.y];
    const char* pb = b.p[t.part.buf] + t.part.off;
    T* out = reinterpret_cast<T*>(b.p[t.out.buf] + t.out.off);
    const int stride = gridDim.x * blockDim.x;
    const int first = blockIdx.x * blockDim.x + threadIdx.x;
    const bool vec = ((((uintptr_t)out) | (uintptr_t)(t.out.ld * (int64_t)sizeof(T))) & 15) == 0 &&
                     t.cols % E == 0 && (t.part.ld * (int)sizeof(T)) % 16 == 0 && ((t.part.off | t.pstride) & 15) == 0;
    if (vec) {
        const int cpr = t.cols / E;
        for (int i = first; i < t.rows * cpr; i += stride) {
            const int r = i / cpr, c0 = (i - r * cpr) * E;
            int32_t v[E];
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = 0;
            for (int q = 0; q < t.nparts; ++q) {
                alignas(16) T x[E];
                *reinterpret_cast<int4*>(x) = *reinterpret_cast<const int4*>(
                    pb + q * t.pstride + ((int64_t)r * t.part.ld + c0) * (int64_t)sizeof(T));
#pragma unroll
                for (int e = 0; e < E; ++e) v[e] = add_mod(v[e], (int32_t)x[e], fp.p);
            }
            alignas(16) T y[E];
#pragma unroll
            for (int e = 0; e < E; ++e) y[e] = (T)v[e];
            *reinterpret_cast<int4*>(out + (int64_t)r * t.out.ld + c0) = *reinterpret_cast<const int4*>(y);
        }
        return;
    }
    for (int i = first; i < t.rows * t.cols; i += stride) {
        const int r = i / t.cols, c = i - r * t.cols;
        int32_t v = 0;
        for (int q = 0; q < t.nparts; ++q)
            v = add_mod(v, (int32_t)reinterpret_cast<const T*>(pb + q * t.pstride)[(int64_t)r * t.part.ld + c], fp.p);
        out[(int64_t)r * t.out.ld + c] = (T)v;
    }
}

// max_rows: the most rows of any task (the tile edge)
int launch_tail_sum(const TailTask* d_tasks, int ntasks, int max_rows, int dt, const Bases& b,
                    const FieldParams& fp, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (ntasks <= 0 || max_rows <= 0) return 0;
    // one 16-byte chunk per thread for 8-bit tiles; wider formats loop
    const dim3 g((unsigned)(((int64_t)max_rows * max_rows / 16 + 255) / 256), ntasks);
    switch (dt) {
    case DT_U8: hipLaunchKernelGGL((tail_sum<uint8_t>), g, dim3(256), 0, s, d_tasks, b, fp); break;
    case DT_U16: hipLaunchKernelGGL((tail_sum<uint16_t>), g, dim3(256), 0, s, d_tasks, b, fp); break;
    case DT_I32: hipLaunchKernelGGL((tail_sum<int32_t>), g, dim3(256), 0, s, d_tasks, b, fp); break;
    case DT_I64: hipLaunchKernelGGL((tail_sum<int64_t>), g, dim3(256), 0, s, d_tasks, b, fp); break;
    case DT_F64: hipLaunchKernelGGL((tail_sum<double>), g, dim3(256), 0, s, d_tasks, b, fp); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

template <typename RT>
static int launch_update_rt(dim3 g, hipStream_t s, const UpdateTask* d, int c_dt, const Bases& b,
                            const FieldParams& fp)
{
    switch (c_dt) {
    case DT_U8: hipLaunchKernelGGL((update_c<RT, uint8_t>), g, dim3(256), 0, s, d, b, fp); break;
    case DT_U16: hipLaunchKernelGGL((update_c<RT, uint16_t>), g, dim3(256), 0, s, d, b, fp); break;
    case DT_I32: hipLaunchKernelGGL((update_c<RT, int32_t>), g, dim3(256), 0, s, d, b, fp); break;
    case DT_I64: hipLaunchKernelGGL((update_c<RT, int64_t>), g, dim3(256), 0, s, d, b, fp); break;
    case DT_F64: hipLaunchKernelGGL((update_c<RT, double>), g, dim3(256), 0, s, d, b, fp); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

int launch_update(const UpdateTask* d_tasks, int ntasks, int max_n, int x_dt, int c_dt, const Bases& b,
                  const FieldParams& fp, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (ntasks <= 0 || max_n <= 0) return 0;
    const int64_t threads = (int64_t)max_n * ((max_n + 7) / 8);
    const dim3 g((unsigned)((threads + 255) / 256), ntasks);
    switch (x_dt) {
    case DT_U8: return launch_update_rt<uint8_t>(g, s, d_tasks, c_dt, b, fp);
    case DT_U16: return launch_update_rt<uint16_t>(g, s, d_tasks, c_dt, b, fp);
    case DT_I32: return launch_update_rt<int32_t>(g, s, d_tasks, c_dt, b, fp);
    default: return (int)hipErrorInvalidValue;
    }
}

}  // namespace ffa
