// Device helpers shared by the HIP kernels: modular reduction, carrier
// encodings, residue loads and stores.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ffa_internal.h"

namespace ffa {

// Two-limb carrier: a residue is represented by r in [REP_MAX - p + 1, REP_MAX]
// and split as r = 256 * hi + lo with hi, lo in [-128, 127].  Two balanced
// int8 limbs cover exactly [-32896, 32639].
constexpr int32_t REP_MAX2 = 32639;

// Canonical residue of an exact integer held in a double (|v| < 2^53).
__device__ __forceinline__ int32_t mod_canon(double v, int32_t p, double inv_p)
{
    double q = floor(v * inv_p);
    int32_t r = (int32_t)(v - q * (double)p);  // exact; within one p of [0, p)
    r += (r < 0) ? p : 0;
    r -= (r >= p) ? p : 0;
    return r;
}

// Centred residue in [-(p-1)/2, (p-1)/2] of a small integer (|x| < 2^20) for odd
// p < 2^11, in five full-rate fp32 operations, all exact except the one rounding
// that is meant: the fused multiply-add of fp32(x) (exact) by fp32(1/p) with
// 1.5 * 2^23 rounds once to an integer (its ulp there is 1), and before that
// rounding it is within |x| 2^-24 / p < 1 / (2p) of x / p, which is at least
// 1 / (2p) away from every half-integer (p odd); so q = round(x / p).  Then
// q (Sterbenz) and x - q p (an integer below p in magnitude) are exact in fp32.
__device__ __forceinline__ int32_t mod_centred_small(int32_t x, int32_t p, float inv_p)
{
    constexpr float MAGIC = 12582912.0f;  // 1.5 * 2^23
    const float xf = (float)x;
    const float q = __builtin_fmaf(xf, inv_p, MAGIC) - MAGIC;
    return (int32_t)__builtin_fmaf(-q, (float)p, xf);
}

// c + a * b for 24-bit signed a, b, with b the same in every lane (one full-rate
// v_mad_i32_i24 reading b from a scalar register).  Written as an instruction
// because the compiler, seeing that only the low bits of a result are used (a
// residue stored as a byte), would otherwise turn the 24-bit multiply into a
// quarter-rate 32-bit one.
__device__ __forceinline__ int32_t mad24_s(int32_t a, int32_t b_uniform, int32_t c)
{
    int32_t r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b_uniform), "v"(c));
    return r;
}

// Centred residue of |v| <= 3 (p - 1) / 2 (a sum of up to three centred residues)
// for odd p < 2^8, with r20 = round(2^20 / p): q = floor((v r20 + 2^19) / 2^20)
// differs from v / p + 1/2 by at most |v| / 2^21 < 2^-12, less than the distance
// 1 / (2p) from v / p + 1/2 to the nearest integer, so q = round(v / p) exactly.
// Three 24-bit operations.
__device__ __forceinline__ int32_t cen_short(int32_t v, int32_t p, int32_t r20)
{
    const int32_t q = (__mul24(v, r20) + (1 << 19)) >> 20;
    return mad24_s(q, -p, v);
}

// Canonical residue of an unsigned 32-bit integer for odd p < 2^16, with two
// fp32 quotient estimates (the first is within a few hundred of x / p, the
// second exact to within one) and a final correction.
__device__ __forceinline__ int32_t mod_u32(uint32_t x, int32_t p, float inv_p)
{
    int32_t q = (int32_t)((float)x * inv_p);
    int32_t r = (int32_t)(x - (uint32_t)q * (uint32_t)p);
    q = (int32_t)floorf((float)r * inv_p);
    r -= q * p;
    r += (r < 0) ? p : 0;
    r -= (r >= p) ? p : 0;
    return r;
}

// a * b mod p for canonical a, b (p < 2^16: the product fits in 32 bits).
__device__ __forceinline__ int32_t mul_mod(int32_t a, int32_t b, int32_t p, float inv_p)
{
    return mod_u32((uint32_t)a * (uint32_t)b, p, inv_p);
}

__device__ __forceinline__ int32_t sub_mod(int32_t a, int32_t b, int32_t p)
{
    const int32_t d = a - b;
    return d < 0 ? d + p : d;
}

// a + b mod p for canonical a, b.
__device__ __forceinline__ int32_t add_mod(int32_t a, int32_t b, int32_t p)
{
    int32_t s = a + b;
    return s >= p ? s - p : s;
}

__device__ __forceinline__ int32_t neg_mod(int32_t a, int32_t p)
{
    return a == 0 ? 0 : p - a;
}

// Representative of a canonical residue for the two-limb carrier.
__device__ __forceinline__ int32_t rep2(int32_t c, int32_t p)
{
    return c > REP_MAX2 ? c - p : c;
}

__device__ __forceinline__ void split2(int32_t r, int8_t& hi, int8_t& lo)
{
    int32_t h = (r + 128) >> 8;  // arithmetic shift: floor division
    hi = (int8_t)h;
    lo = (int8_t)(r - 256 * h);
}

// Bounded wait (one thread of a workgroup) for the int32 counter at p to reach
// target.  The counter is raised, with release ordering at device scope, by the
// workgroups of a kernel that runs beside the waiting one and writes its operands.
// The waiting workgroup has read none of those operands before (its kernel's
// start invalidated the caches of data written earlier), so after the wait its
// loads see the written values.  After about a second of waiting the status word
// err (the context's) is set to 1 and the wait ends; the result of that call is
// then not valid, which ffa_device_status reports.
constexpr uint32_t WAIT_SPINS = 1u << 22;  // s_sleep of 8 x 64 cycles each

__device__ __forceinline__ void wait_counter(char* p, int32_t target, int32_t* err)
{
    int32_t* cnt = reinterpret_cast<int32_t*>(p);
    for (uint32_t i = 0;; ++i) {
        if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
        if (i >= WAIT_SPINS) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(8);
    }
}

// Residue stores and loads in the storage formats of ffa_internal.h.
__device__ __forceinline__ void store_res(char* base, int dt, int64_t idx, int32_t v)
{
    switch (dt) {
    case DT_U8: reinterpret_cast<uint8_t*>(base)[idx] = (uint8_t)v; break;
    case DT_U16: reinterpret_cast<uint16_t*>(base)[idx] = (uint16_t)v; break;
    case DT_I32: reinterpret_cast<int32_t*>(base)[idx] = v; break;
    case DT_I64: reinterpret_cast<int64_t*>(base)[idx] = (int64_t)v; break;
    case DT_F64: reinterpret_cast<double*>(base)[idx] = (double)v; break;
    default: break;
    }
}

}  // namespace ffa
