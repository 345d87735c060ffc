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

// Centred residue in [-(p-1)/2, (p-1)/2] of a small integer (|x| < 2^20) for p < 2^11.
__device__ __forceinline__ int32_t mod_centred_small(int32_t x, int32_t p, float inv_p)
{
    int32_t q = (int32_t)rintf((float)x * inv_p);
    return x - q * p;
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
