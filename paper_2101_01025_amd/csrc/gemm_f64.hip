// Grouped product kernel on FP64 MFMA (gfx950 v_mfma_f64_16x16x4_f64) used as
// an exact integer carrier: operands are centred residues held in doubles and
// every partial sum is an integer below 2^53 (the planner checks
// K * ((p-1)/2)^2 < 2^53), so the fused multiply-adds are exact and a single
// reduction mod p per output ends the product.
//
// Same task table as the INT8 kernel (general products of every level and the
// base-case lower-triangle products in one launch).  LDS rows hold 16 doubles
// of K; element k of row r sits at position k ^ (r & 15) so that the 8-byte
// fragment reads of 16 consecutive rows hit distinct banks.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.h"
#include "ffa_internal.h"

namespace ffa {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

constexpr int KTD = 16;  // doubles of K per pipeline stage

// Two waves per SIMD (two workgroups per CU, bounded by LDS as well): the compiler
// then keeps the accumulators in ordinary VGPRs (212 of 256) instead of spreading
// 330 registers over VGPRs and AGPRs at one wave per SIMD, and the second wave
// hides the fragment-read and barrier latency of the first (products 8.48 -> 6.18 ms
// at n = k = 8192, four levels).
// ST: operand storage, double or float (exact integers below 2^24, widened to
// double on the way into LDS; LDS and the MFMAs always hold doubles).
template <int BT, int WGM, int WGN, typename ST>
__global__ void __launch_bounds__(WGM* WGN * 64) __attribute__((amdgpu_waves_per_eu(2, 2)))
    gemm_f64(Bases bases, const GemmTask* __restrict__ tasks, const TileEnt* __restrict__ sched,
             FieldParams fp)
{
    constexpr int NT = WGM * WGN * 64;
    constexpr int WM = BT / WGM, WN = BT / WGN;
    constexpr int FM = WM / 16, FN = WN / 16;
    constexpr int TILE = BT * KTD;  // doubles
    constexpr int STAGE = 2 * TILE;
    constexpr int EPC = 16 / (int)sizeof(ST);  // elements per 16-byte chunk (2 or 4)
    constexpr int CH = BT * (KTD / EPC) / NT;  // 16-byte chunks per thread per operand
    static_assert(BT * (KTD / EPC) % NT == 0, "chunking");

    extern __shared__ __attribute__((aligned(16))) char lds_raw[];
    double* lds = reinterpret_cast<double*>(lds_raw);

    const TileEnt ent = sched[blockIdx.x];
    if (ent.x < 0) return;  // padding entry of the XCD-balanced schedule
    const GemmTask T = tasks[ent.x];
    const int row0 = (ent.y & 0xffff) * BT, col0 = (ent.y >> 16) * BT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave / WGN) * WM, wn0 = (wave % WGN) * WN;

    // each thread moves CH 16-byte chunks per operand and stage: EPC consecutive
    // elements of row r, i.e. EPC / 2 pairs of doubles in LDS.  LDS element k of row
    // r sits at k ^ (r & 15), so each pair lands on an aligned pair, swapped for odd r.
    typedef float v4f __attribute__((ext_vector_type(4)));
    typedef typename std::conditional<sizeof(ST) == 8, v2d, v4f>::type chunk_t;
    const ST* aptr[CH];
    const ST* bptr[CH];
    int lpos[CH][EPC / 2];
    bool swap[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) {
        const int c = tid + i * NT;
        const int r = c / (KTD / EPC), s = c % (KTD / EPC);
        const int ga = min(row0 + r, T.M - 1), gb = min(col0 + r, T.N - 1);
        aptr[i] = reinterpret_cast<const ST*>(bases.p[T.x.buf] + T.x.off) + (int64_t)ga * T.x.ld + EPC * s;
        bptr[i] = reinterpret_cast<const ST*>(bases.p[T.z.buf] + T.z.off) + (int64_t)gb * T.z.ld + EPC * s;
#pragma unroll
        for (int q = 0; q < EPC / 2; ++q) lpos[i][q] = r * KTD + (((EPC * s + 2 * q) ^ (r & 15)) & ~1);
        swap[i] = (r & 1) != 0;
    }
    const int nst = T.K / KTD;
    chunk_t ra[CH], rb[CH];
    auto gload = [&](int st) {
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            ra[i] = *reinterpret_cast<const chunk_t*>(aptr[i] + st * KTD);
            rb[i] = *reinterpret_cast<const chunk_t*>(bptr[i] + st * KTD);
        }
    };
    auto sstore = [&](int buf) {
        double* base = lds + buf * STAGE;
#pragma unroll
        for (int i = 0; i < CH; ++i)
#pragma unroll
            for (int q = 0; q < EPC / 2; ++q) {
                v2d a = v2d{(double)ra[i][2 * q], (double)ra[i][2 * q + 1]};
                v2d b = v2d{(double)rb[i][2 * q], (double)rb[i][2 * q + 1]};
                if (swap[i]) {
                    a = v2d{a.y, a.x};
                    b = v2d{b.y, b.x};
                }
                *reinterpret_cast<v2d*>(base + lpos[i][q]) = a;
                *reinterpret_cast<v2d*>(base + TILE + lpos[i][q]) = b;
            }
    };

    v4d acc[FM][FN];
#pragma unroll
    for (int m = 0; m < FM; ++m)
#pragma unroll
        for (int n = 0; n < FN; ++n) acc[m][n] = v4d{0.0, 0.0, 0.0, 0.0};

    if (nst > 0) {
        gload(0);
        sstore(0);
    }
    __syncthreads();
    const int lr = lane & 15, lk = lane >> 4;
    for (int st = 0; st < nst; ++st) {
        const int buf = st & 1;
        if (st + 1 < nst) gload(st + 1);
        const double* base = lds + buf * STAGE;
#pragma unroll
        for (int ks = 0; ks < KTD / 4; ++ks) {
            const int k = ks * 4 + lk;
            double af[FM], bf[FN];
#pragma unroll
            for (int m = 0; m < FM; ++m) {
                const int r = wm0 + m * 16 + lr;
                af[m] = base[r * KTD + (k ^ (r & 15))];
            }
#pragma unroll
            for (int n = 0; n < FN; ++n) {
                const int r = wn0 + n * 16 + lr;
                bf[n] = base[TILE + r * KTD + (k ^ (r & 15))];
            }
#pragma unroll
            for (int m = 0; m < FM; ++m)
#pragma unroll
                for (int n = 0; n < FN; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[m], bf[n], acc[m][n], 0, 0, 0);
        }
        if (st + 1 < nst) sstore(buf ^ 1);
        __syncthreads();
    }

    char* cbase = bases.p[T.c.buf] + T.c.off;
#pragma unroll
    for (int m = 0; m < FM; ++m)
#pragma unroll
        for (int n = 0; n < FN; ++n)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // output layout of the 16x16 f64 MFMA: lane group g = lane/16, register v -> row g + 4 v
                const int i = row0 + wm0 + m * 16 + (lane >> 4) + 4 * v;
                const int j = col0 + wn0 + n * 16 + (lane & 15);
                if (i < T.M && j < T.N && (!T.syrk || i >= j))
                    store_res(cbase, T.c.dt, (int64_t)i * T.c.ld + j,
                              mod_canon(acc[m][n][v], fp.p, fp.inv_p));
            }
}

constexpr int BT_F64 = 128;

template <typename ST>
static int launch_f64_st(const GemmTask* d_tasks, const TileEnt* d_sched, int nblocks, const Bases& b,
                         const FieldParams& fp, void* stream)
{
    constexpr int lds_bytes = 2 * 2 * BT_F64 * KTD * 8;
    auto kern = gemm_f64<BT_F64, 2, 2, ST>;
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
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(256), lds_bytes, (hipStream_t)stream, b,
                       d_tasks, d_sched, fp);
    return (int)hipGetLastError();
}

int launch_gemm_f64(const GemmTask* d_tasks, const TileEnt* d_sched, int nblocks, const Bases& b,
                    const FieldParams& fp, void* stream)
{
    if (nblocks <= 0) return 0;
    return fp.st32 ? launch_f64_st<float>(d_tasks, d_sched, nblocks, b, fp, stream)
                   : launch_f64_st<double>(d_tasks, d_sched, nblocks, b, fp, stream);
}

int gemm_tile_f64() { return BT_F64; }

}  // namespace ffa
