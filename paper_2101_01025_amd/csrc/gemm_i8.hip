// Configurations of the grouped INT8 product kernel (gemm_i8_kernel.h) and the
// dispatch to the translation units that instantiate it (gemm_i8_part_*.hip).
#include <hip/hip_runtime.h>

#include "ffa_internal.h"
#include "gemm_i8_configs.h"

namespace ffa {

// Entry points of the units that instantiate the kernel.
#define FFA_I8_DECLARE_PART(PART)                                                                  \
    int gemm_i8_launch_##PART(int cfg, int src, const GemmTask* d_tasks, const TileEnt* d_sched,  \
                              int nblocks, const Bases& b, const FieldParams& fp, hipStream_t s);  \
    int gemm_i8_regs_##PART(int cfg, int* vgprs);
FFA_I8_DECLARE_PART(a)
FFA_I8_DECLARE_PART(b)
FFA_I8_DECLARE_PART(c)
FFA_I8_DECLARE_PART(d)
FFA_I8_DECLARE_PART(e)
#undef FFA_I8_DECLARE_PART

struct CfgInfo {
    int nl, cplx, bt, kt, nthreads, lds, raw;
};

static CfgInfo cfg_info(int id)
{
#define FFA_INFO(ID, NL, CP, BT, WM, WN, KT, PF, MS, OPT) \
    if (id == ID)                                                                              \
        return CfgInfo{NL, CP, BT, KT, WM * WN * 64,                                        \
                       (PF < 0 ? -PF : 2) * ((CP ? 2 : 1) * NL + NL) * BT * KT,           \
                       NL == 2 && !CP && PF > 0};
    FFA_I8_CONFIGS(FFA_INFO)
#undef FFA_INFO
    return CfgInfo{0, 0, 0, 0, 0, 0, 0};
}

int gemm_i8_config_tile(int cfg) { return cfg_info(cfg).bt; }
int gemm_i8_config_ktile(int cfg) { return cfg_info(cfg).kt; }
int gemm_i8_config_raw(int cfg) { return cfg_info(cfg).raw; }
int gemm_i8_config_lds(int cfg) { return cfg_info(cfg).lds; }

int gemm_i8_config_valid(int cfg, int nl, int cplx)
{
    const CfgInfo ci = cfg_info(cfg);
    return ci.bt > 0 && ci.nl == nl && ci.cplx == cplx;
}

int gemm_i8_default_config(int nl, int cplx, int64_t max_dim)
{
    if (cplx) return nl == 1 ? 4 : 8;
    // 8 waves, direct loads into two buffers issued between the k-steps: 7.69 ms (no
    // recursion) and 6.81 ms (one level) per call at n = k = 16384, p = 65521, against
    // 7.82 and 7.20 ms for configuration 16 (two k-tiles in flight in registers);
    // smaller problems keep configuration 16 (the raw uint16 operand path needs
    // register loads)
    if (nl == 2) return max_dim >= 2048 ? 32 : 16;
    // 8 waves of 128x64, operands loaded straight into LDS, 16x16x64 MFMAs: 1.78 ms
    // against 1.86 ms for configuration 24 (the same with 32x32x32 MFMAs) and 1.84 ms
    // for configuration 29 (loads spread over the k-steps) per call at n = k = 16384,
    // p = 251, no recursion (medians of alternating blocks); configuration 40 (each
    // k-tile's last k-step after its barrier) 1.71 vs 1.74 ms without recursion but
    // 1.84 vs 1.81 ms with one level
    return max_dim >= 2048 ? 34 : 2;
}

int gemm_i8_config_regs(int cfg, int* vgprs, int* threads, int* lds)
{
    const CfgInfo ci = cfg_info(cfg);
    if (ci.bt == 0) return (int)hipErrorInvalidValue;
    int r = gemm_i8_regs_a(cfg, vgprs);
    if (r == FFA_I8_NOT_HERE) r = gemm_i8_regs_b(cfg, vgprs);
    if (r == FFA_I8_NOT_HERE) r = gemm_i8_regs_c(cfg, vgprs);
    if (r == FFA_I8_NOT_HERE) r = gemm_i8_regs_d(cfg, vgprs);
    if (r == FFA_I8_NOT_HERE) r = gemm_i8_regs_e(cfg, vgprs);
    if (r == FFA_I8_NOT_HERE) return (int)hipErrorInvalidValue;
    if (r == 0) {
        *threads = ci.nthreads;
        *lds = ci.lds;
    }
    return r;
}

int launch_gemm_i8(int cfg, int src, const GemmTask* d_tasks, const TileEnt* d_sched, int nblocks,
                   const Bases& b, const FieldParams& fp, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (nblocks <= 0) return 0;
    int r = gemm_i8_launch_a(cfg, src, d_tasks, d_sched, nblocks, b, fp, s);
    if (r == FFA_I8_NOT_HERE) r = gemm_i8_launch_b(cfg, src, d_tasks, d_sched, nblocks, b, fp, s);
    if (r == FFA_I8_NOT_HERE) r = gemm_i8_launch_c(cfg, src, d_tasks, d_sched, nblocks, b, fp, s);
    if (r == FFA_I8_NOT_HERE) r = gemm_i8_launch_d(cfg, src, d_tasks, d_sched, nblocks, b, fp, s);
    if (r == FFA_I8_NOT_HERE) r = gemm_i8_launch_e(cfg, src, d_tasks, d_sched, nblocks, b, fp, s);
    return r == FFA_I8_NOT_HERE ? (int)hipErrorInvalidValue : r;
}

}  // namespace ffa
