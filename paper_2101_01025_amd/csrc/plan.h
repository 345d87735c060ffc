// Host planner: turns one call (or a batch of calls) into the launch sequence
// of the level-synchronous schedule and the workspace layout.  No device is
// touched here, so plans can be built and inspected on a host without a GPU.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ffa.h"
#include "ffa_internal.h"

namespace ffa {

struct Problem {
    int64_t n = 0, k = 0, lda = 0, ldc = 0;
    uint32_t p = 0;
    int herm = 0;
    int dA = 0, dC = 0;
    ffa_opts opts{};
    bool aligned = true;       // caller's A pointer is 16-byte aligned
    int64_t a_off = 0;         // element offsets in the caller's buffers (batches)
    int64_t c_off = 0;
    int trans = 0;             // A is k x n and the product is A^T A
    uint32_t alpha = 1, beta = 0;  // C <- alpha Low(A A^T) + beta C
    bool packed = false;       // A in the library's packed layout (rows padded to 16 bytes)
};

struct Plan {
    int status = FFA_OK;
    int carrier = CAR_I8, nl = 1, cplx = 0, levels = 0;
    int64_t npad = 0, kpad = 0;        // first problem (single calls)
    bool direct = false;               // products read the caller's A without conditioning
    int max_abs = 0;                   // largest operand magnitude fed to the products
    int64_t max_k = 0;                 // longest accumulation (carrier elements)
    FieldParams fp{};
    int check_inputs = 0;
    int zero_fill = 0;                 // k == 0: the output is Low(0)
    // task tables
    std::vector<CondTask> cond;
    int cond_max_blocks = 0;           // total blocks (transposed: blocks of the largest task)
    bool cond_trans = false;           // conditioning reads the transpose (tiles of 64 x 64)
    // 2M Hermitian base case: real products (their own launch and schedule) and
    // the combination into each leaf's complex result
    bool herk2m = false;
    std::vector<GemmTask> gemm_r;
    std::vector<TileEnt> sched_r;
    int gemm_cfg_r = 0;
    std::vector<Herk2mTask> h2m;
    int h2m_max_n = 0;
    // Strassen-Winograd for the general products
    bool wino = false;
    int64_t wino_min = 0;              // general products with fewer rows stay one task
    std::vector<WinoPreTask> wpre;
    std::vector<WinoPostTask> wpost;
    int wpre_max_h = 0, wpre_max_w = 0, wpost_max_h = 0;
    std::vector<UpdateTask> upd;       // final C <- alpha X + beta C (no recursion)
    bool fold_update = false;          // the level-0 post-additions apply the update (recursion)
    int upd_max_n = 0;
    std::vector<std::vector<PreaddTask>> pre;   // per level, top-down
    std::vector<std::vector<PostaddTask>> post; // per level
    std::vector<int> pre_max_hw, post_max_h;    // grid sizing per level
    std::vector<int> pre_max_h, pre_max_w;
    // Products, in two groups: [0, gemm_split) read only A (the leaves reached
    // through P1 and P2 alone), [gemm_split, end) read pre-addition outputs.
    // Each group has its own tile schedule so that the first can run while the
    // pre-additions are still being computed.
    std::vector<GemmTask> gemm;
    std::vector<char> gemm_aonly;      // per task while planning: reads only A
    int gemm_split = 0;
    int total_tiles = 0;
    int gemm_cfg = 0;                  // INT8 product kernel configuration
    int gemm_src = SRC_CARRIER;        // operand source of the product launch
    int kernel_req = 0;                // requested configuration + 1 (0: built-in choice)
    int tile = 0;                      // product tile edge
    int ktile = 0;                     // product k-tile (carrier elements); K is padded to it
    std::vector<TileEnt> sched;         // XCD-balanced tile schedule of group 1, one entry per workgroup
    std::vector<TileEnt> sched2;        // same for group 2
    bool split_tail = false;            // may split the launch's last partial round over K
    std::vector<TailTask> tail;         // tiles so split: sums of their pieces
    bool fork = false;                  // run pre-additions + group 2 on a second stream
    // Pre-additions beside the product launch: one limb, one level.  The
    // pre-addition kernel runs on a second stream (PRE_SIGNAL_BLOCKS workgroups,
    // each raising the counter at workspace byte wait_off when done) while the
    // single product launch runs the tiles that read only A first; its tiles
    // that read S1..S4 wait for the counter.
    bool overlap_pre = false;
    int pre_blocks = 0;                 // workgroups of the pre-addition kernel (the counter's target)
    int64_t wait_off = 0;
    // Persistent INT8 product launch: at most the resident workgroups, taking tiles
    // from 8 queue counters (one per XCD) at workspace byte queue_off
    bool persist = false;
    int64_t queue_off = 0;
    int64_t ws_bytes = 0;
    int64_t products_macs = 0;         // multiply-accumulates of the products (per limb product)
    std::vector<int64_t> a_off, c_off; // packed batch layout (elements)
    std::vector<int64_t> a_ld;         // packed batch: row stride of each A_i (elements)
    int64_t a_total = 0, c_total = 0;
    // host and device copies of the tables (filled by the API layer)
    std::vector<char> h_blob;
    void* d_blob = nullptr;
    int64_t blob_bytes = 0;
    int64_t off_cond = 0, off_gemm = 0, off_sched = 0, off_sched2 = 0, off_upd = 0;
    int64_t off_gemm_r = 0, off_sched_r = 0, off_h2m = 0, off_wpre = 0, off_wpost = 0, off_tail = 0;
    std::vector<int64_t> off_pre, off_post;
};

constexpr int PRE_SIGNAL_BLOCKS = 256;

// Validates and plans one call.  status != FFA_OK means the call must fail
// with that status before launching anything.
Plan make_plan(const Problem& pr);
// Plans a batch of independent problems sharing p and the formats.
Plan make_batch_plan(const std::vector<Problem>& prs);
std::string describe(const Plan& pl);
// Serialises the task tables into one blob with the offsets recorded in pl.
std::vector<char> pack_tables(Plan& pl);

}  // namespace ffa
