// Internal definitions shared by the planner (host) and the HIP kernels.
//
// The recursion of Algorithm 1 (Section 3) is executed level by level:
//   conditioning -> pre-additions level 0..l-1 (top-down) -> one grouped launch of
//   every product (all leaf SYRKs and all P3/P4 general products of every level)
//   -> post-additions level l-1..0 (bottom-up).
// Each launch reads a device-resident task table.  Tasks address memory as
// (buffer id, byte offset) so that one table serves every call with the same
// shape: the kernels receive the buffer base pointers as arguments.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define FFA_HD __host__ __device__
#else
#define FFA_HD
#endif

namespace ffa {

// ---- buffer ids -----------------------------------------------------------
enum BufId : int32_t {
    BUF_A = 0,   // caller's A (real part for the Hermitian product)
    BUF_A2 = 1,  // caller's imaginary part of A
    BUF_C = 2,   // caller's C (real part)
    BUF_C2 = 3,  // caller's imaginary part of C
    BUF_WS = 4,  // library workspace
    BUF_ERR = 5, // the context's device status words (int32 [0]: input range, [1]: wait timeout)
    NBUF = 6
};

struct Bases {
    char* p[NBUF];
};

// ---- element formats ------------------------------------------------------
// Residue storage formats (canonical values in [0, p)) and the caller formats.
enum Dtype : int32_t {
    DT_I64 = 0,
    DT_I32 = 1,
    DT_U16 = 2,
    DT_U8 = 3,
    DT_F64 = 4,
    DT_I8C = 5,  // centred int8 (input only)
};

FFA_HD inline int dtype_size(int dt)
{
    switch (dt) {
    case DT_I64: return 8;
    case DT_I32: return 4;
    case DT_U16: return 2;
    case DT_U8: return 1;
    case DT_F64: return 8;
    case DT_I8C: return 1;
    }
    return 0;
}

// Carrier of the products: the representation the MFMA units consume.
enum Carrier : int32_t {
    CAR_I8 = 0,   // NL balanced int8 limbs per plane (NL = 1 or 2)
    CAR_F64 = 1,  // fp64 holding exact integers
};

// Kind of skew-unitary Y (Section 4).
enum YKind : int32_t {
    Y_SCALAR = 0,  // Y = a I, a^2 = -1 (Proposition lemsqrt)
    Y_BLOCKS = 1,  // Y = [[a, b], [-b, a]] (x) I on column halves (Proposition pigeonhole)
    Y_GAUSS = 2,   // Y = (a + i b) I over F_p[i] (Section 4.4)
};

// ---- matrix references ----------------------------------------------------
// Carrier matrix: sub-plane q (q = plane * NL + limb) starts at off + q * ps
// bytes of buffer buf; rows are ld elements apart.
struct CarRef {
    int64_t off;
    int64_t ps;
    int32_t buf;
    int32_t ld;
};

// Residue matrix: real plane at (buf, off), imaginary plane at (buf2, off2);
// rows ld elements apart; element format dt.
struct ResRef {
    int64_t off;
    int64_t off2;
    int32_t buf;
    int32_t buf2;
    int32_t ld;
    int32_t dt;
};

// ---- field parameters -----------------------------------------------------
struct FieldParams {
    int32_t p;
    int32_t half;      // (p - 1) / 2 for the single-limb centred form
    int32_t rep_max;   // largest representative of the two-limb form (32639)
    int32_t ykind;
    int32_t ya, yb;    // Y coefficients (canonical)
    int32_t nl;        // limbs per plane (carrier CAR_I8)
    int32_t cplx;      // 1 for F_p[i]
    double inv_p;      // 1.0 / p
    int32_t alpha, beta;  // C <- alpha X + beta C (canonical) in the update pass
    int32_t npo;          // complex carriers: 4 = planes re, im, -re and re + im (2M base case)
    int32_t st32;         // fp64 carrier held in fp32 storage (exact integers below 2^24)
    int32_t r20;          // round(2^20 / p): centred reduction of short sums for p < 2^8
    int32_t nent;         // product launch: 0, or the schedule's entries when it runs persistent
    int64_t queue_off;    // persistent product launch: workspace offset of its 8 queue counters
};

// ---- tasks ----------------------------------------------------------------
// One node of the recursion: A is 2h x 2w (after padding); its blocks feed
// S1..S4 (each h x w).
struct PreaddTask {
    CarRef a;
    CarRef s[4];
    int32_t h, w;
};

// Post-additions of one node: products P1..P5 (h x h residues) into the
// node's C (2h x 2h), rows/columns >= nvalid are not written.  At the top of an
// update call (C <- alpha Low(A A^T) + beta Low(C), Section 7) the update is
// applied as the results are stored (upd = 1).
struct PostaddTask {
    ResRef p[5];
    ResRef c;
    int32_t h;
    int32_t nvalid;
    int32_t upd;   // 1: c is the caller's C of an update call, which receives alpha U + beta C
    int32_t pad_;
};

// One product C = X * phi(Z) restricted to tiles; syrk: X == Z, only the
// lower triangle (row >= col) is produced.  With raw operands (the caller's
// canonical uint16 residues, split into limbs by the product kernel) x and z
// point at the caller's matrix, ld is its row stride in bytes and the columns
// kvalid .. K-1 are treated as zero.
struct GemmTask {
    CarRef x, z;
    ResRef c;
    int32_t M, N, K;       // K in carrier elements, a multiple of the k-tile
    int32_t syrk;
    int32_t tiles_m, tiles_n;
    int32_t kvalid;        // columns of the operands that hold data (K for carriers)
    // > 0: the task's operands are written by a kernel running beside the launch;
    // before its first load a tile waits until the workspace counter at byte
    // wait_off has reached this value (bounded; a timeout is recorded in the context's
    // status word BUF_ERR[1])
    int32_t wait;
    int64_t wait_off;
};

// Operand source of a product launch (every task of a launch shares it).
enum GemmSrc : int32_t {
    SRC_CARRIER = 0,  // carrier planes prepared by conditioning / pre-additions
    SRC_RAW_U16 = 1,  // the caller's canonical uint16 residues (two limbs, real field)
};

// One entry of a product launch's schedule: x = task index (-1: idle entry),
// y = tile row | tile column << 16.
struct TileEnt {
    int32_t x, y;
};

// One product tile computed as nparts K-pieces (the last partial round of a
// launch, spread over more workgroups): out (rows x cols residues) = the sum of
// the pieces mod p.  Piece q is a tile of residues at part + q * pstride bytes
// (row stride part.ld elements) in the format of out.
struct TailTask {
    ResRef part, out;
    int64_t pstride;
    int32_t rows, cols, nparts, pad_;
};

// Conditioning: caller's A (n x k, format dt_in) into a carrier matrix of
// npad x kpad (zero padded), planes re (and im, -re for F_p[i]).
// trans: the caller's A is k x n and the carrier receives its transpose.
struct CondTask {
    int32_t n, k, npad, kpad;
    int32_t lda, dt_in;
    int32_t buf_re, buf_im;
    int64_t off_re, off_im;
    CarRef out;
    int32_t trans;
    int32_t blk0;  // first block of this task in the one-dimensional grid of the launch
    int32_t skip;  // bit q set: carrier plane q is not written (no product reads it)
    int32_t pad_;
};

// 2M base case of a Hermitian leaf (Algorithm 3 with epsilon = 1): from the real
// residues G = (Xr + Xi)(Xr + Xi)^T (lower triangle) and H = Xr Xi^T (whole),
// Low(X X^H) = Low(G - H - H^T) + i Low(H^T - H) into out (rows and columns
// >= nvalid are not written).
// H may come in two halves over K (h2 valid when split): H = h + h2 mod p.
struct Herk2mTask {
    ResRef g, h, h2, out;
    int32_t n, nvalid;
    int32_t split, pad_;
};

// One level of Strassen-Winograd for a general product C = X Z^T (X, Z: 2h x 2w
// carriers, C: 2h x 2h residues).  With B = Z^T, the operand sums are
//   S1 = X21 + X22, S2 = S1 - X11, S3 = X11 - X21, S4 = X12 - S2 (on X) and
//   T1 = Z21 - Z11, T2 = Z22 - T1, T3 = Z22 - Z21, T4 = T2 - Z12 (on Z, i.e. the
//   sums of the blocks of B transposed), each h x w;
// the seven products R1 = X11 Z11^T, R2 = X12 Z12^T, R3 = S4 Z22^T, R4 = X22 T4^T,
// R5 = S1 T1^T, R6 = S2 T2^T, R7 = S3 T3^T; and
//   C11 = R1 + R2, C12 = R1 + R6 + R5 + R3, C21 = R1 + R6 + R7 - R4, C22 = R1 + R6 + R7 + R5.
struct WinoPreTask {
    CarRef x, z;
    CarRef s[4], t[4];
    int32_t h, w;
};
struct WinoPostTask {
    ResRef r[7];
    ResRef c;
    int32_t h, pad_;
};

// Final update C <- alpha X + beta C on the lower triangle of an n x n result:
// X is the product's residues (workspace), C the caller's matrix.
struct UpdateTask {
    ResRef x, c;
    int32_t n, pad_;
};

// ---- fixed scratch of the entry point that allocates nothing (noalloc.hip) ----
// Looks up the scratch array's device address on `device`, which must be the
// current device; once per device, later calls return at once.  hipError_t as int.
int scratch_setup(int device);
// That address (null before scratch_setup succeeded on the device).
char* scratch_base(int device);

// ---- launch wrappers (defined in the .hip files) ---------------------------
// All return a hipError_t value cast to int.
int launch_zero_flag(int32_t* d_flag, void* stream);
// dt_in: the caller's input format (every task of a launch shares it)
// nblocks: total blocks of all tasks (task t owns blocks blk0 .. of the 1-D grid)
int launch_condition(const CondTask* d_tasks, int ntasks, int nblocks, int dt_in, const Bases& b,
                     const FieldParams& fp, int carrier, int32_t* d_err, void* stream);
// one launch for every task with trans = 1 (the others go to launch_condition)
int launch_condition_trans(const CondTask* d_tasks, int ntasks, int max_tiles, int dt_in, const Bases& b,
                           const FieldParams& fp, int carrier, int32_t* d_err, void* stream);
int launch_wino_pre(const WinoPreTask* d_tasks, int ntasks, int max_h, int max_w, const Bases& b,
                    const FieldParams& fp, int carrier, void* stream);
int launch_wino_post(const WinoPostTask* d_tasks, int ntasks, int max_h, const Bases& b,
                     const FieldParams& fp, void* stream);
int launch_herk2m(const Herk2mTask* d_tasks, int ntasks, int max_n, int res_dt, int out_dt,
                  const Bases& b, const FieldParams& fp, void* stream);
int launch_tail_sum(const TailTask* d_tasks, int ntasks, int max_rows, int dt, const Bases& b,
                    const FieldParams& fp, void* stream);
int launch_update(const UpdateTask* d_tasks, int ntasks, int max_n, int x_dt, int c_dt, const Bases& b,
                  const FieldParams& fp, void* stream);
int launch_preadd(const PreaddTask* d_tasks, int ntasks, int h, int w, const Bases& b,
                  const FieldParams& fp, int carrier, void* stream);
// The same pre-additions (one limb, real field) on a grid of `blocks` x ntasks
// workgroups that loop over the work, each raising the workspace counter at byte
// `counter_off` by one when its part is written (release at device scope): run on
// a second stream beside the product launch whose tiles wait for the counter.
int launch_preadd_signal(const PreaddTask* d_tasks, int ntasks, int h, int w, const Bases& b,
                         const FieldParams& fp, int blocks, int64_t counter_off, void* stream);
// Zeroes `words` int32 words at byte `off` of the workspace (a kernel, so that
// graph capture records no memset node).
int launch_zero_words(const Bases& b, int64_t off, int words, void* stream);
// Resources of the signalling pre-addition kernel (for the co-residency check).
int preadd_signal_regs(int* vgprs, int* threads);
// out_dt: format of the outputs of this level (every task of a launch shares it)
int launch_postadd(const PostaddTask* d_tasks, int ntasks, int h, int out_dt, const Bases& b,
                   const FieldParams& fp, void* stream);
// Product launches read the task table and a schedule: entry blockIdx = (task,
// tile row | tile column << 16), or task = -1 for an idle padding entry.
int launch_gemm_i8(int cfg, int src, const GemmTask* d_tasks, const TileEnt* d_sched, int nblocks,
                   const Bases& b, const FieldParams& fp, void* stream);
int launch_gemm_f64(const GemmTask* d_tasks, const TileEnt* d_sched, int nblocks, const Bases& b,
                    const FieldParams& fp, void* stream);
// INT8 product kernel configurations (tile shapes, pipeline depth)
int gemm_i8_config_tile(int cfg);
int gemm_i8_config_ktile(int cfg);
int gemm_i8_config_raw(int cfg);  // the configuration can read raw uint16 operands
int gemm_i8_config_lds(int cfg);  // dynamic LDS bytes of one workgroup
int gemm_i8_config_valid(int cfg, int nl, int cplx);
int gemm_i8_default_config(int nl, int cplx, int64_t max_dim);
// VGPRs per thread, threads per workgroup and LDS bytes of a configuration's kernel
// (carrier operands); hipError_t as int
int gemm_i8_config_regs(int cfg, int* vgprs, int* threads, int* lds);
int gemm_tile_f64();
// k-tile of the FP64 product kernel, in carrier elements
constexpr int KTILE_F64 = 16;

}  // namespace ffa
