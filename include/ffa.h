/*
 * ffa.h — exact C = Low(A * phi(A)) over a prime field on AMD MI355X (gfx950).
 *
 * The operation is the one of the paper "Some fast algorithms multiplying a
 * matrix by its adjoint" (Dumas, Pernet, Sedoglavic), Section 3, Algorithm 1:
 * given A and an involutive antihomomorphism phi, return the lower triangular
 * part Low(A phi(A)) (Low/Up definition of Section 2: the diagonal belongs to
 * the lower part).  Two antihomomorphisms are provided (Section 2, examples):
 *   - phi = transpose over F_p                       -> ffa_syrk_modp
 *   - phi = conjugate transpose over F_p[i]/(i^2+1)  -> ffa_herk_modp2
 * The recursive algorithm uses 3 recursive and 2 general products per level
 * and a skew-unitary Y (Y phi(Y) = -I) built from a^2 + b^2 = -1 mod p
 * (Section 4, Algorithm 2).  The result is exact: every call returns the
 * same bits as the definition, whatever recursion depth, Y or carrier is used.
 *
 * Conventions common to every entry point
 *   - Matrices are row-major.  A is n x k with leading dimension lda >= k
 *     (elements); C is n x n with ldc >= n.
 *   - A and C are DEVICE pointers owned by the caller.  The library never
 *     frees or keeps them; work is enqueued asynchronously on the context's
 *     stream and the caller keeps the buffers alive until it synchronises.
 *   - Only the lower triangle of C (diagonal included) is written; the strict
 *     upper triangle is never read or written (BLAS uplo = 'L').
 *   - Inputs are canonical residues in [0, p) (FFA_I8_CENTRED: centred
 *     residues in [-(p-1)/2, (p-1)/2], p < 256).  Outputs are canonical.
 *   - n = 0 is valid (nothing written); k = 0 writes zeros.
 *   - Every argument is validated before anything is launched; on an error
 *     nothing is written.  No exception or abort crosses this interface: a
 *     failing host allocation inside the library returns FFA_ENOMEM, any
 *     other C++ exception FFA_EINVAL.
 *   - n is at most FFA_N_MAX (C would not fit one GPU beyond it) and k below
 *     2^31; larger sizes give FFA_EINVAL.
 *   - A context is not thread safe; use one context per host thread.
 */
#ifndef FFA_H
#define FFA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FFA_N_MAX 524288  /* largest n of a call, 2^19 */

typedef struct ffa_ctx ffa_ctx;
typedef struct ffa_batch ffa_batch;

/* status codes (0 = success) */
enum {
    FFA_OK = 0,
    FFA_EINVAL = -1,       /* bad size, stride, pointer, dtype or option */
    FFA_EPRIME = -2,       /* p is not an odd prime, or too large for the carrier */
    FFA_ERANGE = -3,       /* an input entry is outside its residue range (check_inputs) */
    FFA_ENOMEM = -4,       /* device workspace or host memory could not be allocated */
    FFA_EDEVICE = -5,      /* a HIP call failed; ffa_last_device_error() has the code */
    FFA_EUNSUPPORTED = -6, /* valid request this library does not support (e.g. herk with p = 1 mod 4) */
    FFA_EBOUND = -7,       /* the exact-accumulation bound of the carrier is exceeded */
    FFA_ESCRATCH = -8,     /* ffa_syrk_modp_noalloc: the call needs more than FFA_SCRATCH_BYTES */
    FFA_EWAIT = -9         /* a bounded wait inside a kernel gave up (ffa_device_status) */
};

/* element formats of A and C */
enum {
    FFA_I64 = 0,
    FFA_I32 = 1,
    FFA_U16 = 2,
    FFA_U8 = 3,
    FFA_F64 = 4,          /* doubles holding integers */
    FFA_I8_CENTRED = 5    /* input only; p < 256 */
};

enum { FFA_ALGO_AUTO = 0, FFA_ALGO_CLASSICAL = 1, FFA_ALGO_RECURSIVE = 2 };
enum { FFA_CARRIER_AUTO = 0, FFA_CARRIER_INT8 = 1, FFA_CARRIER_F64 = 2 };

/* Options; pass NULL for the defaults (all fields zero except levels = -1, cutoff = 0),
 * or the autotuned choice for the shape when ffa_autotune_syrk has recorded one.
 *   algo          FFA_ALGO_*; CLASSICAL = no recursion (the plain modular SYRK)
 *   levels        recursion depth of Algorithm 1 when >= 0; -1 = from cutoff
 *   cutoff        recurse while the sub-problem has more than cutoff rows (0 = built-in default)
 *   carrier       FFA_CARRIER_*: INT8 = balanced int8 limbs on INT8 MFMA (1 limb for p < 256,
 *                 2 limbs for p < 2^16); F64 = doubles on FP64 MFMA (p < 2^26, real only)
 *   check_inputs  nonzero: verify every entry of A (synchronises the stream; FFA_ERANGE)
 *   kernel        INT8 product-kernel configuration + 1 (tile shape, k-tile, pipeline depth);
 *                 0 = built-in choice; a configuration that does not fit the carrier is ignored.
 *                 Over F_p[i] with the 2M base case, a real configuration applies to the
 *                 real products of the base case, a complex one to the complex products.
 *   launch        batched execution only: FFA_LAUNCH_GRAPH (default) replays the plan's
 *                 launch sequence as one captured hipGraph; FFA_LAUNCH_DIRECT enqueues
 *                 the kernels one by one
 *   operands      FFA_OPERANDS_AUTO: limb planes prepared by a conditioning pass, except
 *                 where those planes would not be addressable with 32-bit offsets, and
 *                 for batches of two-limb uint16 problems under 2048 rows without
 *                 recursion and without a requested configuration, which read their
 *                 rows raw (below) with configuration 39;
 *                 FFA_OPERANDS_PLANES: always; FFA_OPERANDS_RAW: without recursion and
 *                 with uint16 input in 16-byte aligned rows, the product kernel reads A
 *                 itself and forms the limbs on the fly (else ignored); it reads whole
 *                 16-byte chunks, so a single call takes this path only when k is a
 *                 multiple of 8 (batches: any k, their packed rows are padded)
 *   streams       FFA_STREAMS_AUTO: with one level of recursion and one limb of a real
 *                 field, the pre-additions run on the context's second stream beside the
 *                 single product launch on the caller's stream, whose tiles that read only
 *                 A come first and whose tiles that read S1..S4 wait for them (joined
 *                 before the post-additions); otherwise as FFA_STREAMS_ONE.
 *                 FFA_STREAMS_ONE: everything in stream order on the caller's stream;
 *                 FFA_STREAMS_TWO: with recursion, the pre-additions and the products that
 *                 need them run on a second stream as a second product launch while the
 *                 products that read only A run on the caller's stream
 *   herk_base     base case of ffa_herk_modp2: FFA_HERK_AUTO / FFA_HERK_2M = the 2M method
 *                 (Section 6, Algorithm 3 with epsilon = 1): one real SYRK of Xr + Xi and one
 *                 real GEMM Xr Xi^T, 1.5 n^2 k products over F_p; FFA_HERK_4M = the four real
 *                 products of the complex kernel, 2 n^2 k
 *   general       the general products P3, P4 of each recursion node: FFA_GENERAL_CLASSICAL,
 *                 or FFA_GENERAL_WINOGRAD = one level of Strassen-Winograd (7 half-size
 *                 products, 15 block additions; real carriers only, else ignored);
 *                 FFA_GENERAL_AUTO = Winograd on the fp64 carrier, classical on INT8
 *   wino_min      Winograd applies to general products of at least this many rows; the
 *                 smaller ones stay single products (their block additions cost more HBM
 *                 time than the multiplications they save).  0 = built-in: every general
 *                 product under FFA_GENERAL_WINOGRAD, 2048 rows under FFA_GENERAL_AUTO.
 *                 Negative: FFA_EINVAL.
 *   persist       the INT8 product launch of a batch (or of a single call without a
 *                 launch beside it): FFA_PERSIST_ON runs it persistent (at most the
 *                 workgroups that fit the device at once, each taking tiles from an
 *                 in-kernel work queue per XCD until it is drained); FFA_PERSIST_OFF one
 *                 workgroup per tile; FFA_PERSIST_AUTO: persistent for batches.
 *                 Other values: FFA_EINVAL. */
enum { FFA_LAUNCH_GRAPH = 0, FFA_LAUNCH_DIRECT = 1 };
enum { FFA_HERK_AUTO = 0, FFA_HERK_2M = 1, FFA_HERK_4M = 2 };
enum { FFA_GENERAL_AUTO = 0, FFA_GENERAL_CLASSICAL = 1, FFA_GENERAL_WINOGRAD = 2 };
enum { FFA_OPERANDS_AUTO = 0, FFA_OPERANDS_PLANES = 1, FFA_OPERANDS_RAW = 2 };
enum { FFA_STREAMS_AUTO = 0, FFA_STREAMS_ONE = 1, FFA_STREAMS_TWO = 2 };
enum { FFA_PERSIST_AUTO = 0, FFA_PERSIST_OFF = 1, FFA_PERSIST_ON = 2 };
typedef struct {
    int32_t algo;
    int32_t levels;
    int32_t cutoff;
    int32_t carrier;
    int32_t check_inputs;
    int32_t kernel;
    int32_t launch;
    int32_t operands;
    int32_t streams;
    int32_t herk_base;
    int32_t general;
    int32_t wino_min;
    int32_t persist;
} ffa_opts;

/* Context bound to a HIP device and stream (stream NULL = the null stream).
 * Owns the device workspace (grown on demand, freed by ffa_destroy) and a
 * cache of plans.  Returns FFA_EINVAL / FFA_EDEVICE on failure. */
int ffa_create(ffa_ctx** out, int device, void* hip_stream);
int ffa_destroy(ffa_ctx* ctx);
int ffa_set_stream(ffa_ctx* ctx, void* hip_stream);
/* hipError_t of the last failing HIP call of this context (0 if none). */
int ffa_last_device_error(const ffa_ctx* ctx);
/* Synchronises the context's stream and reports FFA_EWAIT if a bounded wait inside
 * a kernel of an earlier call on the context gave up, which makes that call's result
 * invalid (the record is then cleared); FFA_OK otherwise.  Such waits exist where a
 * call runs its pre-additions beside the product launch (opts.streams AUTO, one limb,
 * one level): the product tiles that read S1..S4 wait, for about a second at most,
 * for the pre-addition kernel on the context's second stream. */
int ffa_device_status(ffa_ctx* ctx);
const char* ffa_status_string(int status);

/* The skew-unitary Y used for p (Section 4):
 *   kind 0: Y = a I with a^2 = -1 (p = 1 mod 4, Proposition lemsqrt)
 *   kind 1: Y = [[a, b], [-b, a]] (x) I, column halves (p = 3 mod 4, Proposition pigeonhole)
 *   kind 2: Y = (a + i b) I over F_p[i] (hermitian != 0, p = 3 mod 4, Section 4.4)
 * (a, b) come from Algorithm 2 with k = -1, smaller square roots.  Host only. */
int ffa_skew_unitary(uint32_t p, int hermitian, uint32_t* a, uint32_t* b, int* kind);

/* C = Low(A A^T) mod p  (Algorithm 1 with phi = transpose, Section 3).
 * dA: FFA_I8_CENTRED, FFA_U8, FFA_U16, FFA_I32, FFA_I64 or FFA_F64;
 * dC: FFA_U8 (p < 256), FFA_U16 (p < 2^16), FFA_I32, FFA_I64 or FFA_F64. */
int ffa_syrk_modp(ffa_ctx* ctx, int64_t n, int64_t k, uint32_t p,
                  int dA, const void* A, int64_t lda,
                  int dC, void* C, int64_t ldc, const ffa_opts* opts);

/* For callers that cannot allocate device memory (code under graph capture,
 * serving loops, harnesses that forbid hipMalloc): ffa_syrk_modp with the same
 * arguments, results and errors, which calls no hipMalloc, hipFree or other
 * allocating routine.  Its workspace and task tables live in a fixed device array
 * of FFA_SCRATCH_BYTES per GPU, which the library holds from the moment it is
 * loaded until the process ends (its address is looked up when a context is
 * created on the GPU).  Host memory is still used for the plan (kept in the
 * context's cache, as for ffa_syrk_modp).
 *   - FFA_ESCRATCH: the call's workspace and tables would exceed FFA_SCRATCH_BYTES
 *     (e.g. a recursive 16384 x 16384 call needs 576 MiB); nothing is launched.
 *   - Every call on one GPU, from any context or stream, shares that GPU's array,
 *     which keeps the last call's contents (no kernel of the call expects it to
 *     hold zeros).  Calls that may overlap on one GPU (different streams, or
 *     different host threads) race on it; calls in one stream do not. */
#define FFA_SCRATCH_BYTES (64ll << 20)
int ffa_syrk_modp_noalloc(ffa_ctx* ctx, int64_t n, int64_t k, uint32_t p,
                          int dA, const void* A, int64_t lda,
                          int dC, void* C, int64_t ldc, const ffa_opts* opts);

/* The SYRK update form (Section 7, schedule for alpha A A^T + beta C):
 *   C <- alpha Low(op(A) op(A)^T) + beta Low(C)  mod p,
 * op(A) = A (trans = 0, A is n x k, lda >= k) or A^T (trans = 1, A is k x n, lda >= n,
 * so that C = A^T A).  alpha, beta in [0, p).  With beta != 0 the lower triangle of
 * C must hold canonical residues; with beta = 0 it is not read.  The strict upper
 * triangle is neither read nor written.  trans = 0, alpha = 1, beta = 0 is
 * ffa_syrk_modp; otherwise the product goes to workspace residues and a final
 * pass forms alpha X + beta C (alpha X + beta C < 2^53 in fp64, exact for p < 2^26). */
int ffa_syrk_modp_ex(ffa_ctx* ctx, int trans, int64_t n, int64_t k, uint32_t p, uint32_t alpha,
                     int dA, const void* A, int64_t lda, uint32_t beta, int dC, void* C, int64_t ldc,
                     const ffa_opts* opts);

/* C = Low(A A^H) over F_{p^2} = F_p[i]/(i^2+1), p = 3 mod 4, conj(x + iy) = x - iy
 * (Algorithm 1 with phi = conjugate transpose; Y of Section 4.4).  Planar storage:
 * A = A_re + i A_im and C = C_re + i C_im, each plane as in ffa_syrk_modp, same lda/ldc.
 * Im(C_ii) = 0.  p = 1 mod 4 gives FFA_EUNSUPPORTED (i^2 + 1 is reducible). */
int ffa_herk_modp2(ffa_ctx* ctx, int64_t n, int64_t k, uint32_t p, int dA,
                   const void* A_re, const void* A_im, int64_t lda,
                   int dC, void* C_re, void* C_im, int64_t ldc, const ffa_opts* opts);

/* Batched C_i = Low(A_i A_i^T) mod p for independent problems (one p).
 * Problems use a PACKED layout fixed by the plan (ffa_batch_offsets): A_i starts
 * at element a_off[i] of one buffer with row stride lda[i] = k_i rounded up to 16
 * bytes (the padding columns are never read), C_i at element c_off[i] of another
 * with ldc = n_i; both buffers must be 16-byte aligned.
 * The plan (host work: tables, its own device workspace) is made once and owns
 * that workspace, so later single calls on the context never move it.
 * ffa_batch_syrk_exec allocates nothing.  With opts.launch = FFA_LAUNCH_GRAPH it
 * captures the plan's launch sequence into a hipGraph on a private stream the
 * first time it sees a pair of buffers (and again when the pair changes) and
 * then enqueues one hipGraphLaunch on the context's stream; it falls back to
 * direct launches while phase profiling is on, with check_inputs, and when the
 * context's stream is itself being captured (the kernels then join the caller's
 * graph).  One plan must not be executed from two threads at once. */
#define FFA_BATCH_MAX 4194304  /* most problems in one batch plan (count above it: FFA_EINVAL) */
int ffa_batch_syrk_plan(ffa_ctx* ctx, int64_t count, const int64_t* n, const int64_t* k,
                        uint32_t p, int dA, int dC, const ffa_opts* opts, ffa_batch** out);
int ffa_batch_offsets(const ffa_batch* b, int64_t* a_off, int64_t* lda, int64_t* c_off,
                      int64_t* a_total, int64_t* c_total);
int ffa_batch_syrk_exec(ffa_batch* b, const void* A_packed, void* C_packed);
/* Batched C_i = Low(A_i A_i^H) over F_{p^2} (as ffa_herk_modp2, one p = 3 mod 4),
 * with the packed layout, ownership and launch modes of the real batch.  The four
 * buffers (A_re, A_im, C_re, C_im) each hold the planes at the offsets that
 * ffa_batch_offsets reports, are 16-byte aligned, and key the captured graph
 * together.  FFA_EINVAL: a plan of the other kind, or a null or misaligned buffer. */
int ffa_batch_herk_plan(ffa_ctx* ctx, int64_t count, const int64_t* n, const int64_t* k,
                        uint32_t p, int dA, int dC, const ffa_opts* opts, ffa_batch** out);
int ffa_batch_herk_exec(ffa_batch* b, const void* A_re, const void* A_im, void* C_re, void* C_im);
int ffa_batch_destroy(ffa_batch* b);
/* The batch plan as JSON (the fields of ffa_plan_describe, summed or maximal over
 * the problems: levels is the deepest recursion, macs the total per limb product). */
int ffa_batch_describe(const ffa_batch* b, char* buf, int64_t size);

/* Phase timing with HIP events recorded on the context's stream around each
 * phase of every later call: 0 = conditioning, 1 = pre-additions (all levels),
 * 2 = products (the grouped launch and its last-round sums), 3 = post-additions
 * (all levels).  phases is a bit mask (bit q: phase q; 15 = every phase, 0 = off);
 * each recorded phase adds two events per call to the stream.
 * ffa_profile_read synchronises on the recorded events and returns the summed
 * milliseconds and the number of event pairs measured for the phase. */
int ffa_profile_enable(ffa_ctx* ctx, int phases);
int ffa_profile_read(ffa_ctx* ctx, int phase, double* total_ms, int64_t* calls);
int ffa_profile_reset(ffa_ctx* ctx);

/* Autotuner.  Times every candidate plan for this call (recursion depth 0..4 that
 * the sizes allow x carrier (INT8 limbs, and FP64 where its bound holds) x every
 * INT8 product-kernel configuration of the carrier x operand source, raw uint16 rows
 * where the planner allows them x general products, classical or Strassen-Winograd
 * where the recursion has general products on a real carrier) on the caller's own buffers
 * with HIP events, `reps` timed calls each, and records the fastest for the shape
 * (n, k, p, formats) in the context: later calls with opts = NULL use it, and
 * so do other shapes of the same size class (n and k within the same half-octave)
 * that have no record of their own.  C receives the (identical) result of every
 * candidate.  best (optional) receives the chosen options, best_ms its time per
 * call.  Synchronises the stream. */
int ffa_autotune_syrk(ffa_ctx* ctx, int64_t n, int64_t k, uint32_t p,
                      int dA, const void* A, int64_t lda, int dC, void* C, int64_t ldc,
                      int reps, ffa_opts* best, double* best_ms);
/* Same for a batch plan: re-plans with each carrier, product-kernel configuration,
 * recursion cutoff (classical, 256, 384) and operand source (limb planes, or raw
 * uint16 rows where the planner allows them), keeps the fastest in the plan.
 * Hermitian batches: FFA_EUNSUPPORTED. */
int ffa_batch_autotune(ffa_batch* b, const void* A_packed, void* C_packed, int reps,
                       ffa_opts* best, double* best_ms);

/* The context's autotuner records as JSON text
 *   {"arch":"gfx950","records":[{"n":..,"k":..,"p":..,"herm":..,"dA":..,"dC":..,
 *    "algo":..,"levels":..,"cutoff":..,"carrier":..,"kernel":..,"operands":..,
 *    "general":..,"wino_min":..}, ...]}
 * ("operands", "general" and "wino_min" may be absent on import: the built-in
 * choice then).
 * ffa_tune_export writes it into buf (NUL-terminated; nothing written when size is
 * too small) and returns the length it needs without the NUL, or a negative status.
 * ffa_tune_import adds the records of such a text (records for another arch are
 * skipped) and returns how many it took, or FFA_EINVAL for text it cannot read. */
int64_t ffa_tune_export(const ffa_ctx* ctx, char* buf, int64_t size);
int ffa_tune_import(ffa_ctx* ctx, const char* json);

/* Host-only description of the plan ffa_syrk_modp / ffa_herk_modp2 would use
 * (no device needed): writes a JSON object (levels, padded sizes, carrier,
 * limbs, workspace bytes, launches) into buf (NUL-terminated, truncated to
 * size).  Returns the validation status the call would return. */
int ffa_plan_describe(int64_t n, int64_t k, uint32_t p, int hermitian, int dA, int dC,
                      int64_t lda, int64_t ldc, const ffa_opts* opts, char* buf, int64_t size);

#ifdef __cplusplus
}
#endif

#endif /* FFA_H */
