/*
 * gpgomea_eval.h -- C ABI of the MI355X (gfx950) batched fitness evaluator for
 * GP-GOMEA template individuals.
 *
 * What is computed (the data-parallel hot path of GPU GP-GOMEA):
 *   Every individual is a postfix (Reverse Polish) program over the active
 *   nodes of a fixed-size tree template (Section 3.2, "Data Structure of
 *   Individuals", Fig. 1).  It is evaluated on every row of a dataset with a
 *   stack interpreter (Section 3.2, "Evaluation on the GPU"), and its squared
 *   errors are reduced to one fitness value per individual: the MSE of Eq. 1,
 *   or the MSE after the least-squares affine fit y ~ a + b*p (linear scaling;
 *   App. A.2 notes the paper's GPU path lacks it), with NMSE = fitness/Var(y)
 *   (Eq. 2, population variance).  gpgomea_grad_consts adds the gradient of
 *   that fitness with respect to every constant of every individual (path
 *   forward mode over the tree's root-to-constant paths; not in the paper).
 *   The batch is the set of changed offspring that Alg. 1 collects before its
 *   single Evaluate call.
 *
 * Conventions common to all entry points
 *   - Every pointer named "device" is GPU memory owned by the caller.  The
 *     library never allocates device memory and never reads device data on
 *     the host.  Scratch space is the caller's `workspace` buffer, of at least
 *     gpgomea_workspace_bytes(...) bytes, 256-byte aligned (the no-allocation
 *     entry point uses a static device array of the library instead).
 *   - `stream` is a hipStream_t (NULL = the default stream).  GPU entry points
 *     only enqueue work and return; outputs are valid after the stream has
 *     reached that point.  Inputs and the workspace must stay alive and
 *     unmodified until then.  Two calls that share a workspace must not run
 *     concurrently.
 *   - Return value: GPGOMEA_OK (0) or a negative GPGOMEA_E_* code; the message
 *     of the last failure on the calling thread is gpgomea_last_error().
 *     Argument and shape errors are detected on the host before anything is
 *     enqueued.  Per-individual problems never fail a call: they go to
 *     status[i] (1 = a prediction was NaN or infinite, fitness = +inf;
 *     2 = malformed program, fitness = +inf).
 *
 * Program encoding (one signed byte per postfix token, see gpgomea_ops.h):
 *   0 + | 1 - | 2 * | 3 protected / | 4 sin | 5 cos | 6 square | 7 sqrt|a|
 *   8 exp(clamp(a,-80,80)) | 9 protected log|a| | 10 protected pow
 *   32 constant (takes the next value of the individual's constant list)
 *   64+k variable k | -1 end / padding.
 *   Binary operators take the earlier-pushed operand as the left one.
 */
#ifndef GPGOMEA_EVAL_H
#define GPGOMEA_EVAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define GPGOMEA_OK 0
#define GPGOMEA_E_ARG (-1)         /* NULL pointer or invalid flag            */
#define GPGOMEA_E_SHAPE (-2)       /* a size is out of the supported range    */
#define GPGOMEA_E_PROGRAM (-3)     /* host codec: malformed program/genotype  */
#define GPGOMEA_E_HIP (-4)         /* a HIP runtime call failed               */
#define GPGOMEA_E_WORKSPACE (-5)   /* workspace too small or misaligned       */
#define GPGOMEA_E_UNSUPPORTED (-6) /* combination not implemented             */

/* ---- flags --------------------------------------------------------------- */
#define GPGOMEA_LINEAR_SCALING 0x1u /* fitness = LS-MSE; without it raw MSE (Eq. 1) */
#define GPGOMEA_FP64_NODES 0x2u     /* node arithmetic in binary64 (validation)     */
#define GPGOMEA_PLAIN 0x4u          /* one kernel launch per individual (baseline)  */
#define GPGOMEA_NO_GRAPH 0x8u       /* launch directly, no hipGraph capture/replay  */

/* ---- limits ------------------------------------------------------------- */
#define GPGOMEA_MAX_LEN 511    /* L_max: tokens per program (template depth 8)   */
#define GPGOMEA_MAX_CONSTS 256 /* C_max: constants per program                    */
#define GPGOMEA_MAX_FEATURES 64

/* Library version, major*10000 + minor*100 + patch. */
int gpgomea_version(void);

/* Message of the last failing call on this thread ("" if none).  The pointer
 * stays valid until the next call on this thread. */
const char* gpgomea_last_error(void);

/* Bytes of device workspace that gpgomea_eval_batch and gpgomea_grad_consts
 * need for this problem shape and flag set (same arguments as the calls).
 * Returns 0 if the shape is invalid (see gpgomea_last_error). */
size_t gpgomea_workspace_bytes(int32_t M, int32_t L_max, int32_t C_max, int32_t F, int64_t N,
                               uint32_t flags);

/* Fitness of a batch of M programs on one dataset.
 *   ops      device int8 [M][L_max]: postfix programs, END (-1) terminated or
 *            exactly L_max long.  1 <= L_max <= GPGOMEA_MAX_LEN.
 *   consts   device float [M][C_max]: constant list of each program, in order
 *            of appearance (a program may use at most C_max of them).
 *   X        device float [F][ldx]: feature-major dataset, row r of feature k
 *            at X[k*ldx + r]; ldx >= N.  1 <= F <= GPGOMEA_MAX_FEATURES.
 *   y        device float [N]: targets, N >= 1.
 *   flags    GPGOMEA_* bit set.
 *   fitness  device double [M] out: LS-MSE (LINEAR_SCALING) or MSE; +inf when
 *            status[i] != 0.
 *   aux      device double [M][4] out, or NULL: a, b (the fit; b = 0, a = mean y
 *            without LINEAR_SCALING or when Var(p) <= 1e-12*max(mean(p)^2, 1e-300)),
 *            raw MSE (Eq. 1), NMSE = fitness / Var(y) (Eq. 2).
 *   status   device int8 [M] out, or NULL: 0 ok, 1 non-finite, 2 bad program.
 * Errors: E_ARG (NULL required pointer, unknown flag), E_SHAPE (sizes),
 * E_WORKSPACE, E_HIP. */
int gpgomea_eval_batch(const int8_t* ops, int32_t M, int32_t L_max, const float* consts,
                       int32_t C_max, const float* X, int32_t F, int64_t N, int64_t ldx,
                       const float* y, uint32_t flags, double* fitness, double* aux,
                       int8_t* status, void* workspace, size_t workspace_bytes, void* stream);

/* No-allocation variant of gpgomea_eval_batch, for callers that cannot
 * allocate device memory or create library objects while they run: code
 * inside HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same inputs, outputs, flags and results as gpgomea_eval_batch
 * (the same kernels), but the scratch space is a file-scope device array of
 * the library of gpgomea_noalloc_scratch_bytes() bytes (64 MiB), held by each
 * GPU the library runs on until the process ends, and the call allocates
 * nothing (no hipMalloc or hipFree, no graph instantiation, no events: its
 * kernels are launched directly on `stream`).  The first call on a device
 * resolves the array's address there.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (other streams, other host
 * threads) race and must be serialised by the caller; the array keeps the
 * last call's contents, and every region a call reads is written by that
 * call first.  Errors: as gpgomea_eval_batch, and E_WORKSPACE when the shape
 * needs more scratch than the array holds (about M * (8 KiB + 16 L_max)
 * bytes). */
size_t gpgomea_noalloc_scratch_bytes(void);
int gpgomea_eval_batch_noalloc(const int8_t* ops, int32_t M, int32_t L_max, const float* consts,
                               int32_t C_max, const float* X, int32_t F, int64_t N, int64_t ldx,
                               const float* y, uint32_t flags, double* fitness, double* aux,
                               int8_t* status, void* stream);

/* Fitness and its gradient with respect to every constant.
 *   Same inputs and outputs as gpgomea_eval_batch, plus
 *   grad     device double [M][C_max] out: d fitness / d consts[i][j]; zero for
 *            unused constants and for individuals with status != 0.  May be
 *            NULL when C_max = 0 (there is nothing to differentiate).
 * With linear scaling the gradient is (2b/N) sum_r (a + b p_r - y_r) dp_r/dc_j
 * (the optimal a, b have zero partials); without it (2/N) sum_r (p_r - y_r)
 * dp_r/dc_j.  A protected operator's guarded branch and a clamp outside its
 * range have derivative 0 (a zero partial ends every derivative path through
 * it); sqrt|a| has derivative 0 at a = 0.  Node values are the binary32 ones
 * of the fitness; the chain-rule products dp_r/dc_j are formed in binary32,
 * each lane sums its rows of one row tile in binary32 (R/64 rows per lane)
 * and those lane sums are added in binary64.  Where a row span's binary32 sums are not
 * finite (a product formed from the leaves up left the binary32 range) that
 * span is recomputed with binary64 chain-rule products; an entry stays +-inf
 * or NaN only where the binary64 products overflow too.  FP64_NODES is not
 * supported here (E_UNSUPPORTED). */
int gpgomea_grad_consts(const int8_t* ops, int32_t M, int32_t L_max, const float* consts,
                        int32_t C_max, const float* X, int32_t F, int64_t N, int64_t ldx,
                        const float* y, uint32_t flags, double* fitness, double* aux,
                        double* grad, int8_t* status, void* workspace, size_t workspace_bytes,
                        void* stream);

/* ---- the paper's evaluation designs (comparators) ----------------------------
 * Section 3.2 ("Evaluation on the GPU") and Fig. 2 describe two ways to lay
 * the (program, row) sub-evaluations on the GPU; both are kept here so that
 * the fused batch path can be compared with them at the same accuracy.  Both
 * compute the raw MSE of Eq. 1 (no linear scaling, as in the paper's designs)
 * of M programs in the same encoding and layout as gpgomea_eval_batch, with
 * binary32 nodes and binary64 sums of squared errors.
 *   gpgomea_eval_design1: one workgroup of `block` threads per program (a
 *     power of two in [64, 1024]); the program sits in LDS, each thread
 *     interprets it for rows t, t + block, ... with a private operand stack
 *     and keeps its squared errors in a register; a tree reduction in LDS
 *     gives the program's sum.  One launch.
 *   gpgomea_eval_design2: `blocks_per_program` workgroups per program, each
 *     over one contiguous block of rows, write partial sums to `partial`
 *     (device double [M * blocks_per_program], scratch); a second kernel adds
 *     each program's partials.  Two launches.
 * fitness (device double [M]) gets the MSE; status (device int8 [M], or NULL)
 * 0 ok, 1 a prediction was not finite (fitness +inf), 2 bad program (unknown
 * symbol, variable >= F, more than C_max constants, more than 16 operands on
 * the stack, not exactly one result; fitness +inf).  Programs are not
 * compiled or validated beforehand: every check happens while interpreting.
 * Enqueued on `stream`; nothing is allocated.  Errors: E_SHAPE, E_ARG, E_HIP. */
int gpgomea_eval_design1(const int8_t* ops, int32_t M, int32_t L_max, const float* consts,
                         int32_t C_max, const float* X, int32_t F, int64_t N, int64_t ldx,
                         const float* y, int32_t block, double* fitness, int8_t* status,
                         void* stream);
int gpgomea_eval_design2(const int8_t* ops, int32_t M, int32_t L_max, const float* consts,
                         int32_t C_max, const float* X, int32_t F, int64_t N, int64_t ldx,
                         const float* y, int32_t block, int32_t blocks_per_program,
                         double* partial, double* fitness, int8_t* status, void* stream);

/* One Adam step (Kingma & Ba 2015, Alg. 1) on every program's constants, for
 * constant optimisation driven by gpgomea_grad_consts (the paper names
 * real-valued constant optimisation as the next thing to integrate with GPU
 * evaluation, Section 5).  All arrays are device memory, row i belonging to
 * program i:
 *   consts        float [M][C_max] in/out: the constants the gradient was taken
 *                 at; replaced by the step's result (entries whose gradient is
 *                 0, e.g. unused constants, do not move).
 *   grad, fitness double [M][C_max] and [M]: gpgomea_grad_consts's outputs at
 *                 `consts`.
 *   moments       float [2][M][C_max] in/out: first and second moments; zero
 *                 before step t = 1.
 *   best_consts, best_fitness  float [M][C_max], double [M] in/out: the best
 *                 point seen; before t = 1 set best_fitness to +inf (and
 *                 best_consts to the start).  A program whose fitness is
 *                 strictly below best_fitness copies `consts` (the point the
 *                 fitness belongs to) into best_consts first.
 *   t             step number, 1, 2, ... (bias corrections 1 - beta^t).
 * A program whose fitness is not finite returns to best_consts and restarts
 * its moments.  lr = 0 only records the best point.  The moments and the
 * step are binary32; 1 - beta and the bias corrections are formed in binary64
 * from the given values.  Enqueued on `stream`;
 * nothing is allocated.  Errors: E_SHAPE, E_ARG (NULL arrays, t < 1, lr < 0,
 * betas outside [0, 1), eps <= 0), E_HIP. */
int gpgomea_adam_consts(float* consts, int32_t M, int32_t C_max, const double* grad,
                        const double* fitness, float* moments, float* best_consts,
                        double* best_fitness, int32_t t, double lr, double beta1, double beta2,
                        double eps, void* stream);

/* ---- host-side codec (no GPU needed) --------------------------------------
 * Genotype: int8 genes[M][T] heap-ordered over a full binary template (children
 * of slot s at 2s+1, 2s+2; unary operators read 2s+1), float gene_consts[M][T],
 * T = 2^(H+1)-1.  Individual i has height heights[i] (or `height` for all if
 * heights is NULL); slots past its own template are ignored.
 *
 * gpgomea_encode: post-order traversal of the active nodes (introns dropped),
 * Section 3.2 and Fig. 1.  Writes ops[M][L_max] (END padded), consts[M][C_max]
 * (zero padded, float bit patterns copied), len[M], nconst[M] (either may be
 * NULL).  Fails with E_PROGRAM (an active slot holds no symbol, an operator is
 * active at a leaf slot, or the program exceeds L_max / C_max); on failure
 * *bad_index (if not NULL) names the individual. */
int gpgomea_encode(const int8_t* genes, const float* gene_consts, int32_t M, int32_t T,
                   int32_t height, const int8_t* heights, int8_t* ops, int32_t L_max,
                   float* consts, int32_t C_max, int16_t* len, int16_t* nconst,
                   int32_t* bad_index);

/* gpgomea_decode: rebuild heap-ordered genotypes of height `height` from
 * postfix programs, the inverse of gpgomea_encode on the active nodes (Section
 * 3.2, Fig. 1: a postfix program determines its tree, and the tree's root sits
 * at heap slot 0 with operands in order).  Every other slot becomes -1 with
 * constant 0.  genes[M][2^(height+1)-1] and gene_consts of the same shape are
 * written by the call (host memory, caller-owned).  E_PROGRAM if a program is
 * malformed or taller than the template; *bad_index (if not NULL) names it. */
int gpgomea_decode(const int8_t* ops, const float* consts, int32_t M, int32_t L_max,
                   int32_t C_max, int32_t height, int8_t* genes, float* gene_consts,
                   int32_t* bad_index);

/* gpgomea_validate: check host-resident postfix programs (Section 3.2's
 * population arrays, END padded to L_max) the way the device does, and
 * optionally against a template height.  A program is invalid (status 2) if
 * it holds an unknown symbol, a variable >= F or more than C_max constants,
 * underflows the stack, does not leave exactly one result, or, when
 * max_height >= 0, its tree is taller than max_height (a terminal has height
 * 0, an operator one more than its tallest operand: the depth of a template
 * of that height, Section 3.1).  max_height = -1 skips the height check.
 * status_out[M] (host, may be NULL) receives 0 or 2 per program; *first_bad
 * (may be NULL) the index of the first invalid program or -1.  Returns the
 * number of invalid programs (>= 0), or E_ARG / E_SHAPE before any program is
 * read. */
int gpgomea_validate(const int8_t* ops, int32_t M, int32_t L_max, int32_t C_max, int32_t F,
                     int32_t max_height, int8_t* status_out, int32_t* first_bad);

/* ---- tuning -----------------------------------------------------------------
 * gpgomea_autotune: time the fused kernels over their launch parameters
 * (forward: rows per lane, rows per LDS tile, individuals per group; adjoint:
 * rows per LDS tile, entries per group, rows per lane of each constant class)
 * on a prefix of at most 2^20 rows of the given device inputs, keep the
 * fastest choice for this problem class (precision, log2 L_max, F, log2 N,
 * log2 M, gradient or not)
 * in the process-wide table and, if cache_path is not NULL, merge it into that
 * JSON file.  Synchronises `stream`.  `trials` = timed repetitions per
 * candidate (>= 1).  Writes a one-line description of the choice to
 * `out_desc` (if not NULL, up to desc_len bytes). */
int gpgomea_autotune(const int8_t* ops, int32_t M, int32_t L_max, const float* consts,
                     int32_t C_max, const float* X, int32_t F, int64_t N, int64_t ldx,
                     const float* y, uint32_t flags, int32_t with_grad, void* workspace,
                     size_t workspace_bytes, const char* cache_path, int32_t trials,
                     char* out_desc, int32_t desc_len, void* stream);

/* Load a tuning JSON file written by gpgomea_autotune into the process-wide
 * table (E_ARG if unreadable). */
int gpgomea_load_tuning(const char* cache_path);

/* Graph cache.  A call on a non-default stream (without NO_GRAPH) runs as one
 * hipGraph launch.  Executable graphs are cached per (stream, shapes other
 * than M, flags, launch plan); a call whose pointers or M differ from the
 * cached graph's captures its launch sequence again and updates the cached
 * graph in place (after that graph's previous launch has completed), so a
 * changing batch size or new output buffers reuse it.  At most 16 graphs are
 * kept; the least recently used is destroyed (after its last launch
 * completes).  gpgomea_clear_graphs drops them all; gpgomea_graph_count
 * returns how many are cached. */
int gpgomea_clear_graphs(void);
int gpgomea_graph_count(void);

/* ---- measurement -------------------------------------------------------------
 * gpgomea_profile(1): every kernel a later call enqueues is bracketed by a pair
 * of hipEvents on that call's stream (hipGraph capture is bypassed meanwhile);
 * gpgomea_profile(0) stops.  gpgomea_profile_report writes one line per
 * kernel kind, "name launches total_ms\n", for everything recorded since the
 * previous report (it waits for those events), and clears the record.  With
 * buf == NULL it returns the buffer size needed; otherwise the bytes written. */
int gpgomea_profile(int32_t enable);
int gpgomea_profile_report(char* buf, int32_t len);

/* gpgomea_op_costs: vector-ALU cost of each protected operator as the
 * interpreter executes it, measured on the current device: out[op] (host, n >=
 * 17 doubles, op in the library's internal numbering: 1 +, 2 -, 3 reversed -,
 * 4 *, 5 /, 6 reversed /, 7 pow, 8 reversed pow, 9 sin, 10 cos, 11 square,
 * 12 sqrt, 13 exp, 14 log; out[16] = the binary64 moment update per row) in
 * seconds per lane-application, from kernels that apply the same device
 * routine `iters` times to independent values in every lane of a full grid.
 * dev_scratch: device float [2048] (never read back).  Synchronises `stream`. */
int gpgomea_op_costs(double* out, int32_t n, int32_t iters, float* dev_scratch, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* GPGOMEA_EVAL_H */
