/*
 * gpeval.h -- C ABI of the MI355X (gfx950) batched fitness evaluator for
 * postfix symbolic-regression programs.
 *
 * What it computes ("Scoring" in the paper's Table 1; the GPU side of
 * Sec. "Dividing Tasks Between CPU and GPU"): every program of a population
 * is run over every fitness case, and one aggregate per program comes back:
 *
 *   F(p) = MSE(p) + tax_on_length * len(p)      for a valid program
 *   F(p) = +INFINITY  if for some case exactly one of f_p(x_i) and y_i is
 *                     NaN or +-inf, or MSE(p) > FLT_MAX
 *   MSE(p) = (1/n) * sum over valid pairs i of (f_p(x_i) - y_i)^2
 *
 * A valid pair is a case whose output and target are both finite; a case
 * where both are NaN/inf is a matched invalid pair and adds nothing (Sec.
 * "Fitness Functions": invalid values in the output or the dataset are
 * handled as in Eq. 2, which rewards matched invalid pairs).  With finite
 * targets: any NaN/inf case output gives +INFINITY.
 *
 * f_p is the reverse-Polish evaluation of p (Sec. "Genome Computer Language
 * (GCL)": unary ops replace the top of the stack, binary ops replace the top
 * two; at most 32 stack elements; command semantics and operand order of
 * the GCL command table).  Readings where the paper is silent: DIV is
 * protected (|b| <= fp32(0.001) gives 1, else a/b; a NaN divisor gives
 * NaN), LOG (the paper's LN) is protected (|a| <= fp32(0.001) gives 0, else
 * ln|a|), SQRT is sqrt(|a|), ABS is |a|.  len(p) counts every node, leaves
 * included ("Tax on Length", Table 1; ScriptLengthTaxRateInternal).
 *
 * Arithmetic: each case is evaluated in fp32; squared residuals are summed
 * in Kahan-compensated fp32 (power-of-two pre-scaled so no partial sum can
 * exceed the MSE); the per-program cross-block sum, the tax and the
 * classification are fp64.  Program decoding and indexing are exact.
 *
 * Program format (device arrays, caller owned):
 *   nodes   uint32[n_nodes]    node = op | (arg << 8)
 *   offsets int64[n_programs+1] program p = nodes[offsets[p] .. offsets[p+1])
 *   consts  float32[n_consts]  constant pool; CONST's arg indexes it
 * Fitness cases (device arrays, caller owned, resident across calls):
 *   X       float32, variable major: case i of variable v at X[v*ld_x + i]
 *   y       float32[n_cases]   targets
 *
 * Errors: functions return GP_OK (0) or a negative gp_status; nothing aborts
 * or throws across the ABI.  gp_last_error() gives a thread-local message.
 * Argument checks are synchronous; device faults surface as GP_E_HIP.
 * A program that fails validation on the device (bad opcode or operand,
 * stack underflow, depth > 32, final depth != 1, empty, op not allowed) is
 * never run: its out_fitness is NaN and its out_status (if requested) is
 * the nonzero GP_PROG_* code.
 */
#ifndef GPEVAL_H
#define GPEVAL_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GPEVAL_VERSION 1
#define GP_MAX_STACK 32           /* stack limit (StackSize in the GCL section) */
#define GP_MAX_CONSTS (1 << 24)   /* a node's arg field has 24 bits */
#define GP_MAX_VARS (1 << 24)
#define GP_MAX_REWARD_SCORE 16777216.0   /* |M| of gp_eval_reward: 2^24 */

enum gp_status {
    GP_OK = 0,
    GP_E_INVALID_ARG = -1,   /* null pointer, negative size, ld_x < n_cases, ... */
    GP_E_BAD_PROGRAM = -2,   /* gp_validate found an invalid program */
    GP_E_TOO_LARGE = -3,     /* a size exceeds a documented limit */
    GP_E_NO_MEMORY = -4,     /* device workspace allocation failed */
    GP_E_HIP = -5,           /* a HIP runtime call failed */
    GP_E_CANCELLED = -6      /* a server request was cancelled (gp_server_cancel) */
};

/* Opcodes (GCL command table; ABS is not a GCL command).  0-11 are the
 * benchmark set; 12-27 complete the paper's command table. */
enum gp_op {
    GP_LOAD = 0,    /* push X[arg][i]; arg = zero-based input index   */
    GP_CONST = 1,   /* push consts[arg]                               */
    GP_ADD = 2,     /* a b -> a + b   (b = top, a = second from top)  */
    GP_SUB = 3,     /* a b -> a - b                                   */
    GP_MUL = 4,     /* a b -> a * b                                   */
    GP_DIV = 5,     /* a b -> |b| <= fp32(0.001) ? 1 : a / b          */
    GP_SIN = 6,     /* a -> sin a                                     */
    GP_COS = 7,     /* a -> cos a                                     */
    GP_EXP = 8,     /* a -> e^a                                       */
    GP_LOG = 9,     /* a -> |a| <= fp32(0.001) ? 0 : ln |a|           */
    GP_SQRT = 10,   /* a -> sqrt |a|                                  */
    GP_ABS = 11,    /* a -> |a|                                       */
    GP_DUP = 12,    /* a -> a a                                       */
    GP_SWAP = 13,   /* a b -> b a                                     */
    GP_DEL = 14,    /* a -> (nothing)                                 */
    GP_SQUARE = 15, /* a -> a * a                                     */
    GP_SIGN = 16,   /* a -> -a                                        */
    GP_CUBE = 17,   /* a -> a * a * a (rounded once)                  */
    GP_CBRT = 18,   /* a -> cube root of a (real, any sign)           */
    GP_TAN = 19,    /* a -> tan a                                     */
    GP_ASIN = 20,   /* a -> arcsin a (NaN outside [-1, 1])            */
    GP_ACOS = 21,   /* a -> arccos a (NaN outside [-1, 1])            */
    GP_ATAN = 22,   /* a -> arctan a                                  */
    GP_TANH = 23,   /* a -> tanh a                                    */
    GP_SQRT_RAW = 24, /* a -> sqrt a (NaN below zero; the paper's SQRT) */
    GP_POW = 25,    /* a b -> a^b (C99 pow special cases)             */
    GP_COPY = 26,   /* variable @arg := top; the stack is unchanged  */
    GP_PASTE = 27,  /* push variable @arg; the variable is freed      */
    GP_N_OPS = 28
};
#define GP_ALL_OPS ((1u << GP_N_OPS) - 1u)
/* The benchmark set LOAD..ABS.  Every entry point takes op masks within
 * GP_ALL_OPS (a bit beyond it gives GP_E_INVALID_ARG before device work).
 * For the scoring entry points (gp_eval, gp_eval_noalloc,
 * gp_eval_correlation, gp_eval_reward, gp_eval_batched, plans, the server)
 * 0 means GP_BASE_OPS; for gp_validate and gp_predict 0 means GP_ALL_OPS.
 * A mask that reaches beyond GP_BASE_OPS runs an interpreter built for the
 * whole command table (same values for the benchmark set's commands; more
 * registers, so fewer wavefronts per SIMD). */
#define GP_BASE_OPS ((1u << 12) - 1u)
/* COPY/PASTE variable names: @0 .. @15.  A valid program copies into a free
 * variable only, pastes a held one only, and ends with every variable
 * free; a held variable takes one of the GP_MAX_STACK cells, so the stack
 * depth plus the held variables never exceeds GP_MAX_STACK (else
 * GP_PROG_TOO_DEEP). */
#define GP_GCL_VARS 16

/* Per-program validation codes. */
enum gp_prog_status {
    GP_PROG_OK = 0, GP_PROG_EMPTY = 1, GP_PROG_BAD_OP = 2, GP_PROG_BAD_VAR = 3,
    GP_PROG_BAD_CONST = 4, GP_PROG_UNDERFLOW = 5, GP_PROG_TOO_DEEP = 6,
    GP_PROG_FINAL_DEPTH = 7, GP_PROG_BAD_OFFSETS = 8,
    GP_PROG_BAD_TABLE = 9,    /* gp_eval_batched: invalid dataset/request table */
    GP_PROG_BAD_PAIR = 10     /* COPY/PASTE not paired (see GP_GCL_VARS) */
};

/* Thread-local text for the last non-OK status returned on this thread. */
const char* gp_last_error(void);

/* Library version (GPEVAL_VERSION of the build). */
int gp_version(void);

/*
 * gp_validate -- host-side check of a population (host pointers).
 * allowed_op_mask: bit op set = op allowed (GetAllowedOperations in the
 * optional MLSetup overrides); 0 means GP_ALL_OPS.  status/max_depth:
 * optional host arrays of n_programs entries; max_depth is the largest
 * stack depth plus held variables over the program.  *first_bad (optional) gets
 * the first invalid program index or -1.  Returns GP_OK when every program
 * is valid, GP_E_BAD_PROGRAM otherwise.  Pure and thread-safe.
 */
int gp_validate(const uint32_t* nodes, const int64_t* offsets, int64_t n_programs,
                int64_t n_consts, int32_t n_vars, uint32_t allowed_op_mask,
                int32_t* status, int32_t* max_depth, int64_t* first_bad);

/*
 * gp_eval -- score a population (all pointers are device pointers).
 * n_nodes = offsets[n_programs] (the total node count; needed to size the
 * staging buffer without reading device memory).  X has n_vars rows of
 * leading dimension ld_x >= n_cases.  out_fitness: n_programs doubles.
 * out_status: optional (may be NULL) n_programs int32 GP_PROG_* codes.
 * Asynchronous on `stream`; results are valid after the stream has
 * synchronized.  Inputs must stay alive until then.  The library keeps a
 * per-(device, stream) workspace that grows on demand; concurrent calls on
 * one stream from several host threads are not supported.
 * allowed_op_mask: within GP_ALL_OPS (0 means GP_BASE_OPS; a bit beyond
 * GP_ALL_OPS is GP_E_INVALID_ARG).
 * Determinism: a program's result depends only on the program, the data and
 * n_cases, never on the rest of the population.
 */
int gp_eval(const uint32_t* nodes, const int64_t* offsets, int64_t n_programs,
            int64_t n_nodes, const float* consts, int64_t n_consts,
            const float* X, int32_t n_vars, int64_t ld_x,
            const float* y, int64_t n_cases,
            double tax_on_length, uint32_t allowed_op_mask,
            double* out_fitness, int32_t* out_status, hipStream_t stream);

/*
 * gp_eval_noalloc -- gp_eval with no device allocation, for callers that
 * cannot allocate: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Arguments, result and determinism as
 * gp_eval (the same kernels, so the same bits).  The workspace is a fixed
 * device array of GP_NOALLOC_WORKSPACE_BYTES (64 MiB) that each GPU the
 * library runs on holds until the process ends; the first call on a device
 * takes its address (set-up), later calls make no allocating call of any
 * kind.  Every depth class runs on `stream` (no side streams) and no
 * timing events are recorded.  Returns GP_E_TOO_LARGE, before any device
 * work, when the call needs more workspace than the array holds (about 8
 * bytes per node plus 27 per program plus 9 per (program, case tile);
 * gp_workspace_size reports the need, with 25% slack); other errors as
 * gp_eval.  Every call on one GPU shares that GPU's array: calls that
 * overlap in time on one GPU (several streams or host threads) race, and
 * the caller must order them (one stream, or events).
 */
#define GP_NOALLOC_WORKSPACE_BYTES (64ull << 20)
int gp_eval_noalloc(const uint32_t* nodes, const int64_t* offsets, int64_t n_programs,
                    int64_t n_nodes, const float* consts, int64_t n_consts,
                    const float* X, int32_t n_vars, int64_t ld_x,
                    const float* y, int64_t n_cases,
                    double tax_on_length, uint32_t allowed_op_mask,
                    double* out_fitness, int32_t* out_status, hipStream_t stream);

/*
 * gp_eval_correlation -- score a population with the correlation fitness
 * (the paper's default, Sec. "Fitness Functions", Eq. 1 and Eq. 2), all
 * pointers device pointers, arguments as for gp_eval (no length tax).
 * Per program, over its N = n_cases cases: a valid pair is a case whose
 * output and target are both finite; c1 counts cases with exactly one of
 * the two invalid, c2 cases with both invalid; r is Pearson's coefficient
 * over the valid pairs (0 below two valid pairs or for a constant output or
 * target); out_score = M (r^2)^2 (N - (c1 + c2)) - M (c1 - c2), M =
 * max_score (the paper's maximum score; higher is better).  Invalid
 * programs get NaN and their GP_PROG_* status.  The sums are fp64 sums of
 * shifted values (f - s, (f - s)^2, y - t, (y - t)^2, (f - s)(y - t), the
 * shift (s, t) one valid pair of the data) over the case tiles, merged in a
 * fixed order with exact shift changes: results are deterministic and
 * independent of the rest of the population.  Returns GP_E_INVALID_ARG for
 * a non-finite max_score; other errors as gp_eval.  The workspace's partial
 * buffer takes 80 bytes per (program, tile) instead of 9
 * (gp_workspace_size reports the MSE layout).
 */
int gp_eval_correlation(const uint32_t* nodes, const int64_t* offsets, int64_t n_programs,
                        int64_t n_nodes, const float* consts, int64_t n_consts,
                        const float* X, int32_t n_vars, int64_t ld_x,
                        const float* y, int64_t n_cases, double max_score,
                        uint32_t allowed_op_mask, double* out_score, int32_t* out_status,
                        hipStream_t stream);

/*
 * gp_eval_reward -- score a population with the point-to-point integer
 * reward (Sec. "Fitness Functions", Eq. 5 for power 1, StdFitFunc, and its
 * Square, Cube and Hyper variants for power 2, 3 and 8), all pointers
 * device pointers, arguments as for gp_eval (no length tax).  M = max_score
 * is the paper's maximum score, an integer (exact in fp32).  Per case, in
 * fp32, with o the program's output and y the target:
 *   o and y both finite:  M if max(|o|,|y|) = 0; otherwise
 *                         rint(M * q^power - [sign(o) = -sign(y) != 0] * M/11)
 *                         with q = min(|o|,|y|) / max(|o|,|y|), q^power
 *                         formed by repeated fp32 products (q*q, (q*q)*q,
 *                         ((q*q)^2)^2) and rint rounding half to even;
 *   exactly one invalid:  -M;   both invalid: +M.
 * out_reward is the sum
 * over the cases in int64, converted to double (exact while |sum| < 2^53);
 * higher is better.  Invalid programs get NaN and their GP_PROG_* status.
 * The integer sum makes the result independent of summation order: the
 * output is deterministic.  Returns GP_E_INVALID_ARG for a max_score that
 * is not an integer or exceeds GP_MAX_REWARD_SCORE in magnitude, or a power
 * other than 1, 2, 3, 8; other errors as gp_eval.  The workspace's partial
 * buffer takes 8 bytes per (program, tile).
 */
int gp_eval_reward(const uint32_t* nodes, const int64_t* offsets, int64_t n_programs,
                   int64_t n_nodes, const float* consts, int64_t n_consts,
                   const float* X, int32_t n_vars, int64_t ld_x,
                   const float* y, int64_t n_cases, double max_score, int32_t power,
                   uint32_t allowed_op_mask, double* out_reward, int32_t* out_status,
                   hipStream_t stream);

/*
 * gp_mc_rank -- the paper's Monte-Carlo ranking (Sec. "Monte-Carlo
 * Ranking", Table 2) on the device, without sorting the population.  All
 * pointers are device pointers; asynchronous on `stream`.
 *   fitness         n doubles (e.g. the output of gp_eval: lower is better,
 *                   higher_is_better = 0; or of gp_eval_correlation: 1).
 *                   NaN is the worst value and ties with -inf (after the
 *                   direction is applied).
 *   seed            the sample: draw k (0 <= k < sample_size) is individual
 *                   floor(h_k * n / 2^64), h_k the k-th SplitMix64 output
 *                   of the sequence started at seed (with replacement).
 *   sample_size     1..1024 (the paper samples 100).
 *   out_band        n int32: 10 * floor(p / 10), capped at 90, where the
 *                   percentile p = floor(100 * (sampled values strictly
 *                   worse than the individual) / sample_size).
 *   out_children    optional n floats: the band's expected number of
 *                   children (Table 2: 4, 2.5, 1.5, 1, 0.5, 0.25, 0.15,
 *                   0.06, 0.03, 0.01 from the top band down).
 *   out_sample_keys optional sample_size doubles: the sampled values,
 *                   larger-is-better keys (v or -v, NaN as -inf), ascending.
 * Integer work: results are exact and depend only on (fitness, seed,
 * sample_size, direction).  Errors: GP_E_INVALID_ARG for n < 0, a sample
 * size out of range, or NULL fitness/out_band with n > 0.
 */
int gp_mc_rank(const double* fitness, int64_t n, int32_t higher_is_better, uint64_t seed,
               int32_t sample_size, int32_t* out_band, float* out_children,
               double* out_sample_keys, hipStream_t stream);

/*
 * gp_eval_batched -- score the populations of several requests, each
 * against its own resident dataset, in one launch (scoring requests of
 * many concurrent evolutionary runs; the paper spreads populations over
 * the available devices and batches them, Sec. "Hardware Optimized").
 *
 * requests_dev: n_requests device entries; each names its own program
 * arrays (same format as gp_eval), its dataset (index into datasets_dev)
 * and its own outputs (out_fitness: n_programs doubles; out_status: NULL
 * or n_programs ints).  datasets_dev: n_datasets device entries (X, y,
 * n_vars, ld_x, n_cases, tax as in gp_eval).  The host passes the sums of
 * n_programs and n_nodes over the requests and upper bounds on n_vars and
 * n_cases (they size the workspace and LDS tiles).  Requests may be empty
 * (n_programs 0).  Host-side errors: GP_E_INVALID_ARG for NULL tables or
 * counts < 1, GP_E_TOO_LARGE for more than 4096 requests or sizes beyond
 * gp_eval's limits.  Device-side: if the tables are inconsistent with the
 * host's totals and bounds (a count out of range, a NULL array that is
 * needed, a dataset index out of range, sums that differ), no program is
 * evaluated and every program gets NaN and GP_PROG_BAD_TABLE, written
 * only where a request's own entry makes the write safe.  Each program's
 * result is bit-identical to scoring its request alone with gp_eval on
 * the same dataset.  Nothing is copied: the call reads the programs where
 * they are, so inputs must stay alive until the stream has passed it.
 */
typedef struct {
    const float* X; const float* y;
    int64_t ld_x; int64_t n_cases;
    double tax_on_length;
    int32_t n_vars; int32_t reserved;
} gp_dataset;

typedef struct {
    const uint32_t* nodes; const int64_t* offsets; const float* consts;
    int64_t n_programs; int64_t n_nodes; int64_t n_consts;
    double* out_fitness; int32_t* out_status;
    int32_t dataset; int32_t reserved;
} gp_request;

int gp_eval_batched(const gp_request* requests_dev, int32_t n_requests,
                    const gp_dataset* datasets_dev, int32_t n_datasets,
                    int64_t total_programs, int64_t total_nodes,
                    int32_t max_n_vars, int64_t max_n_cases, uint32_t allowed_op_mask,
                    hipStream_t stream);

/*
 * gp_predict -- per-case outputs f_p(x_i) of every program (the paper's
 * ExecuteGenome utility, Sec. "Useful Utilities": run a genome on input
 * data).  Same program and input arguments as gp_eval (device pointers);
 * out: float32, out[p * ld_out + i] for i < n_cases, ld_out >= n_cases,
 * caller-owned device memory of n_programs * ld_out floats.  Values are the
 * fp32 results of the same interpreter gp_eval runs (NaN and +-inf kept).
 * allowed_op_mask may reach beyond GP_BASE_OPS (0 means GP_ALL_OPS): then
 * the interpreter built for the whole command table runs.
 * Programs that fail validation get a NaN row and a nonzero out_status.
 * Asynchronous on `stream`; shares gp_eval's per-stream workspace.
 */
int gp_predict(const uint32_t* nodes, const int64_t* offsets, int64_t n_programs,
               int64_t n_nodes, const float* consts, int64_t n_consts,
               const float* X, int32_t n_vars, int64_t ld_x, int64_t n_cases,
               uint32_t allowed_op_mask, float* out, int64_t ld_out, int32_t* out_status,
               hipStream_t stream);

/*
 * Plans: one population shape evaluated generation after generation (the
 * paper's loop uploads a new population each generation and scores it,
 * Sec. "Dividing Tasks Between CPU and GPU").  A plan owns its workspace,
 * captures the whole pipeline (validation and staging, the partition by
 * stack depth class and program length -- longest first --, the persistent
 * per-class evaluation kernels and the fp64 reduction) into a hipGraph
 * once, and replays it with gp_plan_launch.  The caller rewrites the
 * program/data buffers in place between launches (same pointers, same
 * sizes) or calls gp_plan_update for new pointers or sizes (re-capture).
 *
 * gp_tuning holds launch knobs; 0 fields mean defaults.  programs_per_item,
 * wg_per_cu and concurrent_classes change no result.  tile_lds_bytes and
 * max_tiles shape how a program's cases are grouped into LDS windows and
 * case tiles, which fixes its summation order together with n_cases, n_vars
 * and its stack depth: every launch with the same knobs gives the same bits,
 * and the defaults (24 KiB, 32 tiles) give gp_eval's bits; other values may
 * differ from gp_eval in the last bits (within the fitness tolerance).
 * With autotune != 0, gp_plan_create times candidate knobs on the given
 * inputs (coordinate descent over the five knobs, two sweeps, the median
 * of five runs per candidate, then a run-off of the three fastest: this
 * runs the evaluation about 140 times and synchronizes `stream`) and keeps
 * the fastest; results are cached per workload shape (device, cases, variables,
 * programs, mean length, requests) in the process and, if the environment
 * variable GPEVAL_TUNE_CACHE names a file, there too.
 */
typedef struct {
    const uint32_t* nodes; const int64_t* offsets; int64_t n_programs; int64_t n_nodes;
    const float* consts; int64_t n_consts;
    const float* X; int32_t n_vars; int64_t ld_x;
    const float* y; int64_t n_cases;
    double tax_on_length; uint32_t allowed_op_mask;
    double* out_fitness; int32_t* out_status;       /* out_status may be NULL */
} gp_problem;                                       /* same meaning as gp_eval's arguments */

typedef struct {
    int32_t programs_per_item;   /* most programs per work item, 1..128 (default 64);
                                    a depth class with few programs uses fewer */
    int32_t wg_per_cu;           /* persistent workgroups per CU, 0 = occupancy limit */
    int32_t concurrent_classes;  /* 1: depth classes run on forked streams; 2: as 1,
                                    and the depth <= 8 class runs one workgroup
                                    per CU below its limit, so that the deeper
                                    classes (whose wavefronts issue first) run
                                    beside it from the start */
    int32_t tile_lds_bytes;      /* LDS budget of an input window, 4096..65536
                                    (default 24576) */
    int32_t max_tiles;           /* case tiles per program, at most, 1..32
                                    (default 32) */
} gp_tuning;

typedef struct gp_plan gp_plan;

/* Create (and capture) a plan; tuning may be NULL.  GP_E_* on failure. */
int gp_plan_create(gp_plan** plan, const gp_problem* problem, const gp_tuning* tuning,
                   int autotune, hipStream_t stream);
/* Replay the captured evaluation on `stream` (asynchronous). */
int gp_plan_launch(gp_plan* plan, hipStream_t stream);
/* Point the plan at new buffers/sizes and re-capture (synchronous). */
int gp_plan_update(gp_plan* plan, const gp_problem* problem);
/* The scheduling knobs the plan uses (after autotuning, if requested). */
int gp_plan_get_tuning(const gp_plan* plan, gp_tuning* out);
/* Waits for outstanding work and frees the plan.  NULL is ignored. */
void gp_plan_destroy(gp_plan* plan);

/* Release every cached workspace of the calling process (all devices). */
void gp_release_workspaces(void);

/* ---------------------------------------------------------------- serving
 * gp_server -- a scoring service shared by many concurrent evolutionary
 * runs.  The paper scores each generation's whole population in one
 * device pass and splits populations into batches that fit device memory
 * (Sec. "Hardware Optimized"); here many runs share one device:
 *   - datasets are uploaded once (gp_server_add_dataset) and stay resident;
 *   - a request (one population, host arrays) is admitted when the device
 *     budget covers its program and output buffers, then uploaded through
 *     pinned staging on a copy stream;
 *   - requests are split into chunks (program ranges) of bounded work and
 *     workspace, and every admitted chunk goes into the next
 *     gp_eval_batched launch; up to n_streams launches are in flight, so
 *     requests that arrive while others run join the next launch
 *     (continuous batching);
 *   - results are copied back per request; latency is measured from
 *     gp_server_submit to the moment the results are in the caller's
 *     arrays;
 *   - a failed launch fails no request by itself: each request it held is
 *     retried once in launches of its own, and only a request whose retry
 *     fails too completes with the error (the others are unaffected);
 *   - a request can be cancelled (gp_server_cancel) until it completes.
 * Each program's result is bit-identical to gp_eval of its population
 * alone.  A scheduler thread owned by the server does all device work; the
 * functions below may be called from any thread.
 */
typedef struct gp_server gp_server;

typedef struct {
    int64_t device_budget_bytes;    /* datasets + requests + launch workspaces
                                       (0: 8 GiB) */
    int64_t pinned_bytes;           /* host staging (0: min(budget, 1 GiB)) */
    int64_t chunk_node_evals;       /* work per chunk, in length x cases
                                       (0: 2^35) */
    int64_t batch_node_evals;       /* work per launch (0: 4 chunks); a launch
                                       takes at least one chunk */
    int32_t n_streams;              /* launches in flight, 1..8 (0: 2) */
    int32_t max_batch_chunks;       /* chunks per launch, 1..4096 (0: 1024) */
    int32_t one_launch_per_request; /* 1: FIFO, one gp_eval per request on one
                                       stream, no chunking (comparison mode) */
    uint32_t allowed_op_mask;       /* within GP_ALL_OPS (0: GP_BASE_OPS) */
} gp_server_config;

typedef struct {
    int64_t submitted, completed, failed;
    int64_t launches, chunks_launched;
    double node_evals;              /* sum of length x n_cases, completed requests */
    double latency_p50_ms, latency_p99_ms, latency_max_ms, latency_mean_ms;
    double busy_ms;                 /* wall time with >= 1 launch in flight */
    double wall_ms;                 /* since creation or the last reset */
    int64_t device_bytes_in_use, device_bytes_peak;
    int32_t waiting, in_flight;     /* requests not admitted / admitted, not done */
    int64_t cancelled;              /* requests completed with GP_E_CANCELLED */
    int64_t retried;                /* requests sent to a retry of their own
                                       after a failed launch */
} gp_server_stats;

/* Creates the server, its streams (default priority), device arena and
 * pinned staging, and its scheduler thread on the current device.
 * GP_E_NO_MEMORY if the budget cannot be allocated. */
int gp_server_create(gp_server** server, const gp_server_config* config);

/* Uploads X (host, X[v * ld_x + i]) and y (host, n_cases) into the
 * server's arena; synchronous.  *dataset_id names it in submits.
 * GP_E_NO_MEMORY if the arena cannot hold it now. */
int gp_server_add_dataset(gp_server* server, const float* X, int32_t n_vars, int64_t ld_x,
                          const float* y, int64_t n_cases, double tax_on_length,
                          int32_t* dataset_id);

/* Frees a dataset; GP_E_INVALID_ARG while requests on it are pending. */
int gp_server_remove_dataset(gp_server* server, int32_t dataset_id);

/* Queues a scoring request.  Host arrays as in gp_eval (nodes[n_nodes],
 * offsets[n_programs + 1], consts[n_consts]); offsets must be
 * non-decreasing within [0, n_nodes] (GP_E_INVALID_ARG otherwise).  The
 * server reads the program arrays until the request completes and then
 * writes out_fitness[n_programs] and, if not NULL, out_status[n_programs];
 * the caller keeps all of them alive and unchanged until then.
 * GP_E_TOO_LARGE if the request could never fit the budget. */
int gp_server_submit(gp_server* server, int32_t dataset_id, const uint32_t* nodes,
                     int64_t n_nodes, const int64_t* offsets, int64_t n_programs,
                     const float* consts, int64_t n_consts, double* out_fitness,
                     int32_t* out_status, int64_t* ticket);

/* Cancels a pending request: one that has not started completes at once
 * with GP_E_CANCELLED; one with chunks on the device launches no further
 * chunk and completes with GP_E_CANCELLED once they have finished (its
 * output arrays are not written).  GP_E_INVALID_ARG for a ticket that is
 * unknown, completed or already cancelled. */
int gp_server_cancel(gp_server* server, int64_t ticket);

/* Waits up to timeout_ms (< 0: no limit, 0: just look) for completed
 * requests and returns up to max_n of them (ticket and result code, GP_OK
 * or the error that failed the request), each once. */
int gp_server_poll(gp_server* server, double timeout_ms, int64_t* tickets, int32_t* results,
                   int32_t max_n, int32_t* n_done);

/* Waits up to timeout_ms for one ticket; *done = 1 and *result set once it
 * has completed (the ticket is then consumed).  GP_E_INVALID_ARG for a
 * ticket that is unknown or already consumed. */
int gp_server_wait(gp_server* server, int64_t ticket, double timeout_ms, int32_t* done,
                   int32_t* result);

int gp_server_get_stats(gp_server* server, gp_server_stats* out);
int gp_server_reset_stats(gp_server* server);

/* Completes every submitted request, then frees everything. */
void gp_server_destroy(gp_server* server);

/*
 * gp_workspace_size -- device bytes the library may hold for one stream
 * after a gp_eval / gp_eval_batched call of this shape (its cached
 * workspace, growth slack included).  Pure host arithmetic: no device
 * call.  For admission control by callers that budget device memory.
 * Returns GP_E_INVALID_ARG for sizes out of range.
 */
int gp_workspace_size(int64_t n_programs, int64_t n_nodes, int32_t n_requests,
                      int32_t n_datasets, int32_t max_n_vars, int64_t max_n_cases,
                      size_t* bytes);

/*
 * Phase timing (the paper's console reports GPU kernel time per generation,
 * Sec. "Understanding Beagle Output").  gp_timing_enable(1) makes later
 * gp_eval calls on the calling thread record HIP events on their stream
 * around each phase; gp_timing_read() synchronizes on the recorded events
 * and accumulates milliseconds per phase since the last reset:
 *   ms[0] prepare + depth-class partition, ms[1..3] evaluation of depth
 *   classes <= 8, <= 16, <= 32, ms[4] fp64 reduction, ms[5] whole call.
 * *n_calls gets the number of timed calls.  gp_timing_enable(0) stops
 * recording; gp_timing_reset() clears the sums.  Returns GP_OK or GP_E_HIP.
 */
#define GP_TIMING_PHASES 6
int gp_timing_enable(int on);
int gp_timing_reset(void);
int gp_timing_read(double* ms, int64_t* n_calls);

#ifdef __cplusplus
}
#endif
#endif /* GPEVAL_H */
