/*
 * gpeval.h -- C ABI of the MI355X (gfx950) batched fitness evaluator for
 * postfix symbolic-regression programs.
 *
 * What it computes ("Scoring" in the paper's Table 1; the GPU side of
 * Sec. "Dividing Tasks Between CPU and GPU"): every program of a population
 * is run over every fitness case, and one aggregate per program comes back:
 *
 *   F(p) = MSE(p) + tax_on_length * len(p)      for a valid program
 *   F(p) = +INFINITY  if some case output is NaN or +-inf, or MSE(p) > FLT_MAX
 *   MSE(p) = (1/n) * sum_i (f_p(x_i) - y_i)^2
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
 * in compensated fp32 (power-of-two pre-scaled so no partial sum can exceed
 * the MSE); the per-program cross-block sum, the tax and the classification
 * are fp64.  Program decoding and indexing are exact.
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

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GPEVAL_VERSION 1
#define GP_MAX_STACK 32           /* stack limit (StackSize in the GCL section) */
#define GP_MAX_CONSTS (1 << 24)   /* a node's arg field has 24 bits */
#define GP_MAX_VARS (1 << 24)

enum gp_status {
    GP_OK = 0,
    GP_E_INVALID_ARG = -1,   /* null pointer, negative size, ld_x < n_cases, ... */
    GP_E_BAD_PROGRAM = -2,   /* gp_validate found an invalid program */
    GP_E_TOO_LARGE = -3,     /* a size exceeds a documented limit */
    GP_E_NO_MEMORY = -4,     /* device workspace allocation failed */
    GP_E_HIP = -5            /* a HIP runtime call failed */
};

/* Opcodes (GCL command table; ABS is not a GCL command). */
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
    GP_N_OPS = 12
};
#define GP_ALL_OPS ((1u << GP_N_OPS) - 1u)

/* Per-program validation codes. */
enum gp_prog_status {
    GP_PROG_OK = 0, GP_PROG_EMPTY = 1, GP_PROG_BAD_OP = 2, GP_PROG_BAD_VAR = 3,
    GP_PROG_BAD_CONST = 4, GP_PROG_UNDERFLOW = 5, GP_PROG_TOO_DEEP = 6,
    GP_PROG_FINAL_DEPTH = 7, GP_PROG_BAD_OFFSETS = 8
};

/* Thread-local text for the last non-OK status returned on this thread. */
const char* gp_last_error(void);

/* Library version (GPEVAL_VERSION of the build). */
int gp_version(void);

/*
 * gp_validate -- host-side check of a population (host pointers).
 * allowed_op_mask: bit op set = op allowed (GetAllowedOperations in the
 * optional MLSetup overrides); 0 means GP_ALL_OPS.  status/max_depth:
 * optional host arrays of n_programs entries.  *first_bad (optional) gets
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
 * gp_predict -- per-case outputs f_p(x_i) of every program (the paper's
 * ExecuteGenome utility, Sec. "Useful Utilities": run a genome on input
 * data).  Same program and input arguments as gp_eval (device pointers);
 * out: float32, out[p * ld_out + i] for i < n_cases, ld_out >= n_cases,
 * caller-owned device memory of n_programs * ld_out floats.  Values are the
 * fp32 results of the same interpreter gp_eval runs (NaN and +-inf kept).
 * Programs that fail validation get a NaN row and a nonzero out_status.
 * Asynchronous on `stream`; shares gp_eval's per-stream workspace.
 */
int gp_predict(const uint32_t* nodes, const int64_t* offsets, int64_t n_programs,
               int64_t n_nodes, const float* consts, int64_t n_consts,
               const float* X, int32_t n_vars, int64_t ld_x, int64_t n_cases,
               uint32_t allowed_op_mask, float* out, int64_t ld_out, int32_t* out_status,
               hipStream_t stream);

/* Release every cached workspace of the calling process (all devices). */
void gp_release_workspaces(void);

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
