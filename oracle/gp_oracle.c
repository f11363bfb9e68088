/*
 * gp_oracle.c -- plain, slow, obviously correct CPU reference for the
 * batched fitness evaluation ("Scoring", paper Table 1) of postfix
 * symbolic-regression programs.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the HIP
 * library: the op numbering below is the interchange format of the program
 * arrays and is written out here independently.
 *
 * What is computed (the plain definition, no blocking, fusion or reordering):
 *
 *   F(p)       = +inf                     if invalid(p)
 *              = MSE(p) + tau * len(p)    otherwise
 *   MSE(p)     = (1/n) * sum over valid pairs i of (f_p(x_i) - y_i)^2
 *                                                        (fp64, plain loop)
 *   invalid(p) = for some case exactly one of f_p(x_i), y_i is NaN or
 *                +-inf, or MSE(p) > FLT_MAX
 *   f_p(x_i)   = postfix (RPN) evaluation of p on case i
 *   a valid pair is a case whose output and target are both finite; a case
 *   where both are NaN/inf is a matched invalid pair and adds nothing
 *
 * Sources in the paper:
 *   - RPN stack machine: unary ops replace the top element, binary ops replace
 *     the top two (Sec. "Genome Computer Language (GCL)").
 *   - Stack limit of 32 elements (same section, StackSize).
 *   - Op semantics and operand order: SUB is second-top minus top, DIV is
 *     second-top divided by top (GCL command table, Table 3).
 *   - Invalid values (NaN, Inf) in the model output or in the dataset are
 *     kept and handled per case, not removed (Sec. "Fitness Functions", the
 *     text around Eq. 1-2, whose Eq. 2 rewards matched invalid pairs and
 *     penalises mismatched ones); here a mismatched case (one side invalid)
 *     gives the program the worst fitness, +inf, and a matched one is an
 *     exact prediction.  With finite targets this is: any invalid case
 *     output gives +inf.
 *   - Length tax = "Tax on Length" / parsimony pressure (Table 1 and the
 *     ScriptLengthTaxRateInternal paragraph), charged per node.
 *   - Inputs and targets are fp32 (MLSetup data interface, float[] / float).
 *   - One aggregate per individual over all fitness cases (Sec. "Dividing
 *     Tasks Between CPU and GPU").
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   - DIV is protected: |b| <= theta gives 1, else a/b; theta = fp32(0.001).
 *     Written so that a NaN divisor still yields NaN.
 *   - LOG (the paper's LN) is protected: |a| <= theta gives 0, else ln|a|.
 *   - SQRT is protected: sqrt(|a|).
 *   - ABS is |a| (not a GCL command; part of the benchmark op set).
 *   - Every op result is passed through R(v): a finite fp64 value whose fp32
 *     rounding would overflow becomes +-inf, so the fp32 overflow range is
 *     emulated; NaN passes through; underflow is not emulated.
 *   - A valid program never underflows the stack, never exceeds depth 32 and
 *     ends with exactly one element.  len = number of nodes, leaves included.
 *
 * Modes:
 *   ORACLE_M64   fp64 values with the R(v) overflow emulation (the reference).
 *   ORACLE_M32E  as M64, but each op result is also rounded to fp32: the
 *                result of a correctly rounded fp32 evaluator.  Sums stay fp64.
 *   ORACLE_M32E_UP / ORACLE_M32E_DN
 *                M32E with every sin/cos/exp/log/sqrt result moved one fp32
 *                ulp up (down): used only to certify that a program is
 *                chaotic.
 *   ORACLE_M32E_RAND + s (s >= 0)
 *                M32E with every sin/cos/exp/log/sqrt result moved by a
 *                pseudo-random d in {-2,...,+2} fp32 ulps, d drawn from
 *                SplitMix64 (Steele, Lea, Flood 2014) keyed by (s, node,
 *                case): an fp32 evaluator whose elementary functions are
 *                within 2 ulps.  Also certification only.
 *
 * The rest of the GCL command table (the paper's Table of GCL commands):
 *   DUP, SWAP, DEL          stack moves;
 *   SQUARE a*a, SIGN -a, CUBE a*a*a, CBRT, TAN, ARCSIN, ARCCOS, ARCTAN,
 *   TANH                    C99 functions, unprotected (NaN outside the
 *                           domain, as the paper's fitness expects);
 *   SQRT_RAW                the paper's SQRT, C99 sqrt (NaN below zero);
 *                           SQRT above stays the protected sqrt(|a|);
 *   POW                     pow(second, top), C99 special cases;
 *   COPY @k, PASTE @k       variables: COPY stores the top without
 *                           touching the stack, PASTE pushes the stored
 *                           value and frees the variable.
 * Readings for the variables (listed in the design notes): k < 16; a valid
 * program copies a variable only while it is free and pastes it only while
 * it holds a value, and ends with every variable free; a live variable
 * occupies one of the 32 stack cells, so stack depth plus live variables
 * never exceeds 32.  The reported maximum depth is the maximum of that sum.
 *
 * Correlation fitness (oracle_correlation; the paper's default fitness,
 * Sec. "Fitness Functions", Eq. 1 and Eq. 2), written out plainly:
 *
 *   a case is a valid pair when f_p(x_i) and y_i are both finite;
 *   c1 = cases where exactly one of the two is invalid (either side),
 *   c2 = cases where both are invalid, n = N - c1 - c2 valid pairs;
 *   r  = sum (y - ybar)(f - fbar) / sqrt(sum (y - ybar)^2 sum (f - fbar)^2)
 *        over the valid pairs, with the means over the valid pairs (Eq. 1;
 *        two passes: means first, then the centred sums);
 *   r  = 0 when n < 2 or either centred sum of squares is 0;
 *   score = M (r^2)^2 (N - (c1 + c2)) - M (c1 - c2)            (Eq. 2)
 *
 * Higher is better.  Readings (listed in the design notes): c1 counts both
 * mismatch directions; r^4 is the square of the squared r; r = 0 for a
 * constant output or target; M is a parameter (the paper's maximum score).
 *
 * Point-to-point integer reward (oracle_reward; StdFitFunc of the section
 * on fitness functions, Eq. 5, and its Square/Cube/Hyper variants), per
 * case, then summed over the cases in int64 (higher is better):
 *
 *   valid pair (output and target finite), in fp32 (the reward function
 *   takes fp32 values; the output is rounded to fp32 first):
 *     M                                   if max(|o|, |y|) = 0
 *     rint(M * ratio^p - M/11)            if o and y have opposite signs
 *     rint(M * ratio^p)                   otherwise
 *     ratio = min(|o|,|y|) / max(|o|,|y|), ratio^p by repeated products
 *     (p = 1, 2 = r*r, 3 = r^2*r, 8 = ((r^2)^2)^2), rint = round half to
 *     even, M/11 the fp32 quotient;
 *   invalid pair: +M when both are invalid, -M when one is.
 */
#include <math.h>
#include <float.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include <unistd.h>

/* ---- program interchange format: node = op | (arg << 8) ---------------- */
enum {
    OP_LOAD = 0,   /* arg = input variable index (zero based)            */
    OP_CONST = 1,  /* arg = index into the constant pool                 */
    OP_ADD = 2, OP_SUB = 3, OP_MUL = 4, OP_DIV = 5,
    OP_SIN = 6, OP_COS = 7, OP_EXP = 8, OP_LOG = 9, OP_SQRT = 10, OP_ABS = 11,
    /* the rest of the GCL command table */
    OP_DUP = 12, OP_SWAP = 13, OP_DEL = 14, OP_SQUARE = 15, OP_SIGN = 16, OP_CUBE = 17,
    OP_CBRT = 18, OP_TAN = 19, OP_ASIN = 20, OP_ACOS = 21, OP_ATAN = 22, OP_TANH = 23,
    OP_SQRT_RAW = 24, OP_POW = 25, OP_COPY = 26, OP_PASTE = 27,
    OP_COUNT = 28
};

enum {
    ORACLE_M64 = 0, ORACLE_M32E = 1, ORACLE_M32E_UP = 2, ORACLE_M32E_DN = 3,
    ORACLE_M32E_RAND = 16
};

/* per-program validation status */
enum {
    ST_VALID = 0, ST_EMPTY = 1, ST_BAD_OP = 2, ST_BAD_VAR = 3, ST_BAD_CONST = 4,
    ST_UNDERFLOW = 5, ST_TOO_DEEP = 6, ST_FINAL_DEPTH = 7, ST_BAD_PAIR = 10
};

#define STACK_LIMIT 32
#define GCL_VARS 16             /* variable names @0 .. @15 */

/* theta = the fp32 number nearest to 0.001 (protected DIV and LOG). */
static double theta(void) { return (double)0.001f; }

/* Stack effect of one op: how many values it needs, and how the depth
 * changes.  Returns 0 for an unknown op. */
static int op_shape(uint32_t op, int* needs, int* delta)
{
    switch (op) {
    case OP_LOAD: case OP_CONST: *needs = 0; *delta = +1; return 1;
    case OP_ADD: case OP_SUB: case OP_MUL: case OP_DIV: case OP_POW:
        *needs = 2; *delta = -1; return 1;
    case OP_SIN: case OP_COS: case OP_EXP: case OP_LOG: case OP_SQRT:
    case OP_ABS: case OP_SQUARE: case OP_SIGN: case OP_CUBE: case OP_CBRT:
    case OP_TAN: case OP_ASIN: case OP_ACOS: case OP_ATAN: case OP_TANH:
    case OP_SQRT_RAW:
        *needs = 1; *delta = 0; return 1;
    case OP_DUP: *needs = 1; *delta = +1; return 1;
    case OP_SWAP: *needs = 2; *delta = 0; return 1;
    case OP_DEL: *needs = 1; *delta = -1; return 1;
    case OP_COPY: *needs = 1; *delta = 0; return 1;
    case OP_PASTE: *needs = 0; *delta = +1; return 1;
    default: return 0;
    }
}

/* Validate one program; writes its maximum stack depth. */
int oracle_check_program(const uint32_t* prog, int64_t len, int64_t n_consts,
                         int32_t n_vars, uint32_t allowed_mask,
                         int32_t* max_depth_out)
{
    int depth = 0, max_depth = 0, live = 0;
    int holds[GCL_VARS] = {0};  /* variable k holds a value */
    if (max_depth_out) *max_depth_out = 0;
    if (len <= 0) return ST_EMPTY;
    for (int64_t i = 0; i < len; ++i) {
        uint32_t op = prog[i] & 0xFFu;
        uint32_t arg = prog[i] >> 8;
        int needs, delta;
        if (!op_shape(op, &needs, &delta)) return ST_BAD_OP;
        if (!((allowed_mask >> op) & 1u)) return ST_BAD_OP;
        if (op == OP_LOAD && (int64_t)arg >= (int64_t)n_vars) return ST_BAD_VAR;
        if (op == OP_CONST && (int64_t)arg >= n_consts) return ST_BAD_CONST;
        if (depth < needs) return ST_UNDERFLOW;
        if (op == OP_COPY) {
            if (arg >= GCL_VARS || holds[arg]) return ST_BAD_PAIR;
            holds[arg] = 1;
            ++live;
        } else if (op == OP_PASTE) {
            if (arg >= GCL_VARS || !holds[arg]) return ST_BAD_PAIR;
            holds[arg] = 0;
            --live;
        }
        depth += delta;
        if (depth + live > STACK_LIMIT) return ST_TOO_DEEP;
        if (depth + live > max_depth) max_depth = depth + live;
    }
    if (max_depth_out) *max_depth_out = max_depth;
    if (depth != 1) return ST_FINAL_DEPTH;
    if (live != 0) return ST_BAD_PAIR;
    return ST_VALID;
}

void oracle_validate(const uint32_t* nodes, const int64_t* offsets,
                     int64_t n_programs, int64_t n_consts, int32_t n_vars,
                     uint32_t allowed_mask, int32_t* status, int32_t* max_depth)
{
    for (int64_t p = 0; p < n_programs; ++p) {
        int32_t md = 0;
        status[p] = oracle_check_program(nodes + offsets[p],
                                         offsets[p + 1] - offsets[p],
                                         n_consts, n_vars, allowed_mask, &md);
        if (max_depth) max_depth[p] = md;
    }
}

/* Smallest magnitude whose fp32 rounding (to nearest, ties to even) is
 * infinite: halfway between FLT_MAX = (2 - 2^-23) * 2^127 and 2^128. */
static double fp32_overflow_edge(void) { return ldexp(2.0 - ldexp(1.0, -24), 127); }

/* R(v): fp32 overflow-range emulation. */
static double clamp_range(double v)
{
    if (isfinite(v) && fabs(v) >= fp32_overflow_edge())
        return copysign(INFINITY, v);
    return v;
}

static double round_mode(double v, int mode)
{
    v = clamp_range(v);
    if (mode != ORACLE_M64 && isfinite(v)) v = (double)(float)v;
    return v;
}

/* SplitMix64 finalizer (Steele, Lea, Flood 2014). */
static uint64_t splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

/* Transcendental results in the perturbed certification modes; k = node
 * index, i = case index. */
static double nudge(double v, int mode, int64_t k, int64_t i)
{
    if (!isfinite(v)) return v;
    float f = (float)v;
    if (mode == ORACLE_M32E_UP) f = nextafterf(f, INFINITY);
    else if (mode == ORACLE_M32E_DN) f = nextafterf(f, -INFINITY);
    else if (mode >= ORACLE_M32E_RAND) {
        uint64_t h = splitmix64(splitmix64((uint64_t)(mode - ORACLE_M32E_RAND)) ^
                                splitmix64(((uint64_t)k << 40) ^ (uint64_t)i));
        int d = (int)(h % 5u) - 2;
        for (; d > 0; --d) f = nextafterf(f, INFINITY);
        for (; d < 0; ++d) f = nextafterf(f, -INFINITY);
    }
    return (double)f;
}

/* Evaluate one valid program on one case.  X is variable major:
 * X[v * ld_x + i].  Inputs and constants are fp32 read exactly as fp64. */
static double eval_case(const uint32_t* prog, int64_t len, const float* consts,
                        const float* X, int64_t ld_x, int64_t i, int mode)
{
    double st[STACK_LIMIT];
    double var[GCL_VARS];       /* COPY/PASTE variables */
    int sp = 0;                 /* number of values on the stack */
    const double th = theta();
    for (int64_t k = 0; k < len; ++k) {
        uint32_t op = prog[k] & 0xFFu;
        uint32_t arg = prog[k] >> 8;
        double a, b, v;
        switch (op) {
        case OP_LOAD: st[sp++] = (double)X[(int64_t)arg * ld_x + i]; break;
        case OP_CONST: st[sp++] = (double)consts[arg]; break;
        case OP_ADD: case OP_SUB: case OP_MUL: case OP_DIV:
            b = st[--sp];       /* top */
            a = st[--sp];       /* second from top */
            if (op == OP_ADD) v = a + b;
            else if (op == OP_SUB) v = a - b;
            else if (op == OP_MUL) v = a * b;
            else v = (fabs(b) <= th) ? 1.0 : a / b;
            st[sp++] = round_mode(v, mode);
            break;
        case OP_POW:            /* second raised to the top */
            b = st[--sp];
            a = st[--sp];
            v = round_mode(pow(a, b), mode);
            if (mode >= ORACLE_M32E_UP) v = nudge(v, mode, k, i);
            st[sp++] = v;
            break;
        case OP_CBRT: case OP_TAN: case OP_ASIN: case OP_ACOS: case OP_ATAN:
        case OP_TANH: case OP_SQRT_RAW:
            a = st[--sp];
            if (op == OP_CBRT) v = cbrt(a);
            else if (op == OP_TAN) v = tan(a);
            else if (op == OP_ASIN) v = asin(a);
            else if (op == OP_ACOS) v = acos(a);
            else if (op == OP_ATAN) v = atan(a);
            else if (op == OP_TANH) v = tanh(a);
            else v = sqrt(a);
            v = round_mode(v, mode);
            if (mode >= ORACLE_M32E_UP) v = nudge(v, mode, k, i);
            st[sp++] = v;
            break;
        case OP_SIGN: a = st[--sp]; st[sp++] = -a; break;
        case OP_CUBE: a = st[--sp]; st[sp++] = round_mode(a * a * a, mode); break;
        case OP_COPY: var[arg] = st[sp - 1]; break;
        case OP_PASTE: st[sp++] = var[arg]; break;
        case OP_SIN: case OP_COS: case OP_EXP: case OP_LOG:
            a = st[--sp];
            if (op == OP_SIN) v = sin(a);
            else if (op == OP_COS) v = cos(a);
            else if (op == OP_EXP) v = exp(a);
            else v = (fabs(a) <= th) ? 0.0 : log(fabs(a));
            v = round_mode(v, mode);
            if (mode >= ORACLE_M32E_UP) v = nudge(v, mode, k, i);
            st[sp++] = v;
            break;
        case OP_SQRT:
            a = st[--sp];
            v = round_mode(sqrt(fabs(a)), mode);
            if (mode >= ORACLE_M32E_UP) v = nudge(v, mode, k, i);
            st[sp++] = v;
            break;
        case OP_ABS: a = st[--sp]; st[sp++] = fabs(a); break;
        case OP_SQUARE: a = st[--sp]; st[sp++] = round_mode(a * a, mode); break;
        case OP_DUP: a = st[sp - 1]; st[sp++] = a; break;
        case OP_SWAP: a = st[sp - 1]; st[sp - 1] = st[sp - 2]; st[sp - 2] = a; break;
        case OP_DEL: --sp; break;
        default: return NAN;    /* unreachable for a validated program */
        }
    }
    return st[0];
}

/* Per-case outputs f_p(x_i) of one program (for tests).  Returns the
 * validation status; out is left untouched for an invalid program. */
int oracle_program_outputs(const uint32_t* prog, int64_t len,
                           const float* consts, int64_t n_consts,
                           const float* X, int32_t n_vars, int64_t ld_x,
                           int64_t n_cases, uint32_t allowed_mask, int mode,
                           double* out)
{
    int st = oracle_check_program(prog, len, n_consts, n_vars, allowed_mask, NULL);
    if (st != ST_VALID) return st;
    for (int64_t i = 0; i < n_cases; ++i)
        out[i] = eval_case(prog, len, consts, X, ld_x, i, mode);
    return ST_VALID;
}

/* Fitness of one program; also returns the fp64 MSE (NaN if invalid).
 * A case is a valid pair when the output and the target are both finite
 * (the invalid pairs of Eq. 2, Sec. "Fitness Functions"): a valid pair adds
 * its squared residual; a case where both are invalid is a matched pair
 * and adds nothing; a case where exactly one of them is invalid makes the
 * fitness the worst value, +inf.  The mean divides by all n cases. */
static double program_fitness(const uint32_t* prog, int64_t len,
                              const float* consts, const float* X, int64_t ld_x,
                              const float* y, int64_t n_cases, double tax,
                              int mode, double* mse_out)
{
    double sum = 0.0;
    int bad = 0;
    for (int64_t i = 0; i < n_cases; ++i) {
        double f = eval_case(prog, len, consts, X, ld_x, i, mode);
        int fv = isfinite(f) != 0, yv = isfinite(y[i]) != 0;
        if (fv != yv) bad = 1;
        if (fv && yv) {
            double r = f - (double)y[i];
            sum += r * r;
        }
    }
    if (bad) { *mse_out = NAN; return INFINITY; }
    double mse = sum / (double)n_cases;
    *mse_out = mse;
    if (mse > (double)FLT_MAX) return INFINITY;
    return mse + tax * (double)len;
}

/* Correlation score of one valid program (Eq. 1-2, see the header); f is
 * scratch for n_cases outputs; *r_out receives r. */
static double program_correlation(const uint32_t* prog, int64_t len,
                                  const float* consts, const float* X, int64_t ld_x,
                                  const float* y, int64_t n_cases, double max_score,
                                  int mode, double* f, double* r_out, int64_t* c12)
{
    int64_t c1 = 0, c2 = 0, nv = 0;
    double sum_f = 0.0, sum_y = 0.0;
    for (int64_t i = 0; i < n_cases; ++i) {
        f[i] = eval_case(prog, len, consts, X, ld_x, i, mode);
        const int fv = isfinite(f[i]) != 0, yv = isfinite((double)y[i]) != 0;
        if (fv && yv) {
            sum_f += f[i];
            sum_y += (double)y[i];
            ++nv;
        } else if (fv != yv) {
            ++c1;
        } else {
            ++c2;
        }
    }
    double r = 0.0;
    if (nv >= 2) {
        const double fbar = sum_f / (double)nv, ybar = sum_y / (double)nv;
        double sxy = 0.0, sxx = 0.0, syy = 0.0;
        for (int64_t i = 0; i < n_cases; ++i) {
            if (!isfinite(f[i]) || !isfinite((double)y[i])) continue;
            const double dx = f[i] - fbar, dy = (double)y[i] - ybar;
            sxy += dy * dx;
            sxx += dx * dx;
            syy += dy * dy;
        }
        if (sxx > 0.0 && syy > 0.0) r = sxy / sqrt(syy * sxx);
    }
    *r_out = r;
    if (c12) { c12[0] = c1; c12[1] = c2; }
    const double r2 = r * r;
    return max_score * r2 * r2 * (double)(n_cases - (c1 + c2)) - max_score * (double)(c1 - c2);
}

/* fp32 reward of one valid pair (see the header). */
static int64_t pair_reward(float o, float y, float M, int power)
{
    const float ao = fabsf(o), ay = fabsf(y);
    const float mx = ao > ay ? ao : ay, mn = ao > ay ? ay : ao;
    if (mx == 0.0f) return (int64_t)M;
    const float r = mn / mx;
    float rp = r;
    if (power == 2) rp = r * r;
    else if (power == 3) rp = (r * r) * r;
    else if (power == 8) { const float r2 = r * r, r4 = r2 * r2; rp = r4 * r4; }
    float v = M * rp;
    if ((o < 0.0f && y > 0.0f) || (o > 0.0f && y < 0.0f)) v = v - M / 11.0f;
    return (int64_t)rintf(v);
}

/* Reward of one case from the program's output f (rounded to fp32 here). */
static int64_t case_reward(double f, float y, float M, int power)
{
    const float o = (float)f;
    const int ov = isfinite(f) && isfinite(o), yv = isfinite(y) != 0;
    if (ov && yv) return pair_reward(o, y, M, power);
    return (ov || yv) ? -(int64_t)M : (int64_t)M;
}

/* Integer reward of one valid program (summed over the cases). */
static double program_reward(const uint32_t* prog, int64_t len, const float* consts,
                             const float* X, int64_t ld_x, const float* y, int64_t n_cases,
                             double max_score, int power, int mode)
{
    const float M = (float)max_score;
    int64_t total = 0;
    for (int64_t i = 0; i < n_cases; ++i)
        total += case_reward(eval_case(prog, len, consts, X, ld_x, i, mode), y[i], M, power);
    return (double)total;
}

typedef struct {
    const uint32_t* nodes; const int64_t* offsets;
    const float* consts; int64_t n_consts;
    const float* X; int32_t n_vars; int64_t ld_x;
    const float* y; int64_t n_cases; double tax;
    uint32_t allowed_mask; int mode;
    double* out; double* mse; int32_t* status;
    int64_t p0, p1;
    int correlation;            /* 1: Eq. 1-2; 2: the integer reward (Eq. 5) */
    double max_score;           /* M of Eq. 2 or Eq. 5 */
    int64_t* c12;               /* optional (c1, c2) per program */
    int power;                  /* reward power (1, 2, 3 or 8) */
} job_t;

static void* run_job(void* arg)
{
    job_t* j = (job_t*)arg;
    double* scratch = NULL;
    if (j->correlation == 1) {
        scratch = (double*)malloc(sizeof(double) * (size_t)(j->n_cases > 0 ? j->n_cases : 1));
        if (!scratch) {
            for (int64_t p = j->p0; p < j->p1; ++p) j->out[p] = NAN;
            return NULL;
        }
    }
    for (int64_t p = j->p0; p < j->p1; ++p) {
        const uint32_t* prog = j->nodes + j->offsets[p];
        int64_t len = j->offsets[p + 1] - j->offsets[p];
        int st = oracle_check_program(prog, len, j->n_consts, j->n_vars,
                                      j->allowed_mask, NULL);
        if (j->status) j->status[p] = st;
        double mse = NAN;
        if (st != ST_VALID) {
            j->out[p] = NAN;    /* not a scorable program */
        } else if (j->correlation == 2) {
            j->out[p] = program_reward(prog, len, j->consts, j->X, j->ld_x, j->y,
                                       j->n_cases, j->max_score, j->power, j->mode);
        } else if (j->correlation) {
            j->out[p] = program_correlation(prog, len, j->consts, j->X, j->ld_x, j->y,
                                            j->n_cases, j->max_score, j->mode, scratch,
                                            &mse, j->c12 ? j->c12 + 2 * p : NULL);
        } else {
            j->out[p] = program_fitness(prog, len, j->consts, j->X, j->ld_x,
                                        j->y, j->n_cases, j->tax, j->mode, &mse);
        }
        if (j->mse) j->mse[p] = mse;
    }
    free(scratch);
    return NULL;
}

/* Fitness of every program.  Structurally invalid programs get NaN and a
 * nonzero status.  n_threads <= 0 uses every online core.  Returns the
 * number of threads used. */
static int run_all(const uint32_t* nodes, const int64_t* offsets,
                   int64_t n_programs, const float* consts, int64_t n_consts,
                   const float* X, int32_t n_vars, int64_t ld_x,
                   const float* y, int64_t n_cases, double tax,
                   uint32_t allowed_mask, int mode, int n_threads,
                   double* out_fitness, double* out_mse, int32_t* status,
                   int correlation, double max_score, int64_t* c12, int power)
{
    if (n_threads <= 0) n_threads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    if ((int64_t)n_threads > n_programs) n_threads = n_programs > 0 ? (int)n_programs : 1;

    job_t jobs[256];
    pthread_t tids[256];
    /* contiguous program ranges balanced by node count */
    int64_t total = offsets[n_programs] - offsets[0];
    int64_t p = 0;
    for (int t = 0; t < n_threads; ++t) {
        int64_t target = offsets[0] + (total * (t + 1)) / n_threads;
        int64_t q = p;
        while (q < n_programs && (offsets[q + 1] <= target || q == p)) ++q;
        if (t == n_threads - 1) q = n_programs;
        job_t j = { nodes, offsets, consts, n_consts, X, n_vars, ld_x, y,
                    n_cases, tax, allowed_mask, mode, out_fitness, out_mse,
                    status, p, q, correlation, max_score, c12, power };
        jobs[t] = j;
        p = q;
    }
    for (int t = 0; t < n_threads; ++t)
        pthread_create(&tids[t], NULL, run_job, &jobs[t]);
    for (int t = 0; t < n_threads; ++t)
        pthread_join(tids[t], NULL);
    return n_threads;
}

int oracle_fitness(const uint32_t* nodes, const int64_t* offsets,
                   int64_t n_programs, const float* consts, int64_t n_consts,
                   const float* X, int32_t n_vars, int64_t ld_x,
                   const float* y, int64_t n_cases, double tax,
                   uint32_t allowed_mask, int mode, int n_threads,
                   double* out_fitness, double* out_mse, int32_t* status)
{
    return run_all(nodes, offsets, n_programs, consts, n_consts, X, n_vars, ld_x, y,
                   n_cases, tax, allowed_mask, mode, n_threads, out_fitness, out_mse,
                   status, 0, 0.0, NULL, 1);
}

/* Correlation score (Eq. 1-2) of every program; out_r (optional) receives
 * r, out_c12 (optional, 2 per program) the counts c1 and c2.  Structurally
 * invalid programs get NaN and a nonzero status. */
int oracle_correlation(const uint32_t* nodes, const int64_t* offsets,
                       int64_t n_programs, const float* consts, int64_t n_consts,
                       const float* X, int32_t n_vars, int64_t ld_x,
                       const float* y, int64_t n_cases, double max_score,
                       uint32_t allowed_mask, int mode, int n_threads,
                       double* out_score, double* out_r, int64_t* out_c12, int32_t* status)
{
    return run_all(nodes, offsets, n_programs, consts, n_consts, X, n_vars, ld_x, y,
                   n_cases, 0.0, allowed_mask, mode, n_threads, out_score, out_r,
                   status, 1, max_score, out_c12, 1);
}

/* Integer reward (Eq. 5 and its powers; see the header) of every program,
 * summed over the cases.  power is 1, 2, 3 or 8.  Structurally invalid
 * programs get NaN and a nonzero status. */
/* Per-case rewards of given outputs: out[i] = the reward of output o[i]
 * against target y[i] (the per-case rule above, o rounded to fp32). */
void oracle_case_rewards(const double* o, const float* y, int64_t n, double max_score,
                         int power, int64_t* out)
{
    const float M = (float)max_score;
    for (int64_t i = 0; i < n; ++i) out[i] = case_reward(o[i], y[i], M, power);
}

int oracle_reward(const uint32_t* nodes, const int64_t* offsets,
                  int64_t n_programs, const float* consts, int64_t n_consts,
                  const float* X, int32_t n_vars, int64_t ld_x,
                  const float* y, int64_t n_cases, double max_score, int power,
                  uint32_t allowed_mask, int mode, int n_threads,
                  double* out_reward, int32_t* status)
{
    return run_all(nodes, offsets, n_programs, consts, n_consts, X, n_vars, ld_x, y,
                   n_cases, 0.0, allowed_mask, mode, n_threads, out_reward, NULL,
                   status, 2, max_score, NULL, power);
}
