// gpeval.hip -- gfx950 kernels and C ABI of the batched fitness evaluator.
//
// Path of one scoring call (all on the caller's stream):
//   k_tables         one workgroup: check the dataset and request tables, lay
//                    the requests out back to back, derive tile shapes.
//   k_validate       one thread per program: validate (GCL stack and
//                    variable discipline, 32-cell limit, opcode/operand
//                    ranges, allowed ops), count staged instructions, depth
//                    class and partition key; per-block key counts and
//                    staged sizes.  With an op mask within the benchmark
//                    set the same walk stages the program in place (below).
//   k_class_scan     one workgroup: scans of both; class ranges (and for a
//                    single request its per-class work-item tables).
//   k_stage          one thread per program: stage each instruction as one
//                    8-byte word {flags | selector | cell, payload} in a
//                    range of its own (unless k_validate did), folding
//                    constant subtrees and a leaf into the operator after
//                    it (stack moves and variables become cell moves);
//                    stable scatter of program ids by (depth class, length
//                    band): each depth class (max depth <= 8, <= 16, <= 32)
//                    runs a kernel whose register stack is only as deep as
//                    needed, longest programs first.
//   k_seg_tables     several requests: per (class, request) program counts,
//                    positions and work-item prefixes.
//   k_eval<MAXD,K,FIT> persistent workgroups pull (program group, case tile)
//                    items from an atomic counter (tile-major, or group-major
//                    for the depth <= 8 class when the classes run one after
//                    another); the tile's inputs and
//                    targets are staged in LDS; each wavefront takes the
//                    group's programs one at a time and runs one over the
//                    64*K cases of the sub-tile (K per lane) with the value
//                    stack in VGPRs; the fitness epilogue is fused (MSE:
//                    scaled square with Kahan accumulation; correlation:
//                    shifted fp64 sums over valid pairs; integer reward:
//                    int64 per case) and a wave shuffle tree gives one
//                    partial per (program, tile).
//   k_reduce[_corr|_reward]  one thread per program: its tile partials in
//                    fixed order, then the score.
// gp_predict runs the same staging and k_predict<MAXD,K,EXT> (per-case
// outputs; EXT: the interpreter for the whole command table); gp_mc_rank
// runs k_rank_sample and k_rank_assign.
//
// Semantics follow the paper's GCL section (RPN stack machine, 32-element
// stack, command table operand order) and the protected-operator readings
// stated in gpeval.h.  One program per wavefront keeps the opcode stream
// wave-uniform (the paper's divergence argument, Sec. "Avoiding Thread
// Divergence", moved from a block to a wavefront).

#include "gpeval.h"

#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <array>
#include <map>
#include <vector>
#include <mutex>
#include <string>
#include <utility>

namespace {

// ------------------------------------------------------------------ errors
thread_local std::string g_last_error;

int set_error(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

}  // namespace

// Shared with the other translation units of the library (not exported).
__attribute__((visibility("hidden"))) void gp_internal_set_error(int code, const char* msg)
{
    (void)code;
    g_last_error = msg;
}

namespace {

#define GP_HIP_TRY(expr)                                                      \
    do {                                                                      \
        hipError_t e_ = (expr);                                               \
        if (e_ != hipSuccess)                                                 \
            return set_error(GP_E_HIP, "%s failed: %s", #expr,                \
                             hipGetErrorString(e_));                          \
    } while (0)

// ------------------------------------------------------------------ layout
constexpr int kWG = 256;                 // 4 wavefronts of 64
constexpr int kWaves = kWG / 64;
constexpr int kClasses = 3;              // max depth <= 8, <= 16, <= 32
constexpr int kLenBuckets = 8;           // staged length 1, 2-3, ..., 64-127, 128+
constexpr int kKeys = kClasses * kLenBuckets;
constexpr int kK1 = 4;                  // cases per lane of the depth <= 16 class
constexpr int kMaxTiles = 32;            // case tiles per program (cap)
constexpr int kBucketBlock = 128;        // programs per staging/partition block
constexpr int kStageNodes = 6656;        // LDS node cache of a staging block (26 KB, 52 per program)
// The short walk's cache (op masks within the benchmark set) holds an op
// byte and a payload per node (30 KB for 6144 nodes, 48 per program),
// which with the held constants keeps four staging blocks per CU.
constexpr int kStageNodesEmit = 6144;
constexpr uint32_t kOpByteBadConst = 0xFEu;   // its op byte of a constant out of range
// Fourth word of a raw buffer resource on gfx9 parts (32-bit data format).
constexpr int kBufferWord3 = 0x00020000;
// Constants held back for folding per program while staging: a longer run
// of constants is pushed (as runtime values) before the next one is held.
// 16 keeps the staging block at four per CU (with the node cache).
constexpr int kHeldConsts = 16;
constexpr int kMaxRequests = 4096;       // requests per batched call (tables are scanned by one workgroup)

// Per-program record written by the staging passes.
struct ProgMeta {
    int64_t start;      // first staged instruction
    int32_t len;        // node count (the length taxed)
    int32_t slen;       // staged instructions (0: not staged)
};
static_assert(sizeof(ProgMeta) == 16, "ProgMeta layout");

// Cases per lane for a depth class: deeper stacks hold fewer cases per
// lane so that the register stack (MAXD * K VGPRs) stays bounded.  (8 cases
// per lane for the shallow class measured slower on gfx950: occupancy drops
// from 5 to 3 waves per SIMD and LDS input reads are exposed.)  Depends only
// on the class and the dataset, never on the rest of the population.
__host__ __device__ inline int class_k(int c, int n_vars)
{
    if (c == 0) return 4;
    return c == 1 ? kK1 : 2;
}

// Tile geometry for one class.  A sub-tile is 64*K cases (one wavefront, K
// per lane).  The inputs and targets of `window` sub-tiles fit the LDS tile
// budget together ((n_vars + 1) rows of 64*K floats each), so a wavefront
// runs a program over a whole window without a barrier.  A tile is `passes`
// consecutive sub-tiles (a whole number of windows where the case count
// allows, at most 32 tiles per program); a work item covers one tile of G
// programs.  Depends only on (n_cases, K, n_vars) -- the dataset -- so a
// program's summation order never depends on the rest of the population or
// the batch.
constexpr int kTileLds = 24 * 1024;      // LDS bytes for input windows (6 workgroups per CU)
constexpr int kMaxWindow = 8;

struct TileShape {
    int32_t sub;        // cases per sub-tile (64 * K)
    int32_t passes;     // sub-tiles per tile
    int32_t n_tiles;    // tiles covering n_cases
    int32_t window;     // sub-tiles staged in LDS at once
};

__host__ __device__ inline int32_t tile_window(int k, int n_vars, int32_t lds_bytes)
{
    const int64_t block = (int64_t)(n_vars + 1) * 64 * k * 4;
    int64_t w = lds_bytes / block;
    return (int32_t)(w < 1 ? 1 : (w > kMaxWindow ? kMaxWindow : w));
}

__host__ __device__ inline TileShape tile_shape(int64_t n_cases, int k, int n_vars,
                                               int32_t lds_bytes, int32_t max_t)
{
    TileShape t;
    t.sub = 64 * k;
    const int64_t n_sub = (n_cases + t.sub - 1) / t.sub;
    t.window = tile_window(k, n_vars, lds_bytes);
    int64_t passes = (n_sub + max_t - 1) / max_t;
    if (passes < t.window) passes = t.window < n_sub ? t.window : n_sub;
    if (passes < 1) passes = 1;
    t.passes = (int32_t)passes;
    t.n_tiles = (int32_t)((n_sub + passes - 1) / passes);
    return t;
}

// Partial slots per program that any dataset of at most max_cases cases
// can need: n_tiles never exceeds kMaxTiles or the sub-tile count, and the
// sub-tile count grows with n_cases, so a smaller dataset can need more
// tiles than the largest one (33 sub-tiles make 17 tiles, 32 make 32).
__host__ __device__ inline int32_t max_tiles(int64_t max_cases, int k, int32_t max_t)
{
    const int64_t n_sub = (max_cases + 64 * k - 1) / (64 * k);
    return (int32_t)(n_sub < max_t ? (n_sub < 1 ? 1 : n_sub) : max_t);
}


// Power-of-two pre-scale s = 2^-e with 4^e >= n: every scaled partial sum
// of squared residuals is then <= MSE, so it overflows fp32 only when the
// MSE itself is beyond FLT_MAX.
__host__ __device__ inline int scale_exponent(int64_t n)
{
    int e = 0;
    while ((int64_t(1) << (2 * e)) < n) ++e;
    return e;
}

// ---------------------------------------------------- datasets, segments
// Dataset entry as the kernels use it (derived on the device each call).
struct DevDataset {
    const float* X;
    const float* y;
    int64_t ld_x;
    int64_t n_cases;
    double tax;
    double unscale;                 // 4^e / n_cases
    float scale;                    // 2^-e
    int32_t n_vars;
    int32_t passes[kClasses];
    int32_t n_tiles[kClasses];
    int32_t window[kClasses];
};

// Request entry as the kernels use it: the caller's entry with its
// program and node offsets inside the whole call (derived each call).
struct DevRequest {
    const uint32_t* nodes;
    const int64_t* offsets;
    const float* consts;
    int64_t n_programs;
    int64_t n_nodes;
    int64_t n_consts;
    int64_t node_base;              // first staged slot of this request
    double* out;
    int32_t* out_status;
    int32_t dataset;
};

// One workgroup: check the dataset and request tables, derive each
// dataset's tile shapes and scales, and lay the requests out one after the
// other (program starts seg_start[], staged-node bases).  With ds_in == NULL
// the single dataset `one` is used; with req_in == NULL the single request
// `one_req`.  *bad becomes 1 for inconsistent tables; then no program is
// staged and sizes are clamped so that every later index stays in range.
// bad[1] (k_validate's restage flag) is cleared.
__global__ __launch_bounds__(256) void k_tables(
    const gp_dataset* __restrict__ ds_in, int32_t n_ds, gp_dataset one,
    const gp_request* __restrict__ req_in, int32_t n_req, gp_request one_req,
    int64_t n_programs, int64_t n_nodes, int32_t max_vars, int64_t max_cases, int32_t need_out,
    int32_t tile_lds, int32_t tile_max, DevDataset* __restrict__ ds_out, DevRequest* __restrict__ req_out,
    int32_t* __restrict__ seg_ds, int64_t* __restrict__ seg_start, int32_t* __restrict__ bad)
{
    __shared__ int s_bad;
    __shared__ int64_t s_prog[256], s_node[256];
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    for (int d = threadIdx.x; d < n_ds; d += blockDim.x) {
        const gp_dataset in = ds_in ? ds_in[d] : one;
        DevDataset o;
        const bool ok = in.n_cases >= 1 && in.n_cases <= max_cases && in.n_vars >= 0 &&
                        in.n_vars <= max_vars && in.y != nullptr &&
                        (in.n_vars == 0 || (in.X != nullptr && in.ld_x >= in.n_cases)) &&
                        __builtin_isfinite(in.tax_on_length);
        if (!ok) atomicOr(&s_bad, 1);
        const int64_t n = ok ? in.n_cases : 1;
        const int e = scale_exponent(n);
        o.X = in.X;
        o.y = in.y;
        o.ld_x = in.ld_x;
        o.n_cases = n;
        o.tax = in.tax_on_length;
        o.unscale = ldexp(1.0, 2 * e) / (double)n;
        o.scale = ldexpf(1.0f, -e);
        o.n_vars = ok ? in.n_vars : 0;
        for (int c = 0; c < kClasses; ++c) {
            const TileShape t = tile_shape(n, class_k(c, o.n_vars), o.n_vars, tile_lds, tile_max);
            o.passes[c] = t.passes;
            o.n_tiles[c] = t.n_tiles;
            o.window[c] = t.window;
        }
        ds_out[d] = o;
    }
    // each thread takes a contiguous chunk of requests: check, clamp, sum
    const int chunk = (n_req + 255) / 256;
    const int r0 = min(n_req, (int)threadIdx.x * chunk), r1 = min(n_req, r0 + chunk);
    int64_t sp = 0, sn = 0;
    for (int r = r0; r < r1; ++r) {
        const gp_request q = req_in ? req_in[r] : one_req;
        const bool ok = q.n_programs >= 0 && q.n_programs <= n_programs && q.n_nodes >= 0 &&
                        q.n_nodes <= n_nodes && q.n_consts >= 0 && q.n_consts <= GP_MAX_CONSTS &&
                        (q.n_programs == 0 || q.offsets != nullptr) &&
                        (q.n_nodes == 0 || q.nodes != nullptr) &&
                        (q.n_consts == 0 || q.consts != nullptr) &&
                        (!need_out || q.n_programs == 0 || q.out_fitness != nullptr) &&
                        q.dataset >= 0 && q.dataset < n_ds;
        if (!ok) atomicOr(&s_bad, 1);
        sp += q.n_programs >= 0 && q.n_programs <= n_programs ? q.n_programs : 0;
        sn += q.n_nodes >= 0 && q.n_nodes <= n_nodes ? q.n_nodes : 0;
    }
    s_prog[threadIdx.x] = sp;
    s_node[threadIdx.x] = sn;
    __syncthreads();
    // inclusive Hillis-Steele scan of the chunk sums
    for (int off = 1; off < 256; off <<= 1) {
        const int64_t vp = threadIdx.x >= off ? s_prog[threadIdx.x - off] : 0;
        const int64_t vn = threadIdx.x >= off ? s_node[threadIdx.x - off] : 0;
        __syncthreads();
        s_prog[threadIdx.x] += vp;
        s_node[threadIdx.x] += vn;
        __syncthreads();
    }
    if (threadIdx.x == 0 && (s_prog[255] != n_programs || s_node[255] != n_nodes))
        atomicOr(&s_bad, 1);
    int64_t pp = s_prog[threadIdx.x] - sp, pn = s_node[threadIdx.x] - sn;
    for (int r = r0; r < r1; ++r) {
        const gp_request q = req_in ? req_in[r] : one_req;
        const int64_t np = q.n_programs >= 0 && q.n_programs <= n_programs ? q.n_programs : 0;
        const int64_t nn = q.n_nodes >= 0 && q.n_nodes <= n_nodes ? q.n_nodes : 0;
        DevRequest o;
        o.nodes = q.nodes;
        o.offsets = q.offsets;
        o.consts = q.consts;
        o.n_programs = np;
        o.n_nodes = nn;
        o.n_consts = q.n_consts;
        o.node_base = pn;
        o.out = q.out_fitness;
        o.out_status = q.out_status;
        o.dataset = q.dataset >= 0 && q.dataset < n_ds ? q.dataset : 0;
        req_out[r] = o;
        seg_ds[r] = o.dataset;
        // starts beyond the call's programs are clamped: such a table is bad
        seg_start[r] = pp < n_programs ? pp : n_programs;
        pp += np;
        pn += nn;
    }
    if (threadIdx.x == 0) seg_start[n_req] = n_programs;
    __syncthreads();
    if (threadIdx.x == 0) {
        bad[0] = s_bad;
        bad[1] = 0;                     // the restage flag, raised by k_validate
    }
}

// ------------------------------------------------------------------ sin/cos
// Constants from gen_sin_poly.py: minimax odd polynomial of degree 9 for sin
// on |r| <= pi/2 + 0.01 (relative error 6.8e-9 before fp32 evaluation) and
// a three-part fp32 split of pi for Cody-Waite reduction.  Measured against
// correctly rounded results: <= 1.75 ulp for |x| <= 2^17, including inputs
// next to multiples of pi; larger or non-finite inputs take the library
// path (which carries a Payne-Hanek reduction).
constexpr float kSinC0 = -1.666665971e-01f;
constexpr float kSinC1 = 8.333066478e-03f;
constexpr float kSinC2 = -1.980943489e-04f;
constexpr float kSinC3 = 2.605112741e-06f;
constexpr float kPiA = 3.141592741e+00f;
constexpr float kPiB = -8.742277657e-08f;
constexpr float kPiC = -3.430249020e-15f;
constexpr float kInvPi = 3.183098733e-01f;
constexpr float kTrigFastLimit = 131072.0f;
// 1.5 * 2^23: adding it to |v| < 2^22 rounds v to an integer n (the value's
// spacing there is 1) and leaves n's parity in the lowest significand bit.
constexpr float kRoundInt = 12582912.0f;

// sin(r) for |r| <= pi/2 (+ margin)
__device__ __forceinline__ float sin_poly(float r)
{
    const float u = r * r;
    float q = fmaf(u, kSinC3, kSinC2);
    q = fmaf(u, q, kSinC1);
    q = fmaf(u, q, kSinC0);
    return fmaf(u * r, q, r);
}

// r = x - kh * pi in three fused steps (exact first step for |x| <= 2^17)
__device__ __forceinline__ float reduce_pi(float x, float kh)
{
    float r = fmaf(-kh, kPiA, x);
    r = fmaf(-kh, kPiB, r);
    return fmaf(-kh, kPiC, r);
}

// Flips the sign of s when the integer held in the low bit of t's
// significand is odd (adding the bit at position 31 flips the sign bit).
__device__ __forceinline__ float flip_if_odd(float s, float t)
{
    return __uint_as_float(__float_as_uint(s) + (__float_as_uint(t) << 31));
}

// sin x = (-1)^k sin(x - k pi), k = the integer nearest x / pi
__device__ __forceinline__ float sin_fast(float x)
{
    const float t = fmaf(x, kInvPi, kRoundInt);
    const float k = t - kRoundInt;
    return flip_if_odd(sin_poly(reduce_pi(x, k)), t);
}

// cos x = (-1)^(k+1) sin(x - (k + 1/2) pi), k = the integer nearest
// x / pi - 1/2; t carries k + 1 (the offset is odd, so the parity is k+1's)
__device__ __forceinline__ float cos_fast(float x)
{
    const float t = fmaf(x, kInvPi, -0.5f) + (kRoundInt + 1.0f);
    const float k = t - (kRoundInt + 1.0f);
    return flip_if_odd(sin_poly(reduce_pi(x, k + 0.5f)), t);
}

// ---------------------------------------------------------------------- exp
// e^x = 2^(x log2 e): h = fp32(x log2 e), n = the integer nearest h, and
// 2^((h - n) + (x log2 e - h)) from the hardware exp2 on |f| <= 1/2 + tiny,
// scaled by 2^n; log2 e is split into an fp32 head and tail so the product
// keeps about 48 bits.  For |x| <= 87 no step overflows or underflows (the
// scaled result stays a normal number); other inputs take ROCm's expf.
constexpr float kLog2eHi = 1.442695022e+00f;   // fp32(log2 e), 0x3fb8aa3b
constexpr float kLog2eLo = 1.925963034e-08f;   // fp32(log2 e - kLog2eHi), 0x32a57060
constexpr float kExpFastLimit = 87.0f;

__device__ __forceinline__ float exp_fast(float x)
{
    const float h = x * kLog2eHi;
    const float n = rintf(h);
    const float f = (h - n) + fmaf(x, kLog2eLo, fmaf(x, kLog2eHi, -h));
    return ldexpf(__builtin_amdgcn_exp2f(f), (int)n);
}

// --------------------------------------------------------- sqrt|a|, ln|a|
// sqrt|a| with the hardware square root (faithful, <= 1 ulp); magnitudes
// below 2^-100 are scaled by 2^64 first (and the root by 2^-32 after), so
// no denormal reaches the instruction.
constexpr float kSqrtTiny = 0x1p-100f;
__device__ __forceinline__ float sqrt_abs(float a)
{
    const float x = fabsf(a);
    const bool tiny = x < kSqrtTiny;
    const float r = __builtin_amdgcn_sqrtf(tiny ? x * 0x1p64f : x);
    return tiny ? r * 0x1p-32f : r;
}

// Protected logarithm: 0 for |a| <= fp32(0.001), else ln|a| =
// log2|a| * ln 2 with ln 2 split into an fp32 head (rounded toward zero)
// and a positive fp32 tail, so log2|a| = +inf gives +inf + +inf = +inf.
// The hardware log2 only ever sees |a| > 0.001 (never a denormal); NaN
// propagates (the comparison with the threshold is false for NaN).
constexpr float kLn2Hi = 6.931471229e-01f;    // fp32 below ln 2
constexpr float kLn2Lo = 5.769998879e-08f;    // fp32(ln 2 - kLn2Hi) > 0
__device__ __forceinline__ float log_protected(float a)
{
    const float x = fabsf(a);
    const float l2 = __builtin_amdgcn_logf(x);
    const float ln = fmaf(l2, kLn2Hi, l2 * kLn2Lo);
    return x <= 0.001f ? 0.f : ln;
}

// ------------------------------------------------------ scalar op values
// Protected division (the divisor threshold is fp32(0.001)); shared by the
// interpreter and by constant folding, so both give the same bits.
__device__ __forceinline__ float div_protected(float a, float b)
{
    return fabsf(b) <= 0.001f ? 1.f : a / b;
}

// Per-case values of the elementary functions: the fast formula inside its
// range, the library function outside.  Constant folding uses the inline
// forms.  The interpreter calls the out-of-line forms, only when some case
// of a wavefront is outside a fast range (it takes the fast formulas
// directly otherwise): out of line, their per-case range tests are not
// merged into the interpreter's wavefront-wide tests (which would keep the
// per-case results live across the branch) and their library reductions
// do not raise the interpreter's register count.  Both forms run the same
// arithmetic, so they give the same bits.
__device__ __forceinline__ float sin_value_inl(float x)
{
    return fabsf(x) <= kTrigFastLimit ? sin_fast(x) : sinf(x);
}
__device__ __forceinline__ float cos_value_inl(float x)
{
    return fabsf(x) <= kTrigFastLimit ? cos_fast(x) : cosf(x);
}
__device__ __forceinline__ float exp_value_inl(float x)
{
    return fabsf(x) <= kExpFastLimit ? exp_fast(x) : expf(x);
}
__attribute__((noinline)) __device__ float sin_value(float x) { return sin_value_inl(x); }
__attribute__((noinline)) __device__ float cos_value(float x) { return cos_value_inl(x); }
__attribute__((noinline)) __device__ float exp_value(float x) { return exp_value_inl(x); }
__attribute__((noinline)) __device__ float sqrt_value(float x) { return sqrt_abs(x); }

// The rest of the command table: ROCm's fp32 library functions, out of
// line (the full-table interpreter calls them per case; constant folding
// calls the same functions, so both give the same bits).  CUBE is formed
// in fp64 (a*a is exact there) and rounded once; SQRT_RAW is the
// benchmark set's root with NaN below zero.
__attribute__((noinline)) __device__ float cbrt_value(float x) { return cbrtf(x); }
__attribute__((noinline)) __device__ float tan_value(float x) { return tanf(x); }
__attribute__((noinline)) __device__ float asin_value(float x) { return asinf(x); }
__attribute__((noinline)) __device__ float acos_value(float x) { return acosf(x); }
__attribute__((noinline)) __device__ float atan_value(float x) { return atanf(x); }
__attribute__((noinline)) __device__ float tanh_value(float x) { return tanhf(x); }
__attribute__((noinline)) __device__ float pow_value(float a, float b) { return powf(a, b); }
__device__ __forceinline__ float cube_value(float x)
{
    const double d = (double)x;
    return (float)(d * d * d);
}
__device__ __forceinline__ float sqrt_raw(float x)
{
    return x < 0.f ? __builtin_nanf("") : sqrt_abs(x);
}

// One operator of the benchmark set on one value, exactly as the
// interpreter computes it for a case (used to fold constant subtrees while
// staging; the commands beyond the set are not folded, so staging makes no
// calls).
__device__ __forceinline__ float binary_value(uint32_t op, float a, float b)
{
    switch (op) {
    case GP_ADD: return a + b;
    case GP_SUB: return a - b;
    case GP_MUL: return a * b;
    default: return div_protected(a, b);
    }
}

__device__ __forceinline__ float unary_value(uint32_t op, float x)
{
    switch (op) {
    case GP_SIN: return sin_value_inl(x);
    case GP_COS: return cos_value_inl(x);
    case GP_EXP: return exp_value_inl(x);
    case GP_LOG: return log_protected(x);
    case GP_SQRT: return sqrt_abs(x);
    default: return fabsf(x);
    }
}

// ------------------------------------------------------------- staging
// Request of program p: the last request whose first program is <= p.
__device__ __forceinline__ int request_of(const int64_t* __restrict__ seg_start, int32_t n_seg,
                                          int64_t p)
{
    int lo = 0, hi = n_seg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg_start[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// LDS-qualified pointers (per-lane LDS addressing without generic loads).
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) float lds_f32;
typedef __attribute__((address_space(3))) uint8_t lds_u8;

// Node readers for the staging passes: straight from the request's array,
// or from the block's LDS copy of its node range.
struct GlobalNodes {
    const uint32_t* __restrict__ p;
    __device__ uint32_t operator()(int64_t k) const { return p[k]; }
};
struct LdsNodes {
    const lds_u32* p;           // the block's node cache
    int64_t lo;                 // first cached node
    __device__ uint32_t operator()(int64_t k) const { return p[k - lo]; }
};
// Constant reader.
struct GlobalConsts {
    const float* __restrict__ p;
    __device__ float operator()(uint32_t j) const { return p[j]; }
};

// The node range [min s, max e) of the block's programs, when they all
// belong to one request and the range holds at most `cap` nodes.  `mine`:
// this thread has a program with a valid node range.  Every thread of the
// block must call it.  Returns true when the range is usable (then *req is
// the request, *lo the first node and *n the node count).
__device__ bool block_node_range(bool mine, int r, int64_t s, int64_t e, int cap, int* req,
                                 int64_t* lo, int* n)
{
    __shared__ long long s_lo, s_hi;
    __shared__ int s_r, s_mixed, s_any;
    if (threadIdx.x == 0) {
        s_lo = LLONG_MAX;
        s_hi = LLONG_MIN;
        s_r = -1;
        s_mixed = 0;
        s_any = 0;
    }
    __syncthreads();
    // reduced inside each wavefront first: one LDS atomic per wavefront
    // instead of one per thread
    long long wlo = mine ? (long long)s : LLONG_MAX, whi = mine ? (long long)e : LLONG_MIN;
    int wr = mine ? r : -1;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        wlo = min(wlo, __shfl_xor(wlo, off));
        whi = max(whi, __shfl_xor(whi, off));
        wr = max(wr, __shfl_xor(wr, off));
    }
    if ((threadIdx.x & 63) == 0 && wr >= 0) {
        atomicMin(&s_lo, wlo);
        atomicMax(&s_hi, whi);
        atomicMax(&s_r, wr);
        s_any = 1;
    }
    __syncthreads();
    if (mine && r != s_r) s_mixed = 1;
    __syncthreads();
    const bool use = s_any && !s_mixed && s_hi - s_lo <= cap;
    *req = s_r;
    *lo = s_lo;
    *n = use ? (int)(s_hi - s_lo) : 0;
    return use;
}

// Cooperative, coalesced copy of the block's node range into LDS (see
// block_node_range).  Every thread of the block must call it.  Returns true
// when the copy is used (then *lo is the first cached node).
__device__ bool cache_block_nodes(bool mine, int r, int64_t s, int64_t e,
                                  const DevRequest* __restrict__ reqs, lds_u32* cache,
                                  int64_t* lo)
{
    int rq = 0, n = 0;
    const bool use = block_node_range(mine, r, s, e, kStageNodes, &rq, lo, &n);
    if (use) {
        // 16 independent loads in flight per thread and round: a plain copy
        // loop would wait out the memory latency once per element
        constexpr int kU = 16;
        const uint32_t* __restrict__ src = reqs[rq].nodes + *lo;
        const int step = (int)blockDim.x * kU;
        for (int i0 = 0; i0 < n; i0 += step) {
            uint32_t v[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = i0 + u * (int)blockDim.x + (int)threadIdx.x;
                v[u] = i < n ? src[i] : 0u;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = i0 + u * (int)blockDim.x + (int)threadIdx.x;
                if (i < n) cache[i] = v[u];
            }
        }
    }
    __syncthreads();
    return use;
}

// The short walk's LDS copy of the block's node range: the op byte of
// each node (kOpByteBadConst for a constant whose index is out of range,
// 0xFF for any opcode from 32 on) and its payload: the constant's value
// bits for a constant in range, the argument otherwise.  The constants are
// gathered here, many loads in flight per thread, so the walk reads only
// LDS.  Every thread of the block must call it.
__device__ bool cache_block_stage(bool mine, int r, int64_t s, int64_t e,
                                  const DevRequest* __restrict__ reqs, lds_u8* ops,
                                  lds_u32* pay, int64_t* lo)
{
    int rq = 0, n = 0;
    const bool use = block_node_range(mine, r, s, e, kStageNodesEmit, &rq, lo, &n);
    if (use) {
        // one round: each thread has all its loads in flight at once (the
        // block's cache, 48 nodes per program), then all its constants'
        // gathers; raw buffer loads take a 32-bit lane offset plus the
        // round-invariant row offset as a scalar, so the loads in flight
        // cost one register each (loads past a range read 0)
        constexpr int kU = kStageNodesEmit / kBucketBlock;
        const int64_t nc = reqs[rq].n_consts;
        const __amdgpu_buffer_rsrc_t nr = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint32_t*>(reqs[rq].nodes + *lo), 0, n * 4, kBufferWord3);
        const __amdgpu_buffer_rsrc_t cr = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float*>(reqs[rq].consts), 0, (int)(nc * 4), kBufferWord3);
        const int t4 = (int)threadIdx.x * 4;
        uint32_t v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u)
            v[u] = __builtin_amdgcn_raw_buffer_load_b32(nr, t4, u * kBucketBlock * 4, 0);
        uint32_t c[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const uint32_t a = v[u] >> 8;
            c[u] = (v[u] & 0xFFu) == GP_CONST ? __builtin_amdgcn_raw_buffer_load_b32(cr, (int)(a * 4u), 0, 0)
                                              : 0u;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int i = u * kBucketBlock + (int)threadIdx.x;
            if (i < n) {
                const uint32_t op = v[u] & 0xFFu;
                const bool cst = op == GP_CONST;
                const bool bad = cst && (int64_t)(v[u] >> 8) >= nc;
                ops[i] = (uint8_t)(bad ? kOpByteBadConst : (op < 32u ? op : 0xFFu));
                pay[i] = cst ? (bad ? 0u : c[u]) : v[u] >> 8;
            }
        }
    }
    __syncthreads();
    return use;
}

#define GP_STAGING_FN __device__
#include "staging.h"
static_assert(kOpByteBadConst == kOpBadConst, "the LDS copy stores the walk's opcodes as they are");

// Readers of the benchmark-set walk (stage_check_base): op (kOpBadConst
// for a constant out of range), payload word, constant value, from the
// block's LDS copy (the payload holds the constant's value) or straight
// from the request's arrays (the payload is the constant's index).
struct LdsStageReader {
    const lds_u8* o;
    const lds_u32* p;
    int64_t lo;
    __device__ uint32_t op(int64_t k) const { return o[k - lo]; }
    __device__ uint32_t pay(int64_t k) const { return p[k - lo]; }
    __device__ float cval(int64_t, uint32_t pay) const { return __uint_as_float(pay); }
};
struct GlobalStageReader {
    const uint32_t* __restrict__ n;
    const float* __restrict__ c;
    int64_t n_consts;
    __device__ uint32_t op(int64_t k) const
    {
        const uint32_t w = n[k], op = (w & 0xFFu) < 32u ? (w & 0xFFu) : 0xFFu;
        return op == GP_CONST && (int64_t)(w >> 8) >= n_consts ? kOpBadConst : op;
    }
    __device__ uint32_t pay(int64_t k) const { return n[k] >> 8; }
    __device__ float cval(int64_t, uint32_t pay) const { return c[pay]; }
};

// LDS words of a staging block's node copy: the general walk's node
// words, or the short walk's payloads followed by its op bytes.
constexpr int kCacheWords = kStageNodes > kStageNodesEmit + kStageNodesEmit / 4
                                ? kStageNodes : kStageNodesEmit + kStageNodesEmit / 4;

// Pass 1, one thread per program (blocks of kBucketBlock): validate, count
// staged instructions, derive the depth class and the partition key, and
// accumulate per-block key counts and staged sizes for the scans that
// follow.  The block's nodes are read from an LDS copy when they fit.
// With an op mask within the benchmark set the same walk also stages the
// program, at its own node offset in the request's part of `code` (staged
// words never outnumber nodes, so the programs' ranges hold them, disjoint
// while the offsets never decrease); a program whose offsets do decrease
// sets *restage, and k_stage then stages every program again, packed.
__global__ __launch_bounds__(kBucketBlock) void k_validate(
    int64_t n_programs, uint32_t allowed, const DevDataset* __restrict__ ds,
    const DevRequest* __restrict__ reqs, const int64_t* __restrict__ seg_start, int32_t n_seg,
    const int32_t* __restrict__ tables_bad, int32_t lpt, int32_t n_blk,
    ProgMeta* __restrict__ meta, uint8_t* __restrict__ cls, int32_t* __restrict__ pds,
    int32_t* __restrict__ blk_counts, int64_t* __restrict__ blk_slen, uint2* __restrict__ code,
    int32_t* __restrict__ restage)
{
    __shared__ int cnt[kKeys];
    __shared__ unsigned long long s_slen;
    __shared__ uint32_t cache_mem[kCacheWords];
    __shared__ float pv_mem[kHeldConsts * kBucketBlock];
    lds_u32* cache = (lds_u32*)cache_mem;
    // a mask within the benchmark set: the short walk, which also stages
    const bool base = (allowed & ~GP_BASE_OPS) == 0u;
    lds_u8* ops = (lds_u8*)(cache + kStageNodesEmit);
    if (threadIdx.x < kKeys) cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) s_slen = 0ull;
    const int64_t p = (int64_t)blockIdx.x * kBucketBlock + threadIdx.x;
    const bool have = p < n_programs;
    const bool tab_ok = *tables_bad == 0;
    int r = 0;
    int64_t q = 0, s = 0, e = 0;
    DevRequest R{};
    if (have) {
        r = request_of(seg_start, n_seg, p);
        R = reqs[r];
        q = p - seg_start[r];                 // index inside the request
        pds[p] = r;
        if (tab_ok) {
            s = R.offsets[q];
            e = R.offsets[q + 1];
            if (e < s) *restage = 1;
        }
    }
    const bool range_ok = s >= 0 && e >= s && e <= R.n_nodes && e - s <= INT32_MAX - 1;
    const bool mine = have && tab_ok && range_ok && e > s;
    int64_t lo = 0;
    const bool cached = base ? cache_block_stage(mine, r, s, e, reqs, ops, cache, &lo)
                             : cache_block_nodes(mine, r, s, e, reqs, cache, &lo);
    long long slen = 0;                       // this program's staged size
    int pkey = 0xFF;                          // and its partition key
    if (have) {
        int status = GP_PROG_OK;
        int maxd = 0;
        int64_t n_staged = 0;
        if (!tab_ok) {
            status = GP_PROG_BAD_TABLE;
        } else if (!range_ok) {
            status = GP_PROG_BAD_OFFSETS;
        } else if (e == s) {
            status = GP_PROG_EMPTY;
        } else {
            const int32_t n_vars = ds[R.dataset].n_vars;
            uint2* dst = code + R.node_base + s;
            lds_f32* pvs = (lds_f32*)pv_mem + threadIdx.x;
            if (base && cached)
                n_staged = stage_check_base(LdsStageReader{ops, cache, lo}, s, e, allowed, n_vars,
                                            dst, pvs, status, maxd);
            else if (base)
                n_staged = stage_check_base(GlobalStageReader{R.nodes, R.consts, R.n_consts}, s, e,
                                            allowed, n_vars, dst, pvs, status, maxd);
            else if (cached)
                check_program(LdsNodes{cache, lo}, s, e, allowed, n_vars, R.n_consts, status, maxd,
                              n_staged);
            else
                check_program(GlobalNodes{R.nodes}, s, e, allowed, n_vars, R.n_consts, status,
                              maxd, n_staged);
        }
        const int c = status == GP_PROG_OK ? depth_class(maxd) : -1;
        ProgMeta m;
        m.start = R.node_base + s;            // where the short walk staged it
        m.len = (int32_t)(status == GP_PROG_BAD_OFFSETS || status == GP_PROG_BAD_TABLE ? 0 : e - s);
        m.slen = c >= 0 ? (int32_t)n_staged : 0;
        meta[p] = m;
        // partition key: depth class, then (single-request calls) length
        // band from longest to shortest; with several requests the order
        // inside a class stays the input order, so each request's programs
        // stay together
        int lb = 31 - __clz((uint32_t)(m.slen > 0 ? m.slen : 1));
        lb = lb < kLenBuckets - 1 ? lb : kLenBuckets - 1;
        const int key = c >= 0 ? c * kLenBuckets + (lpt ? kLenBuckets - 1 - lb : 0) : 0xFF;
        cls[p] = (uint8_t)key;
        pkey = key;
        slen = m.slen;
        if (R.out_status && q < R.n_programs) R.out_status[q] = status;
    }
    // per-key counts: one LDS atomic per distinct key in the wavefront
    const int lane = threadIdx.x & 63;
    for (uint64_t todo = __ballot(pkey < kKeys); todo != 0ull;) {
        const int first = __ffsll((unsigned long long)todo) - 1;
        const int k0 = __shfl(pkey, first);
        const uint64_t same = __ballot(pkey == k0);
        if (lane == first) atomicAdd(&cnt[k0], (int)__popcll(same));
        todo &= ~same;
    }
    // the block's staged size, summed in each wavefront first
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) slen += __shfl_xor(slen, off);
    if (lane == 0 && slen) atomicAdd(&s_slen, (unsigned long long)slen);
    __syncthreads();
    if (threadIdx.x < kKeys) blk_counts[threadIdx.x * n_blk + blockIdx.x] = cnt[threadIdx.x];
    if (threadIdx.x == 0) blk_slen[blockIdx.x] = (int64_t)s_slen;
}

// Programs per work item of a class with prog_tiles (program, case tile)
// pairs: see class_seg_tables.
__device__ __forceinline__ int class_group(double prog_tiles, int32_t g_max, int32_t target_items)
{
    int G = g_max;
    while (G > 4 && prog_tiles / G < (double)target_items) G >>= 1;
    return G < 1 ? 1 : G;
}

// Per depth class c, from its programs per segment (seg_cnt[c * n_seg +
// s]): the group size (programs per work item) and, per segment, where its
// programs start inside the class's range of `order` and the prefix of work
// items (groups times the segment dataset's case tiles).  Groups are as
// large as g_max allows while the class still has about target_items items
// (a small class gets smaller groups, so its few programs still spread over
// the GPU); never below 4, one program per wavefront of a workgroup.
// Grouping never changes a result.
__device__ void class_seg_tables(int c, int32_t n_seg, const int32_t* __restrict__ seg_cnt,
                                 const int32_t* __restrict__ seg_ds,
                                 const DevDataset* __restrict__ ds, int32_t g_max,
                                 int32_t target_items, int32_t* __restrict__ seg_pos,
                                 uint32_t* __restrict__ item_pre, int32_t* __restrict__ class_g)
{
    double prog_tiles = 0.0;
    for (int s = 0; s < n_seg; ++s)
        prog_tiles += (double)seg_cnt[c * n_seg + s] * (double)ds[seg_ds[s]].n_tiles[c];
    const int G = class_group(prog_tiles, g_max, target_items);
    class_g[c] = G;
    int32_t pos = 0;
    uint32_t items = 0;
    for (int s = 0; s < n_seg; ++s) {
        const int32_t n = seg_cnt[c * n_seg + s];
        seg_pos[c * n_seg + s] = pos;
        item_pre[c * (n_seg + 1) + s] = items;
        pos += n;
        items += (uint32_t)((n + G - 1) / G) * (uint32_t)ds[seg_ds[s]].n_tiles[c];
    }
    item_pre[c * (n_seg + 1) + n_seg] = items;
}

// Where a call of a single request gets its per-class work-item tables
// (k_class_scan writes them when `single` is set).
struct SegOut {
    int32_t single;
    int32_t g_max, target_items;
    const int32_t* seg_ds;
    const DevDataset* ds;
    int32_t* seg_cnt;
    int32_t* seg_pos;
    uint32_t* item_pre;
    int32_t* class_g;
};

// One workgroup: exclusive scans of the per-block key counts (key-major
// order) into blk_base and of the per-block staged sizes into blk_code;
// class_info[2c] = first position of depth class c, [2c+1] = its size (its
// keys are contiguous); also clears the per-class work counters.  Staged
// code never exceeds the call's node count unless programs' node ranges
// overlap; then *overflow is set, nothing is staged and every class is
// left empty.  With a single request it also writes the request's
// per-class tables (class_seg_tables).
__global__ __launch_bounds__(1024) void k_class_scan(
    const int32_t* __restrict__ blk_counts, const int64_t* __restrict__ blk_slen, int32_t n_blk,
    int64_t code_capacity, int32_t* __restrict__ blk_base, int64_t* __restrict__ blk_code,
    int32_t* __restrict__ class_info, uint32_t* __restrict__ work_counters,
    int32_t* __restrict__ overflow, SegOut so)
{
    __shared__ int part[1024];
    __shared__ long long lpart[1024];
    const int t = threadIdx.x;
    // a single request's dataset tiles, loaded while the scan runs
    const int32_t tiles = so.single && t < kClasses ? so.ds[so.seg_ds[0]].n_tiles[t] : 0;
    const int total = kKeys * n_blk;
    const int chunk = (total + 1023) / 1024;
    const int lo = t * chunk, hi = min(total, lo + chunk);
    // loads in batches of 8, so that a thread's loads are in flight together
    int sum = 0;
    {
        int i = lo;
        for (; i + 8 <= hi; i += 8) {
            int v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = blk_counts[i + u];
#pragma unroll
            for (int u = 0; u < 8; ++u) sum += v[u];
        }
        for (; i < hi; ++i) sum += blk_counts[i];
    }
    part[t] = sum;
    const int chunk2 = (n_blk + 1023) / 1024;
    const int lo2 = t * chunk2, hi2 = min(n_blk, lo2 + chunk2);
    long long sum2 = 0;
    for (int i = lo2; i < hi2; ++i) sum2 += blk_slen[i];
    lpart[t] = sum2;
    __syncthreads();
    // inclusive Hillis-Steele scans of the chunk sums
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = t >= off ? part[t - off] : 0;
        const long long v2 = t >= off ? lpart[t - off] : 0;
        __syncthreads();
        part[t] += v;
        lpart[t] += v2;
        __syncthreads();
    }
    int run = part[t] - sum;
    {
        int i = lo;
        for (; i + 8 <= hi; i += 8) {
            int v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = blk_counts[i + u];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                blk_base[i + u] = run;
                run += v[u];
            }
        }
        for (; i < hi; ++i) {
            blk_base[i] = run;
            run += blk_counts[i];
        }
    }
    long long run2 = lpart[t] - sum2;
    for (int i = lo2; i < hi2; ++i) {
        blk_code[i] = run2;
        run2 += blk_slen[i];
    }
    if (t < kClasses) {
        // exclusive prefix of entry i from the scanned chunk sums (LDS)
        // and the entries before it in its chunk, loaded all at once
        auto prefix = [&](int i) {
            if (i >= total) return part[1023];
            const int owner = i / chunk;
            int b = owner > 0 ? part[owner - 1] : 0;
            const int j0 = owner * chunk;
            if (chunk <= 32) {
                int v[32];
#pragma unroll
                for (int u = 0; u < 32; ++u) v[u] = j0 + u < i ? blk_counts[j0 + u] : 0;
#pragma unroll
                for (int u = 0; u < 32; ++u) b += v[u];
            } else {
                for (int j = j0; j < i; ++j) b += blk_counts[j];
            }
            return b;
        };
        const bool ovf = lpart[1023] > code_capacity;
        const int start = prefix(t * kLenBuckets * n_blk);
        const int end = prefix((t + 1) * kLenBuckets * n_blk);
        class_info[2 * t] = start;
        class_info[2 * t + 1] = ovf ? 0 : end - start;
        work_counters[t] = 0u;
        if (t == 0) *overflow = ovf ? 1 : 0;
        if (so.single) {
            // one request holds the whole class (class_seg_tables with one
            // segment)
            const int32_t n = ovf ? 0 : end - start;
            const int G = class_group((double)n * (double)tiles, so.g_max, so.target_items);
            so.seg_cnt[t] = n;
            so.class_g[t] = G;
            so.seg_pos[t] = 0;
            so.item_pre[2 * t] = 0u;
            so.item_pre[2 * t + 1] = (uint32_t)((n + G - 1) / G) * (uint32_t)tiles;
        }
    }
}

// Pass 2, same blocks as pass 1: each program's id is scattered (stably)
// into the partition order.  Programs the short walk of pass 1 staged in
// place stay there.  Otherwise (the whole command table, or node offsets
// that decrease somewhere, so that programs' node ranges may overlap) each
// program is staged here, at its block's base plus the exclusive scan of
// staged sizes inside the block, so ranges never overlap whatever the
// offsets.
//
// Staged instruction (8 bytes, one scalar load):
//   x = flags | sel << 8 | cell << 16, y = payload
//   kFPush  save the top into stack cell `cell`, then the top = leaf
//   kFUn    the top = unary sel (SIN..ABS as 0..5) of the top
//   kFSBin  the top = stack cell `cell`  OP_sel  top  (ADD..DIV as 0..3)
//   kFLBin  the top = top  OP_sel  leaf
//   kFLast  (with any of the above) the program's last instruction
// A leaf is the constant with bits y when kFConst is set, else the input
// row at LDS byte offset y (variable index * 1024, halved at two cases per
// lane).  Eight bytes (not sixteen) keep the code of the programs that the
// resident wavefronts run at once small enough to stay in the scalar cache
// while each program passes over its window.
__global__ __launch_bounds__(kBucketBlock) void k_stage(
    int64_t n_programs, const DevDataset* __restrict__ ds, const DevRequest* __restrict__ reqs,
    const int64_t* __restrict__ seg_start, const int32_t* __restrict__ pds, int32_t n_blk,
    const int64_t* __restrict__ blk_code, const int32_t* __restrict__ blk_base,
    const int32_t* __restrict__ overflow, const int32_t* __restrict__ restage, uint32_t allowed,
    uint8_t* __restrict__ cls, ProgMeta* __restrict__ meta, uint2* __restrict__ code,
    int32_t* __restrict__ order)
{
    __shared__ long long sc[kBucketBlock];
    constexpr int kW = kBucketBlock / 64;
    __shared__ int wcnt[kW][kKeys];
    const int t = threadIdx.x;
    const int64_t p = (int64_t)blockIdx.x * kBucketBlock + t;
    int key = p < n_programs ? (int)cls[p] : 0xFF;
    if (*overflow) {
        // overlapping node ranges: no program of this call is staged
        if (key < kKeys) {
            cls[p] = 0xFF;
            const int r = pds[p];
            const DevRequest& R = reqs[r];
            const int64_t q = p - seg_start[r];
            if (R.out_status && q < R.n_programs) R.out_status[q] = GP_PROG_BAD_OFFSETS;
        }
        return;
    }
    const bool base = (allowed & ~GP_BASE_OPS) == 0u;
    if (!base || *restage) {
        __shared__ uint32_t cache_mem[kCacheWords];
        __shared__ float pv_mem[kHeldConsts * kBucketBlock];
        lds_u32* cache = (lds_u32*)cache_mem;
        lds_u8* ops = (lds_u8*)(cache + kStageNodesEmit);
        ProgMeta m;
        m.start = 0;
        m.len = 0;
        m.slen = 0;
        if (p < n_programs) m = meta[p];
        // inclusive scan of staged sizes inside the block
        sc[t] = m.slen;
        __syncthreads();
        for (int off = 1; off < kBucketBlock; off <<= 1) {
            const long long v = t >= off ? sc[t - off] : 0;
            __syncthreads();
            sc[t] += v;
            __syncthreads();
        }
        const int64_t start = blk_code[blockIdx.x] + sc[t] - m.slen;
        int r = 0;
        int64_t s = 0, e = 0;
        DevRequest R{};
        if (key < kKeys) {
            r = pds[p];
            R = reqs[r];
            const int64_t q = p - seg_start[r];
            s = R.offsets[q];
            e = R.offsets[q + 1];
        }
        int64_t lo = 0;
        const bool cached = base ? cache_block_stage(key < kKeys, r, s, e, reqs, ops, cache, &lo)
                                 : cache_block_nodes(key < kKeys, r, s, e, reqs, cache, &lo);
        if (key < kKeys) {
            lds_f32* pvs = (lds_f32*)pv_mem + t;
            const int32_t n_vars = ds[R.dataset].n_vars;
            int st = 0, md = 0;
            if (base && cached)
                stage_check_base(LdsStageReader{ops, cache, lo}, s, e, allowed, n_vars,
                                 code + start, pvs, st, md);
            else if (base)
                stage_check_base(GlobalStageReader{R.nodes, R.consts, R.n_consts}, s, e, allowed,
                                 n_vars, code + start, pvs, st, md);
            else if (cached)
                stage_walk(LdsNodes{cache, lo}, s, e, GlobalConsts{R.consts}, code + start, m.slen,
                           pvs);
            else
                stage_walk(GlobalNodes{R.nodes}, s, e, GlobalConsts{R.consts}, code + start,
                           m.slen, pvs);
            meta[p].start = start;
        }
    }
    // stable scatter into the partition order
    const int wave = t >> 6, lane = t & 63;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int rank = 0;
    if (lane < kKeys) wcnt[wave][lane] = 0;
    // one pass per distinct key in the wavefront
    for (uint64_t todo = __ballot(key < kKeys); todo != 0ull;) {
        const int first = __ffsll((unsigned long long)todo) - 1;
        const int k0 = __shfl(key, first);
        const uint64_t bm = __ballot(key == k0);
        if (lane == first) wcnt[wave][k0] = __popcll(bm);
        if (key == k0) rank = __popcll(bm & below);
        todo &= ~bm;
    }
    __syncthreads();
    if (key < kKeys) {
        for (int w2 = 0; w2 < wave; ++w2) rank += wcnt[w2][key];
        order[blk_base[key * n_blk + blockIdx.x] + rank] = (int32_t)p;
    }
}

// One workgroup, calls of several requests: the programs of each depth
// class inside each segment (seg_cnt[c * n_seg + s]; the partition keeps
// each class in program order, so they are the class's entries between two
// lower bounds of the segment's program range), then class_seg_tables per
// class.  (A single request's tables come from k_class_scan.)
__global__ __launch_bounds__(256) void k_seg_tables(
    const int32_t* __restrict__ order, const int32_t* __restrict__ class_info,
    const int64_t* __restrict__ seg_start, int32_t n_seg, const int32_t* __restrict__ tables_bad,
    const int32_t* __restrict__ seg_ds, const DevDataset* __restrict__ ds, int32_t g_max,
    int32_t target_items, int32_t* __restrict__ seg_cnt, int32_t* __restrict__ seg_pos,
    uint32_t* __restrict__ item_pre, int32_t* __restrict__ class_g)
{
    const bool bad = *tables_bad != 0;              // then no program was staged
    for (int i = threadIdx.x; i < kClasses * n_seg; i += blockDim.x) {
        const int c = i / n_seg, sg = i - c * n_seg;
        const int32_t* __restrict__ ord = order + class_info[2 * c];
        const int n = class_info[2 * c + 1];
        // first position whose program id is >= v
        auto lower = [&](int64_t v) {
            int lo = 0, hi = n;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if ((int64_t)ord[mid] < v) lo = mid + 1; else hi = mid;
            }
            return lo;
        };
        seg_cnt[i] = bad ? 0 : lower(seg_start[sg + 1]) - lower(seg_start[sg]);
    }
    __syncthreads();
    if (threadIdx.x < kClasses)
        class_seg_tables(threadIdx.x, n_seg, seg_cnt, seg_ds, ds, g_max, target_items, seg_pos,
                         item_pre, class_g);
}

// ------------------------------------------------------------ evaluation
// Scalars of one class launch (pointers travel as restrict-qualified kernel
// parameters so that uniform loads of programs and metadata become scalar
// memory loads).
struct EvalConst {
    int32_t cls;
    int32_t G;              // programs per work item
    int32_t part_stride;    // partial of (program p, tile t) at t * part_stride + p
    int32_t max_vars;       // largest n_vars of the call
    int32_t n_seg;
    int32_t tile_floats;    // LDS floats for input windows
    int32_t group_major;    // depth <= 8 class: a group's case tiles are consecutive items
    // single-dataset form (gp_predict)
    int64_t ld_x;
    int64_t n_cases;
    int32_t n_vars;
    // integer reward mode
    int32_t reward_power;
    float reward_M;
};

// Error-free sum: s + e == a + b exactly (Knuth's TwoSum).
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e)
{
    s = a + b;
    const float bp = s - a;
    e = (a - (s - bp)) + (b - bp);
}

// Compensated pair (hi, lo) += (h2, l2).
__device__ __forceinline__ void acc_pair(float& hi, float& lo, float h2, float l2)
{
    float s, e;
    two_sum(hi, h2, s, e);
    hi = s;
    lo = (lo + l2) + e;
}

// One case of the MSE fitness into a lane's Kahan pair (the represented sum
// is hi + lo).  ys is the target pre-scaled by the dataset's power of two s,
// so fma(f, s, -ys) is the scaled residual (f - y) s rounded once: the same
// value as rounding f - y and scaling it.  CHECK: the targets may hold NaN
// or +-inf (Sec. "Fitness Functions": invalid values in the dataset are
// handled as in Eq. 2): a case whose output and target are both invalid is
// a matched pair and adds nothing, a case where exactly one of them is
// invalid marks the program (worst fitness).  Without CHECK (every target
// finite) an invalid output needs no mark: its residual is NaN or +-inf and
// so is the lane's sum from then on, which the reduction turns into the
// worst fitness, as it does a sum that overflows.
template <bool CHECK>
__device__ __forceinline__ void mse_case(float f, float ys, float s, float& hi, float& lo,
                                         bool& bad)
{
    const float d = fmaf(f, s, -ys);
    float t = d * d;
    if constexpr (CHECK) {
        const bool fv = __builtin_isfinite(f), yv = __builtin_isfinite(ys);
        bad |= fv != yv;
        t = fv && yv ? t : 0.f;
    }
    // Kahan's compensated step (every term is >= 0, so the running sum
    // dominates the term after the first few cases)
    const float yk = t + lo;
    const float u = hi + yk;
    lo = yk - (u - hi);
    hi = u;
}

// The value stack below the top lives in VGPR arrays of 32 floats ("chunks"):
// chunk c holds cases [c*J, (c+1)*J) of every slot, element index
// slot*J + (case mod J), J = 32 / MAXD.  A uniform dynamic index into a
// 32-element vector compiles to GPR-index-mode moves (smaller vectors would
// be expanded into compare/select chains).  `ix` is a staged cell number
// scaled by J, modulo 32 (so always inside the chunk).
#define GP_CHUNK_PUT(ix, j, v)                                                     \
    do {                                                                           \
        const uint32_t i_ = (ix) + ((j) % J);                                      \
        if ((j) / J == 0) c0[i_] = (v);                                            \
        else if ((j) / J == 1) c1[i_] = (v);                                       \
        else if ((j) / J == 2) c2[i_] = (v);                                       \
        else c3[i_] = (v);                                                         \
    } while (0)
#define GP_CHUNK_GET(ix, j)                                                        \
    (((j) / J == 0) ? c0[(ix) + ((j) % J)]                                         \
     : ((j) / J == 1) ? c1[(ix) + ((j) % J)]                                       \
     : ((j) / J == 2) ? c2[(ix) + ((j) % J)] : c3[(ix) + ((j) % J)])

// out[j] = a[j] OP b[j] for the four binary ops (b = top of stack, a = the
// element below it; SUB and DIV take a - b and a / b, GCL command table).
#define GP_BINARY_AB(bop, a, b, out)                                               \
    do {                                                                           \
        switch (bop) {                                                             \
        case GP_ADD:                                                               \
            _Pragma("unroll") for (int j = 0; j < K; ++j) out[j] = a[j] + b[j];    \
            break;                                                                 \
        case GP_SUB:                                                               \
            _Pragma("unroll") for (int j = 0; j < K; ++j) out[j] = a[j] - b[j];    \
            break;                                                                 \
        case GP_MUL:                                                               \
            _Pragma("unroll") for (int j = 0; j < K; ++j) out[j] = a[j] * b[j];    \
            break;                                                                 \
        default:                                                                   \
            _Pragma("unroll") for (int j = 0; j < K; ++j)                          \
                out[j] = div_protected(a[j], b[j]);                                \
            break;                                                                 \
        }                                                                          \
    } while (0)
#define GP_BINARY(bop, a, top) GP_BINARY_AB(bop, a, top, top)

// Runs one staged program on K cases per lane; xl points at this lane's
// first case of the LDS input tile.  A sub-tile's cases are laid out case-
// major: case j of lane t is element j*64 + t of a variable's row (row
// stride 64*K floats), so each of the K reads of a LOAD is a conflict-free,
// lane-contiguous LDS access.  The top of the stack is returned in tos[].
// Loads a leaf for K cases: the constant with bits `payload` when is_const,
// else the input row whose byte offset at four cases per lane is `payload`
// (halved at two cases per lane).
#define GP_LEAF(is_const, payload, out)                                            \
    do {                                                                           \
        if (is_const) {                                                            \
            const float c_ = __uint_as_float(payload);                             \
            _Pragma("unroll") for (int j = 0; j < K; ++j) out[j] = c_;             \
        } else {                                                                   \
            const float* xp_ = reinterpret_cast<const float*>(                     \
                reinterpret_cast<const char*>(xl) + ((payload) >> kRowShift));     \
            _Pragma("unroll") for (int j = 0; j < K; ++j) out[j] = xp_[j * 64];    \
        }                                                                          \
    } while (0)

// Whether any lane of the wavefront holds, among its K values, one with
// |v| > limit or a NaN: one compare per value into a lane mask, the masks
// OR-ed on the scalar unit.
template <int K>
__device__ __forceinline__ bool wave_any_above(const float (&v)[K], float limit)
{
    // the largest magnitude on the vector unit (a NaN drops out of the
    // maximum: the fast formulas propagate it), one compare into a mask
    float m = fabsf(v[0]);
#pragma unroll
    for (int j = 1; j < K; ++j) m = __builtin_fmaxf(m, fabsf(v[j]));
    return __ballot(m > limit) != 0ull;
}

// The commands beyond the benchmark set on the top values (unary
// selectors kUnSquare..15), per case, with the functions constant folding
// uses.
template <int K>
__device__ __forceinline__ void ext_unary(uint32_t sel, float (&t)[K])
{
    switch (sel) {
    case kUnSquare:
#pragma unroll
        for (int j = 0; j < K; ++j) t[j] = t[j] * t[j];
        break;
    case kUnSquare + 1:
#pragma unroll
        for (int j = 0; j < K; ++j) t[j] = -t[j];
        break;
    case kUnSquare + 2:
#pragma unroll
        for (int j = 0; j < K; ++j) t[j] = cube_value(t[j]);
        break;
    case kUnSquare + 3:
#pragma unroll
        for (int j = 0; j < K; ++j) t[j] = cbrt_value(t[j]);
        break;
    case kUnSquare + 4:
#pragma unroll
        for (int j = 0; j < K; ++j) t[j] = tan_value(t[j]);
        break;
    case kUnSquare + 5:
#pragma unroll
        for (int j = 0; j < K; ++j) t[j] = asin_value(t[j]);
        break;
    case kUnSquare + 6:
#pragma unroll
        for (int j = 0; j < K; ++j) t[j] = acos_value(t[j]);
        break;
    case kUnSquare + 7:
#pragma unroll
        for (int j = 0; j < K; ++j) t[j] = atan_value(t[j]);
        break;
    case kUnSquare + 8:
#pragma unroll
        for (int j = 0; j < K; ++j) t[j] = tanh_value(t[j]);
        break;
    default:
#pragma unroll
        for (int j = 0; j < K; ++j) t[j] = sqrt_raw(t[j]);
        break;
    }
}

// EXT: the interpreter for the whole command table (POW, the unary
// commands beyond the benchmark set, cell moves); without it the code is
// the benchmark set's alone.
template <int MAXD, int K, bool EXT>
__device__ __forceinline__ void run_program(const uint2* __restrict__ pc,
                                            const float* __restrict__ xl, float (&tos)[K])
{
    constexpr int J = 32 / MAXD;                  // cases per 32-float chunk
    static_assert(K % J == 0 && K / J <= 4, "chunking");
    // staged cell numbers times J, by one shift of the word (bits 14-15 of
    // a staged word are zero)
    constexpr uint32_t kLogJ = J == 4 ? 2u : (J == 2 ? 1u : 0u);
    static_assert((1 << kLogJ) == J, "J is 1, 2 or 4");
    // variable payloads are row offsets at four cases per lane
    constexpr uint32_t kRowShift = K == 4 ? 0u : 1u;
    static_assert(K == 4 || K == 2, "row offsets for 4 or 2 cases per lane");
    float c0[32], c1[32], c2[32], c3[32];
#pragma unroll
    for (int j = 0; j < K; ++j) tos[j] = 0.f;

    // Dispatch on flag bits, unary forms first (the most frequent); the
    // program's last instruction carries kFLast in the sign bit (no separate
    // trip count).  The loop is bound by scalar instructions per dispatch,
    // so the word is fetched with a 32-bit offset (one add per step) and
    // range tests run on the vector unit.  Stack indices are masked to the
    // 32-element chunk: the register index can never leave the chunk,
    // whatever the staged word says.
    uint32_t f;
    uint32_t off = 0;                          // byte offset of the next word
    do {
        const uint2 w = *reinterpret_cast<const uint2*>(
            reinterpret_cast<const char*>(pc) + off);
        off += 8u;
        f = w.x;
        const uint32_t sel = (f >> 8) & 0xFu;
        const uint32_t slot = (f >> (16u - kLogJ)) & 31u;
        if (f & kFUn) {
            if (f & kFPush) {
                // f(leaf): the old top is saved first
#pragma unroll
                for (int j = 0; j < K; ++j) GP_CHUNK_PUT(slot, j, tos[j]);
                GP_LEAF(f & kFConst, w.y, tos);
            }
        // unary: replaces the top
        const uint32_t uop = GP_SIN + sel;
        if (EXT && sel >= kUnSquare) {
            ext_unary<K>(sel, tos);
        } else {
            switch (uop) {
            case GP_SIN:
                // the fast kernel when every case of the wavefront has
                // |x| <= 2^17; otherwise per case, the library function
                // (with its large-argument reduction) beyond the fast range
                if (__builtin_expect(wave_any_above<K>(tos, kTrigFastLimit), 0)) {
#pragma unroll
                    for (int j = 0; j < K; ++j) tos[j] = sin_value(tos[j]);
                } else {
#pragma unroll
                    for (int j = 0; j < K; ++j) tos[j] = sin_fast(tos[j]);
                }
                break;
            case GP_COS:
                if (__builtin_expect(wave_any_above<K>(tos, kTrigFastLimit), 0)) {
#pragma unroll
                    for (int j = 0; j < K; ++j) tos[j] = cos_value(tos[j]);
                } else {
#pragma unroll
                    for (int j = 0; j < K; ++j) tos[j] = cos_fast(tos[j]);
                }
                break;
            case GP_EXP:
                // same split as sin/cos, at |x| <= 87 (per case values equal
                // exp_value's either way)
                if (__builtin_expect(wave_any_above<K>(tos, kExpFastLimit), 0)) {
#pragma unroll
                    for (int j = 0; j < K; ++j) tos[j] = exp_value(tos[j]);
                } else {
#pragma unroll
                    for (int j = 0; j < K; ++j) tos[j] = exp_fast(tos[j]);
                }
                break;
            case GP_LOG:
#pragma unroll
                for (int j = 0; j < K; ++j) tos[j] = log_protected(tos[j]);
                break;
            case GP_SQRT: {
                // the hardware root directly unless some case of the
                // wavefront is below the scaling threshold (or NaN);
                // sqrt_abs gives the same value for the others
                float mn = fabsf(tos[0]);
#pragma unroll
                for (int j = 1; j < K; ++j) mn = __builtin_fminf(mn, fabsf(tos[j]));
                if (__builtin_expect(__ballot(!(mn >= kSqrtTiny)) != 0ull, 0)) {
#pragma unroll
                    for (int j = 0; j < K; ++j) tos[j] = sqrt_value(tos[j]);
                } else {
#pragma unroll
                    for (int j = 0; j < K; ++j) tos[j] = __builtin_amdgcn_sqrtf(fabsf(tos[j]));
                }
                break;
            }
            default:
#pragma unroll
                for (int j = 0; j < K; ++j) tos[j] = fabsf(tos[j]);
                break;
            }
            }
        } else if (f & kFSBin) {
            // a = second from top (stack slot `slot`), b = top
            float sv[K];
#pragma unroll
            for (int j = 0; j < K; ++j) sv[j] = GP_CHUNK_GET(slot, j);
            if (EXT && sel == kBinPow) {
#pragma unroll
                for (int j = 0; j < K; ++j) tos[j] = pow_value(sv[j], tos[j]);
            } else {
                GP_BINARY(GP_ADD + sel, sv, tos);
            }
        } else if (f & kFLBin) {
            // top OP leaf; a constant leaf gets its own copy of the op
            // switch so the constant stays a scalar operand instead of
            // being broadcast into registers first
            if (EXT && sel == kBinPow) {
                float lv[K];
                GP_LEAF(f & kFConst, w.y, lv);
#pragma unroll
                for (int j = 0; j < K; ++j) tos[j] = pow_value(tos[j], lv[j]);
            } else if (f & kFConst) {
                float cv[K];
#pragma unroll
                for (int j = 0; j < K; ++j) cv[j] = __uint_as_float(w.y);
                GP_BINARY_AB(GP_ADD + sel, tos, cv, tos);
            } else {
                float lv[K];
                GP_LEAF(false, w.y, lv);
                GP_BINARY_AB(GP_ADD + sel, tos, lv, tos);
            }
        } else if (EXT && (f & kFMove)) {
            // cell move; every cell number is scaled by J and masked to a
            // multiple of J inside the chunk
            constexpr uint32_t kCellMask = 32u - J;
            const uint32_t rs = slot & kCellMask;
            const uint32_t ws = (w.y << kLogJ) & kCellMask;
            float tv[K];
#pragma unroll
            for (int j = 0; j < K; ++j) tv[j] = tos[j];
            if (sel & kMvRead) {
#pragma unroll
                for (int j = 0; j < K; ++j) tv[j] = GP_CHUNK_GET(rs, j);
            }
            if (sel & kMvWrite) {
#pragma unroll
                for (int j = 0; j < K; ++j) GP_CHUNK_PUT(ws, j, tos[j]);
            }
            if (sel & kMvTop) {
#pragma unroll
                for (int j = 0; j < K; ++j) tos[j] = tv[j];
            }
            if (sel & kMvCompact) {
                const uint32_t cs = ((w.y >> 8) << kLogJ) & kCellMask;
                const uint32_t cd = ((w.y >> 16) << kLogJ) & kCellMask;
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    const float v = GP_CHUNK_GET(cs, j);
                    GP_CHUNK_PUT(cd, j, v);
                }
            }
        } else {
            // the old top moves into the stack (slot MAXD-1 never holds a
            // live element, so a push onto an empty stack writes there),
            // the leaf becomes the top
#pragma unroll
            for (int j = 0; j < K; ++j) GP_CHUNK_PUT(slot, j, tos[j]);
            GP_LEAF(f & kFConst, w.y, tos);
        }
    } while ((int32_t)f >= 0);             // until kFLast (the sign bit)
}

// ------------------------------------------------- correlation fitness
// Per (program, tile) sums of the correlation fitness (Eq. 1-2) over the
// valid pairs (output and target both finite), kept about a shift (s, t)
// that is itself one valid pair of the data, so a large mean cancels before
// anything is squared: n valid pairs, Sd = sum (f - s), Sdd = sum (f - s)^2,
// Se = sum (y - t), See = sum (y - t)^2, Sde = sum (f - s)(y - t) in fp64,
// and the pairs with one (c1) or both (c2) sides invalid.  A wavefront
// shares one shift per (program, window), so its lanes add plainly; windows
// and tiles merge by the exact shift-change identities, in a fixed order.
struct CorrPart {
    double s, t, sd, sdd, se, see, sde;
    int64_t n, c1, c2;
};
static_assert(sizeof(CorrPart) == 80, "CorrPart layout");

// one lane's sums over its cases of a window (the shift is the wavefront's)
struct CorrLane {
    double sd, sdd, se, see, sde;
    int32_t n, c1, c2;
};

enum : int { kFitMse = 0, kFitCorr = 1, kFitReward = 2 };
constexpr int kCorrMaxG = 32;            // programs per work item in correlation mode (LDS)

__device__ __forceinline__ void corr_zero(CorrPart& c)
{
    c.s = c.t = c.sd = c.sdd = c.se = c.see = c.sde = 0.0;
    c.n = c.c1 = c.c2 = 0;
}
__device__ __forceinline__ void corr_zero(CorrLane& c)
{
    c.sd = c.sdd = c.se = c.see = c.sde = 0.0;
    c.n = c.c1 = c.c2 = 0;
}

// one case: f the program's output, y the target, (s, t) the shift
__device__ __forceinline__ void corr_case(CorrLane& c, float f, float y, double s, double t)
{
    const bool fv = __builtin_isfinite(f), yv = __builtin_isfinite(y);
    if (fv && yv) {
        const double d = (double)f - s, e = (double)y - t;
        c.sd += d;
        c.sdd = fma(d, d, c.sdd);
        c.se += e;
        c.see = fma(e, e, c.see);
        c.sde = fma(d, e, c.sde);
        ++c.n;
    } else if (fv != yv) {
        ++c.c1;
    } else {
        ++c.c2;
    }
}

// Integer point-to-point reward of one case (StdFitFunc, Eq. 5, and its
// Square/Cube/Hyper variants: the ratio raised to `power`), in fp32 as the
// paper's reward function takes fp32 values: M when both are zero, else
// rint(M ratio^p), less M/11 for opposite signs; an invalid pair gives -M
// (one side invalid) or +M (both).  rint rounds half to even.
__device__ __forceinline__ long long pair_reward(float o, float y, float M, int power)
{
    const bool ov = __builtin_isfinite(o), yv = __builtin_isfinite(y);
    if (!(ov && yv)) return (ov || yv) ? -(long long)M : (long long)M;
    const float ao = fabsf(o), ay = fabsf(y);
    const float mx = ao > ay ? ao : ay, mn = ao > ay ? ay : ao;
    if (mx == 0.0f) return (long long)M;
    const float r = mn / mx;
    float rp = r;
    if (power == 2) rp = r * r;
    else if (power == 3) rp = (r * r) * r;
    else if (power == 8) { const float r2 = r * r, r4 = r2 * r2; rp = r4 * r4; }
    float v = M * rp;
    if ((o < 0.0f && y > 0.0f) || (o > 0.0f && y < 0.0f)) v = v - M / 11.0f;
    return (long long)rintf(v);
}

// a += b (fixed order: the result depends only on the two operands).  b's
// sums move to a's shift: with dl = b.s - a.s and el = b.t - a.t,
// sum (f - a.s) = Sd + n dl, sum (f - a.s)^2 = Sdd + dl (2 Sd + n dl),
// sum (f - a.s)(y - a.t) = Sde + dl Se + el (Sd + n dl), and likewise in y.
__device__ __forceinline__ void corr_merge(CorrPart& a, const CorrPart& b)
{
    a.c1 += b.c1;
    a.c2 += b.c2;
    if (b.n == 0) return;
    if (a.n == 0) {
        a.s = b.s; a.t = b.t;
        a.sd = b.sd; a.sdd = b.sdd; a.se = b.se; a.see = b.see; a.sde = b.sde;
        a.n = b.n;
        return;
    }
    const double dl = b.s - a.s, el = b.t - a.t, nb = (double)b.n;
    a.sdd += b.sdd + dl * (2.0 * b.sd + nb * dl);
    a.see += b.see + el * (2.0 * b.se + nb * el);
    a.sde += b.sde + dl * b.se + el * (b.sd + nb * dl);
    a.sd += b.sd + nb * dl;
    a.se += b.se + nb * el;
    a.n += b.n;
}

// wavefront tree: every lane ends with the same sums (one shared shift,
// and fp64 addition is commutative, so both lanes of a pair agree)
__device__ __forceinline__ void corr_wave_reduce(CorrLane& c)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        c.sd += __shfl_xor(c.sd, off);
        c.sdd += __shfl_xor(c.sdd, off);
        c.se += __shfl_xor(c.se, off);
        c.see += __shfl_xor(c.see, off);
        c.sde += __shfl_xor(c.sde, off);
        c.n += __shfl_xor(c.n, off);
        c.c1 += __shfl_xor(c.c1, off);
        c.c2 += __shfl_xor(c.c2, off);
    }
}

template <int MAXD, int K, int FIT, bool EXT>
__global__ __launch_bounds__(kWG) void k_eval(
    const uint2* __restrict__ code, const ProgMeta* __restrict__ meta,
    const int32_t* __restrict__ order, const int32_t* __restrict__ class_info,
    uint32_t* __restrict__ work_counter, const DevDataset* __restrict__ ds,
    const int32_t* __restrict__ seg_ds, const int32_t* __restrict__ seg_cnt,
    const int32_t* __restrict__ seg_pos, const uint32_t* __restrict__ item_pre,
    const int32_t* __restrict__ class_g, float2* __restrict__ part, uint8_t* __restrict__ part_bad,
    CorrPart* __restrict__ part_corr, EvalConst a)
{
    static_assert(K == 2 || K == 4 || K == 8, "cases per lane");
    static_assert(MAXD == 8 || MAXD == 16 || MAXD == 32, "stack class");
    constexpr int J = 32 / MAXD;                  // cases per 32-float chunk
    static_assert(K % J == 0 && K / J <= 4, "chunking");
    constexpr int SUB = 64 * K;                   // cases per sub-tile
    extern __shared__ float lds[];
    float* xt = lds;                              // window: [W][n_vars + 1][SUB]
    float2* acc = reinterpret_cast<float2*>(lds + a.tile_floats);            // [G]
    uint32_t* accbad = reinterpret_cast<uint32_t*>(acc + a.G);               // [G]
    // correlation mode: one CorrPart per program instead (the tile floats are
    // a multiple of 2, so the array is 8-byte aligned)
    CorrPart* cacc = reinterpret_cast<CorrPart*>(lds + a.tile_floats);       // [G]
    // integer reward mode: one int64 total per program
    long long* racc = reinterpret_cast<long long*>(lds + a.tile_floats);     // [G]
    __shared__ uint32_t s_item, s_next;
    // With the classes overlapped, a deeper class's workgroups run beside
    // the depth <= 8 class's; their wavefronts issue first there, so the
    // deeper classes, which end last, finish sooner (alone, all wavefronts
    // of a kernel share one priority and nothing changes).
    if constexpr (MAXD >= 16) __builtin_amdgcn_s_setprio(1);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int c = a.cls;
    const int G = class_g[c];                     // <= a.G, the accumulators' capacity
    const int cstart = class_info[2 * c];
    const int32_t* __restrict__ cnt_c = seg_cnt + c * a.n_seg;
    const int32_t* __restrict__ pos_c = seg_pos + c * a.n_seg;
    const uint32_t* __restrict__ pre_c = item_pre + c * (a.n_seg + 1);
    const uint32_t n_items = pre_c[a.n_seg];
    int staged_d = -1;                            // dataset and first sub-tile in LDS
    int64_t staged = -1;
    int ynf = 0;                                  // the staged window holds a NaN/inf target

    for (;;) {
        if (tid == 0) s_item = atomicAdd(work_counter, 1u);
        if (tid < G) {
            if constexpr (FIT == kFitCorr) {
                corr_zero(cacc[tid]);
            } else if constexpr (FIT == kFitReward) {
                racc[tid] = 0;
            } else {
                acc[tid] = make_float2(0.f, 0.f);
                accbad[tid] = 0u;
            }
        }
        __syncthreads();
        const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= n_items) break;
        // segment of this item: last s with pre_c[s] <= item
        int sl = 0, sh = a.n_seg - 1;
        while (sl < sh) {
            const int mid = (sl + sh + 1) >> 1;
            if (pre_c[mid] <= item) sl = mid; else sh = mid - 1;
        }
        const int d = seg_ds[sl];
        // fields one by one: a struct copy indexed by the class would live
        // in scratch memory
        const DevDataset* __restrict__ Dp = ds + d;
        const float* __restrict__ Xd = Dp->X;
        const float* __restrict__ yd = Dp->y;
        const int64_t ld_x = Dp->ld_x;
        const int64_t n_cases = Dp->n_cases;
        const int n_vars = Dp->n_vars;
        const float scale = Dp->scale;
        const int passes = Dp->passes[c];
        const int window = Dp->window[c];
        const int count = cnt_c[sl];
        const int n_groups = (count + G - 1) / G;
        // item order inside a segment: tile-major (tile t of every group,
        // then tile t + 1), or, for the depth <= 8 class when the classes
        // run one after another, group-major (a group's case tiles are
        // consecutive items, so workgroups running at the same time read
        // the group's instruction words while they are in the cache).  The
        // order changes no result.
        const uint32_t local = item - pre_c[sl];
        const uint32_t n_tiles = (uint32_t)Dp->n_tiles[c];
        const bool gm = MAXD == 8 && a.group_major != 0;
        const int tile = gm ? (int)(local % n_tiles) : (int)(local / (uint32_t)n_groups);
        const int grp = gm ? (int)(local / n_tiles) : (int)(local % (uint32_t)n_groups);
        const int g0 = grp * G;
        const int gn = min(G, count - g0);
        const int obase = cstart + pos_c[sl] + g0;
        const int64_t n_sub = (n_cases + SUB - 1) / SUB;
        const int rows = n_vars + 1;              // inputs, then the targets

        for (int w0 = 0; w0 < passes; w0 += window) {
            const int64_t first = (int64_t)tile * passes + w0;      // first sub-tile
            if (first >= n_sub) break;
            const int nw = (int)min((int64_t)min(window, passes - w0), n_sub - first);
            if (first != staged || d != staged_d) {
                // lane t's case j of a sub-tile is element j*64 + t of a
                // row: conflict-free, lane-contiguous reads.  MSE mode
                // stores the targets pre-scaled (an exact power of two).
                int nf = 0;
                for (int i = tid; i < nw * rows * SUB; i += kWG) {
                    const int blk = i / (rows * SUB);
                    const int r = i - blk * rows * SUB;
                    const int v = r / SUB, cc = r - v * SUB;
                    const int64_t gi = (first + blk) * SUB + cc;
                    float val = 0.f;
                    if (gi < n_cases) {
                        if (v < n_vars) {
                            val = Xd[(int64_t)v * ld_x + gi];
                        } else {
                            val = FIT == kFitMse ? yd[gi] * scale : yd[gi];
                            nf |= !__builtin_isfinite(val);
                        }
                    }
                    xt[i] = val;
                }
                // (block-uniform branch: every thread reaches the barrier)
                ynf = __syncthreads_or(nf);
                staged = first;
                staged_d = d;
            }
            if (tid == 0) s_next = 0u;
            __syncthreads();
            // each wavefront takes the group's programs one at a time and
            // runs each over the whole window.  The loop has no lane-0-only
            // region at its head or tail: every lane adds one to the claim
            // counter (a wavefront's 64 claims are one block of 64, so the
            // block index is the program), and every lane writes the same
            // accumulator value after the wavefront tree.  A lane-0-only
            // claim followed by a lane-0-only update lets the optimizer rotate
            // the two into one region that lane 0 alone runs between
            // iterations, so the other lanes would re-read a stale claim.
            for (;;) {
                const int g = (int)(__builtin_amdgcn_readfirstlane(atomicAdd(&s_next, 1u)) >> 6);
                if (g >= gn) break;
                const int pid = order[obase + g];
                const ProgMeta m = meta[pid];
                // fused residual, validity and scaled compensated square sum
                // (MSE), or the sums of the correlation fitness
                float hi = 0.f, lo_ = 0.f;
                bool bad = false;
                CorrLane cl;
                if constexpr (FIT == kFitCorr) corr_zero(cl);
                double cs = 0.0, ct = 0.0;                // the wavefront's shift
                bool have_shift = false;
                long long rl = 0;
                for (int b = 0; b < nw; ++b) {
                    const float* blk = xt + b * rows * SUB;
                    float tos[K];
                    run_program<MAXD, K, EXT>(code + m.start, blk + lane, tos);
                    const int64_t base = (first + b) * SUB;
                    const float* yt = blk + n_vars * SUB;
                    if constexpr (FIT == kFitCorr) {
                        // the shift: the window's first valid pair, in the
                        // order (sub-tile, j, lane)
#pragma unroll
                        for (int j = 0; j < K; ++j) {
                            if (!have_shift) {
                                const float yj = yt[lane + j * 64];
                                const bool v = base + lane + j * 64 < n_cases &&
                                               __builtin_isfinite(tos[j]) && __builtin_isfinite(yj);
                                const unsigned long long mk = __ballot(v);
                                if (mk != 0ull) {
                                    const int src = __builtin_ctzll(mk);
                                    cs = (double)__int_as_float(__builtin_amdgcn_readlane(
                                        __float_as_int(tos[j]), src));
                                    ct = (double)__int_as_float(__builtin_amdgcn_readlane(
                                        __float_as_int(yj), src));
                                    have_shift = true;
                                }
                            }
                        }
                    }
                    if constexpr (FIT == kFitMse) {
                        // a whole sub-tile in range with finite targets: no
                        // per-case tests (wave-uniform branches)
                        if (base + SUB <= n_cases && !ynf) {
#pragma unroll
                            for (int j = 0; j < K; ++j)
                                mse_case<false>(tos[j], yt[lane + j * 64], scale, hi, lo_, bad);
                        } else {
#pragma unroll
                            for (int j = 0; j < K; ++j)
                                if (base + lane + j * 64 < n_cases)
                                    mse_case<true>(tos[j], yt[lane + j * 64], scale, hi, lo_,
                                                   bad);
                        }
                    } else {
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        if (base + lane + j * 64 < n_cases) {
                            const float f = tos[j];
                            if constexpr (FIT == kFitCorr) {
                                corr_case(cl, f, yt[lane + j * 64], cs, ct);
                            } else {
                                rl += pair_reward(f, yt[lane + j * 64], a.reward_M,
                                                  a.reward_power);
                            }
                        }
                    }
                    }
                }
                if constexpr (FIT == kFitCorr) {
                    corr_wave_reduce(cl);
                    // the windows add up in order, whichever wavefront ran
                    // them (every lane holds the same sums and writes the
                    // same merged value)
                    {
                        CorrPart w;
                        w.s = cs; w.t = ct;
                        w.sd = cl.sd; w.sdd = cl.sdd; w.se = cl.se; w.see = cl.see;
                        w.sde = cl.sde;
                        w.n = cl.n; w.c1 = cl.c1; w.c2 = cl.c2;
                        corr_merge(cacc[g], w);
                    }
                } else if constexpr (FIT == kFitReward) {
                    // integers: exact in any order (every lane holds the
                    // same total and writes the same sum)
#pragma unroll
                    for (int off = 32; off >= 1; off >>= 1) rl += __shfl_xor(rl, off);
                    racc[g] += rl;
                } else {
                // wavefront tree: every lane ends with the same pair
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) {
                    const float h2 = __shfl_xor(hi, off);
                    const float l2 = __shfl_xor(lo_, off);
                    acc_pair(hi, lo_, h2, l2);
                }
                const bool wave_bad = __ballot(bad) != 0ull;
                // one wavefront per program and window: the windows add up
                // in order, whichever wavefront ran them (every lane writes
                // the same pair)
                {
                    float h = acc[g].x, l = acc[g].y;
                    acc_pair(h, l, hi, lo_);
                    acc[g] = make_float2(h, l);
                    if (wave_bad) accbad[g] = 1u;
                }
                }
            }
            __syncthreads();
        }
        if (tid < gn) {
            const int pid = order[obase + tid];
            // tile-major partials: the reduction reads neighbours' together
            const int64_t slot = (int64_t)tile * a.part_stride + pid;
            if constexpr (FIT == kFitCorr) {
                part_corr[slot] = cacc[tid];
            } else if constexpr (FIT == kFitReward) {
                reinterpret_cast<long long*>(part)[slot] = racc[tid];
            } else {
                part[slot] = acc[tid];
                part_bad[slot] = (uint8_t)(accbad[tid] != 0u);
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ k_predict
// Per-case outputs f_p(x_i) of the programs of one depth class: persistent
// workgroups pull (group of four programs, sub-tile) items; each wavefront
// runs one program of the group and each lane writes its K values.
template <int MAXD, int K, bool EXT>
__global__ __launch_bounds__(kWG) void k_predict(
    const uint2* __restrict__ code, const ProgMeta* __restrict__ meta,
    const int32_t* __restrict__ order, const int32_t* __restrict__ class_info,
    uint32_t* __restrict__ work_counter, const float* __restrict__ X,
    float* __restrict__ out, int64_t ld_out, EvalConst a)
{
    constexpr int SUB = 64 * K;
    extern __shared__ float lds[];
    float* xt = lds;                              // [n_vars][SUB]
    __shared__ uint32_t s_item;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int start = class_info[2 * a.cls];
    const int count = class_info[2 * a.cls + 1];
    const int n_groups = (count + kWaves - 1) / kWaves;
    const int64_t n_sub = (a.n_cases + SUB - 1) / SUB;
    const uint64_t n_items = (uint64_t)n_groups * (uint64_t)n_sub;
    int64_t staged = -1;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(work_counter, 1u);
        __syncthreads();
        const uint64_t item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= n_items) break;
        const int64_t sub = (int64_t)(item / (uint64_t)n_groups);
        const int grp = (int)(item % (uint64_t)n_groups);
        const int64_t base = sub * SUB;
        if (sub != staged) {
            for (int i = tid; i < a.n_vars * SUB; i += kWG) {
                const int v = i / SUB, c = i - v * SUB;
                const int64_t gi = base + c;
                xt[i] = gi < a.n_cases ? X[(int64_t)v * a.ld_x + gi] : 0.f;
            }
            staged = sub;
        }
        __syncthreads();
        // wave-uniform (readfirstlane tells the compiler), so the
        // interpreter below keeps its scalar branches
        const int g = __builtin_amdgcn_readfirstlane(grp * kWaves + wave);
        if (g < count) {
            const int pid = order[start + g];
            const ProgMeta m = meta[pid];
            float tos[K];
            run_program<MAXD, K, EXT>(code + m.start, xt + lane, tos);
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int64_t gi = base + lane + j * 64;
                if (gi < a.n_cases) out[(int64_t)pid * ld_out + gi] = tos[j];
            }
        }
        __syncthreads();
    }
}

// NaN rows for programs that failed validation (one workgroup per program).
__global__ __launch_bounds__(256) void k_fill_invalid(const uint8_t* __restrict__ cls,
                                                      int64_t n_cases, float* __restrict__ out,
                                                      int64_t ld_out)
{
    const int64_t p = blockIdx.x;
    if (cls[p] < kKeys) return;
    for (int64_t i = threadIdx.x; i < n_cases; i += 256) out[p * ld_out + i] = __builtin_nanf("");
}

// ------------------------------------------------------------ k_reduce
struct ReduceArgs {
    const ProgMeta* meta;
    const uint8_t* cls;
    const int32_t* pds;             // request of each program
    const DevRequest* reqs;
    const int64_t* seg_start;
    const DevDataset* ds;
    const float2* part;
    const uint8_t* part_bad;
    const CorrPart* part_corr;
    int64_t n_programs;
    int32_t part_stride;    // tile stride of the partials (the program count)
    double max_score;
    int32_t* restage;       // k_validate's restage flag, cleared for the next call
};

// The restage flag is cleared here as well as by k_tables, for plans that
// run k_tables once, when they are captured.
__device__ __forceinline__ void clear_restage(const ReduceArgs& a)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.restage = 0;
}

__global__ __launch_bounds__(256) void k_reduce(ReduceArgs a)
{
    clear_restage(a);
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n_programs) return;
    const int r = a.pds[p];
    const DevRequest& R = a.reqs[r];
    const int64_t q = p - a.seg_start[r];
    if (!R.out || q >= R.n_programs) return;     // only for inconsistent tables
    const int c = a.cls[p];
    if (c >= kKeys) { R.out[q] = __builtin_nan(""); return; }
    const ProgMeta m = a.meta[p];
    const DevDataset& D = a.ds[R.dataset];
    const int nt = D.n_tiles[c / kLenBuckets];
    double s = 0.0;
    bool bad = false;
    for (int t = 0; t < nt; ++t) {
        const float2 v = a.part[(int64_t)t * a.part_stride + p];
        s += (double)v.x + (double)v.y;
        bad |= a.part_bad[(int64_t)t * a.part_stride + p] != 0;
    }
    const double mse = s * D.unscale;
    R.out[q] = (bad || !(mse <= (double)FLT_MAX)) ? __builtin_inf() : mse + D.tax * (double)m.len;
}

// Correlation score per program (Eq. 2 with r of Eq. 1 over the valid
// pairs): the tiles' shifted sums merged in order, then the centred sums
// Sxx = Sdd - Sd^2/n, Sxy = Sde - Sd Se/n, Syy = See - Se^2/n.  r = 0 below
// two valid pairs, or when a centred sum of squares is not positive (a
// constant output or target gives exactly zero: every shifted value is 0).
__global__ __launch_bounds__(256) void k_reduce_corr(ReduceArgs a)
{
    clear_restage(a);
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n_programs) return;
    const int r = a.pds[p];
    const DevRequest& R = a.reqs[r];
    const int64_t q = p - a.seg_start[r];
    if (!R.out || q >= R.n_programs) return;     // only for inconsistent tables
    const int c = a.cls[p];
    if (c >= kKeys) { R.out[q] = __builtin_nan(""); return; }
    const DevDataset& D = a.ds[R.dataset];
    const int nt = D.n_tiles[c / kLenBuckets];
    CorrPart acc;
    corr_zero(acc);
    for (int t = 0; t < nt; ++t) corr_merge(acc, a.part_corr[(int64_t)t * a.part_stride + p]);
    const int64_t n = acc.n, c1 = acc.c1, c2 = acc.c2;
    double rr = 0.0;
    if (n >= 2) {
        // centred sums from the shifted ones (the shift is a data value, so
        // these subtract quantities of the size of the spread)
        const double dn = (double)n;
        const double vx = acc.sdd - acc.sd * (acc.sd / dn);
        const double vy = acc.see - acc.se * (acc.se / dn);
        const double vxy = acc.sde - acc.sd * (acc.se / dn);
        if (vx > 0.0 && vy > 0.0) rr = vxy / sqrt(vx * vy);
    }
    const double r2 = rr * rr;
    R.out[q] = a.max_score * r2 * r2 * (double)n - a.max_score * (double)(c1 - c2);
}

// Integer reward per program (Eq. 5 and its power variants): the tiles'
// int64 totals added exactly, returned as a double (exact below 2^53).
__global__ __launch_bounds__(256) void k_reduce_reward(ReduceArgs a)
{
    clear_restage(a);
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n_programs) return;
    const int r = a.pds[p];
    const DevRequest& R = a.reqs[r];
    const int64_t q = p - a.seg_start[r];
    if (!R.out || q >= R.n_programs) return;     // only for inconsistent tables
    const int c = a.cls[p];
    if (c >= kKeys) { R.out[q] = __builtin_nan(""); return; }
    const DevDataset& D = a.ds[R.dataset];
    const int nt = D.n_tiles[c / kLenBuckets];
    const long long* part = reinterpret_cast<const long long*>(a.part);
    long long s = 0;
    for (int t = 0; t < nt; ++t) s += part[(int64_t)t * a.part_stride + p];
    R.out[q] = (double)s;
}

// ----------------------------------------------------------- workspaces
struct Layout {
    size_t code, meta, cls, order, blk_counts, blk_base, blk_slen, blk_code, class_info, class_g;
    size_t counters;
    size_t part, part_bad;
    size_t ds, req, seg_ds, seg_start, seg_cnt, seg_pos, item_pre, pds, bad, overflow, total;
};

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

Layout make_layout(int64_t n_programs, int64_t n_nodes, int32_t part_stride, int32_t n_ds,
                   int32_t n_seg, int fit = kFitMse)
{
    Layout L;
    const int64_t n_blk = (n_programs + kBucketBlock - 1) / kBucketBlock;
    size_t off = 0;
    // a staged program never holds more instructions than nodes
    L.code = off;       off = align_up(off + (size_t)(n_nodes + 1) * sizeof(uint2));
    L.meta = off;       off = align_up(off + (size_t)n_programs * sizeof(ProgMeta));
    L.cls = off;        off = align_up(off + (size_t)n_programs);
    L.order = off;      off = align_up(off + (size_t)n_programs * 4);
    L.blk_counts = off; off = align_up(off + (size_t)kKeys * n_blk * 4);
    L.blk_base = off;   off = align_up(off + (size_t)kKeys * n_blk * 4);
    L.blk_slen = off;   off = align_up(off + (size_t)n_blk * 8);
    L.blk_code = off;   off = align_up(off + (size_t)n_blk * 8);
    L.class_info = off; off = align_up(off + 2 * kClasses * 4);
    L.class_g = off;    off = align_up(off + kClasses * 4);
    L.counters = off;   off = align_up(off + kClasses * 4);
    // per (program, tile) partials: a compensated pair and a bad flag
    // (MSE), the correlation sums, or an int64 reward total
    const size_t part_elem = fit == kFitCorr ? sizeof(CorrPart) : sizeof(float2);
    L.part = off;       off = align_up(off + (size_t)n_programs * part_stride * part_elem);
    L.part_bad = off;   off = align_up(off + (fit != kFitMse ? 0 : (size_t)n_programs * part_stride));
    L.ds = off;         off = align_up(off + (size_t)n_ds * sizeof(DevDataset));
    L.req = off;        off = align_up(off + (size_t)n_seg * sizeof(DevRequest));
    L.seg_ds = off;     off = align_up(off + (size_t)n_seg * 4);
    L.seg_start = off;  off = align_up(off + (size_t)(n_seg + 1) * 8);
    L.seg_cnt = off;    off = align_up(off + (size_t)kClasses * n_seg * 4);
    L.seg_pos = off;    off = align_up(off + (size_t)kClasses * n_seg * 4);
    L.item_pre = off;   off = align_up(off + (size_t)kClasses * (n_seg + 1) * 4);
    L.pds = off;        off = align_up(off + (size_t)n_programs * 4);
    L.bad = off;        off = align_up(off + 8);    // tables bad, restage
    L.overflow = off;   off = align_up(off + 4);
    L.total = off;
    return L;
}

// Device views of one call's workspace.
struct Staged {
    uint2* code;
    ProgMeta* meta;
    uint8_t* cls;
    int32_t* order;
    int32_t* blk_counts;
    int32_t* blk_base;
    int64_t* blk_slen;
    int64_t* blk_code;
    int32_t* class_info;
    int32_t* class_g;
    uint32_t* counters;
    float2* part;
    uint8_t* part_bad;
    CorrPart* part_corr;            // the same memory as part, correlation mode
    DevDataset* ds;
    DevRequest* req;
    int32_t* seg_ds;
    int64_t* seg_start;
    int32_t* seg_cnt;
    int32_t* seg_pos;
    uint32_t* item_pre;
    int32_t* pds;
    int32_t* bad;
    int32_t* restage;
    int32_t* overflow;
};

Staged carve(void* base, const Layout& L)
{
    char* ws = static_cast<char*>(base);
    Staged st;
    st.code = reinterpret_cast<uint2*>(ws + L.code);
    st.meta = reinterpret_cast<ProgMeta*>(ws + L.meta);
    st.cls = reinterpret_cast<uint8_t*>(ws + L.cls);
    st.order = reinterpret_cast<int32_t*>(ws + L.order);
    st.blk_counts = reinterpret_cast<int32_t*>(ws + L.blk_counts);
    st.blk_base = reinterpret_cast<int32_t*>(ws + L.blk_base);
    st.blk_slen = reinterpret_cast<int64_t*>(ws + L.blk_slen);
    st.blk_code = reinterpret_cast<int64_t*>(ws + L.blk_code);
    st.class_info = reinterpret_cast<int32_t*>(ws + L.class_info);
    st.class_g = reinterpret_cast<int32_t*>(ws + L.class_g);
    st.counters = reinterpret_cast<uint32_t*>(ws + L.counters);
    st.part = reinterpret_cast<float2*>(ws + L.part);
    st.part_corr = reinterpret_cast<CorrPart*>(ws + L.part);
    st.part_bad = reinterpret_cast<uint8_t*>(ws + L.part_bad);
    st.ds = reinterpret_cast<DevDataset*>(ws + L.ds);
    st.req = reinterpret_cast<DevRequest*>(ws + L.req);
    st.seg_ds = reinterpret_cast<int32_t*>(ws + L.seg_ds);
    st.seg_start = reinterpret_cast<int64_t*>(ws + L.seg_start);
    st.seg_cnt = reinterpret_cast<int32_t*>(ws + L.seg_cnt);
    st.seg_pos = reinterpret_cast<int32_t*>(ws + L.seg_pos);
    st.item_pre = reinterpret_cast<uint32_t*>(ws + L.item_pre);
    st.pds = reinterpret_cast<int32_t*>(ws + L.pds);
    st.bad = reinterpret_cast<int32_t*>(ws + L.bad);
    st.restage = st.bad + 1;
    st.overflow = reinterpret_cast<int32_t*>(ws + L.overflow);
    return st;
}

// Side streams and fork/join events used when depth classes run
// concurrently.  Default priority, non-blocking.
struct SideStreams {
    hipStream_t s[2] = {nullptr, nullptr};
    hipEvent_t fork = nullptr, join[2] = {nullptr, nullptr};
    int create()
    {
        for (auto& x : s) GP_HIP_TRY(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
        GP_HIP_TRY(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        for (auto& e : join) GP_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        return GP_OK;
    }
    void destroy()
    {
        for (auto& x : s) if (x) (void)hipStreamDestroy(x);
        if (fork) (void)hipEventDestroy(fork);
        for (auto& e : join) if (e) (void)hipEventDestroy(e);
        s[0] = s[1] = nullptr;
        fork = join[0] = join[1] = nullptr;
    }
};

// Per-(device, caller stream) state of gp_eval / gp_predict.
struct Workspace {
    void* ptr = nullptr;
    size_t bytes = 0;
    SideStreams side;
};

std::mutex g_ws_mutex;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

int get_workspace(hipStream_t stream, size_t bytes, Workspace** out)
{
    int dev = 0;
    GP_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_ws_mutex);
    Workspace& w = g_ws[std::make_pair(dev, stream)];
    if (!w.side.s[0]) {
        int rc = w.side.create();
        if (rc != GP_OK) return rc;
    }
    if (w.bytes < bytes) {
        if (w.ptr) {
            // earlier work on this stream may still use the old buffer
            GP_HIP_TRY(hipStreamSynchronize(stream));
            GP_HIP_TRY(hipFree(w.ptr));
            w.ptr = nullptr;
            w.bytes = 0;
        }
        size_t want = bytes + bytes / 4;
        if (hipMalloc(&w.ptr, want) != hipSuccess) {
            (void)hipGetLastError();
            w.ptr = nullptr;
            return set_error(GP_E_NO_MEMORY, "workspace allocation of %zu bytes failed", want);
        }
        w.bytes = want;
    }
    *out = &w;
    return GP_OK;
}

struct DeviceInfo {
    int cus = 0;
};
std::mutex g_dev_mutex;
std::map<int, DeviceInfo> g_dev;

int device_cus(int* cus)
{
    int dev = 0;
    GP_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_dev_mutex);
    DeviceInfo& di = g_dev[dev];
    if (di.cus == 0) GP_HIP_TRY(hipDeviceGetAttribute(&di.cus, hipDeviceAttributeMultiprocessorCount, dev));
    *cus = di.cus;
    return GP_OK;
}

// ---------------------------------------------------------------- timing
struct Timing {
    bool on = false;
    // events of calls not yet read: GP_TIMING_PHASES boundaries per call
    std::vector<std::array<hipEvent_t, GP_TIMING_PHASES>> pending;
    double ms[GP_TIMING_PHASES] = {0, 0, 0, 0, 0, 0};
    int64_t calls = 0;
};
thread_local Timing g_timing;

// boundaries: b0 before prepare, b1 before class 0, b2 before class 1,
// b3 before class 2, b4 before reduce, b5 after reduce
struct CallEvents {
    std::array<hipEvent_t, GP_TIMING_PHASES> ev{};
    bool on = false;
    int begin(bool enable)
    {
        on = enable && g_timing.on;
        if (!on) return GP_OK;
        for (auto& e : ev) GP_HIP_TRY(hipEventCreate(&e));
        return GP_OK;
    }
    int mark(int i, hipStream_t s)
    {
        if (on) GP_HIP_TRY(hipEventRecord(ev[i], s));
        return GP_OK;
    }
    void commit()
    {
        if (on) g_timing.pending.push_back(ev);
    }
};

// ------------------------------------------------------------- problem
// Everything one evaluation needs (device pointers, sizes, scoring).  A
// single-population call carries its request and dataset inline (req_dev
// and ds_dev NULL); a batched call points at device tables.
struct Problem {
    gp_request one_req;             // inline request ...
    const gp_request* req_dev;      // ... or a device table of n_req
    int32_t n_req;
    gp_dataset one;                 // inline dataset ...
    const gp_dataset* ds_dev;       // ... or a device table of n_ds
    int32_t n_ds;
    int64_t n_programs;             // over all requests
    int64_t n_nodes;
    int32_t max_vars;
    int64_t max_cases;
    uint32_t allowed;
    int32_t need_out;               // fitness outputs required (not for gp_predict)
    int32_t fit;                    // kFitMse, kFitCorr or kFitReward
    double max_score;               // M of the correlation score or the reward
    int32_t reward_power;           // 1, 2, 3 or 8 (reward mode)
};

int check_common(int64_t n_programs, int64_t n_nodes, int64_t n_consts, int32_t n_vars,
                 int64_t ld_x, int64_t n_cases)
{
    if (n_programs < 0) return set_error(GP_E_INVALID_ARG, "n_programs < 0");
    if (n_programs > INT32_MAX - 1) return set_error(GP_E_TOO_LARGE, "n_programs > 2^31-2");
    if (n_nodes < 0) return set_error(GP_E_INVALID_ARG, "n_nodes < 0");
    if (n_nodes > (int64_t(1) << 40)) return set_error(GP_E_TOO_LARGE, "n_nodes > 2^40");
    if (n_consts < 0) return set_error(GP_E_INVALID_ARG, "n_consts < 0");
    if (n_consts > GP_MAX_CONSTS) return set_error(GP_E_TOO_LARGE, "n_consts > 2^24");
    if (n_vars < 0) return set_error(GP_E_INVALID_ARG, "n_vars < 0");
    if (n_vars > 4096) return set_error(GP_E_TOO_LARGE, "n_vars > 4096 (inputs are staged in LDS)");
    if (n_cases < 1) return set_error(GP_E_INVALID_ARG, "n_cases < 1");
    if (n_cases > (int64_t(1) << 40)) return set_error(GP_E_TOO_LARGE, "n_cases > 2^40");
    if (n_vars > 0 && ld_x < n_cases) return set_error(GP_E_INVALID_ARG, "ld_x < n_cases");
    return GP_OK;
}

int check_pointers(const uint32_t* nodes, int64_t n_nodes, const float* consts, int64_t n_consts,
                   const float* X, int32_t n_vars)
{
    if (n_nodes > 0 && !nodes) return set_error(GP_E_INVALID_ARG, "nodes is NULL");
    if (n_consts > 0 && !consts) return set_error(GP_E_INVALID_ARG, "consts is NULL");
    if (n_vars > 0 && !X) return set_error(GP_E_INVALID_ARG, "X is NULL");
    return GP_OK;
}

int check_problem(const Problem& pb)
{
    const bool batched = pb.req_dev != nullptr;
    int rc = check_common(pb.n_programs, pb.n_nodes, batched ? 0 : pb.one_req.n_consts,
                          pb.max_vars, batched ? pb.max_cases : pb.one.ld_x, pb.max_cases);
    if (rc != GP_OK) return rc;
    if (pb.allowed & ~GP_ALL_OPS)
        return set_error(GP_E_INVALID_ARG, "allowed_op_mask has bits beyond GP_ALL_OPS");
    if (batched) {
        if (!pb.ds_dev) return set_error(GP_E_INVALID_ARG, "datasets_dev is NULL");
        if (pb.n_ds < 1) return set_error(GP_E_INVALID_ARG, "n_datasets < 1");
        if (pb.n_req < 1) return set_error(GP_E_INVALID_ARG, "n_requests < 1");
        if (pb.n_req > kMaxRequests) return set_error(GP_E_TOO_LARGE, "more than %d requests", kMaxRequests);
        return GP_OK;
    }
    if (pb.n_programs == 0) return GP_OK;
    const gp_request& q = pb.one_req;
    if (!q.offsets) return set_error(GP_E_INVALID_ARG, "offsets is NULL");
    if (pb.need_out && !q.out_fitness) return set_error(GP_E_INVALID_ARG, "out_fitness is NULL");
    if ((rc = check_pointers(q.nodes, q.n_nodes, q.consts, q.n_consts, nullptr, 0)) != GP_OK) return rc;
    if (!pb.one.y) return set_error(GP_E_INVALID_ARG, "y is NULL");
    if (pb.one.n_vars > 0 && !pb.one.X) return set_error(GP_E_INVALID_ARG, "X is NULL");
    if (!std::isfinite(pb.one.tax_on_length)) return set_error(GP_E_INVALID_ARG, "tax_on_length is not finite");
    return GP_OK;
}

// --------------------------------------------------- launch configuration
// Launch knobs.  G, wg_per_cu and concurrent change no result.  The tile
// knobs (the LDS budget of an input window and the cap on case tiles per
// program) set how a program's cases are grouped into windows and tiles,
// so they fix its summation order together with (n_cases, its depth class,
// n_vars): every call with the same knobs gives the same bits, and the
// defaults are those of gp_eval, gp_eval_batched and the server.
struct Tuning {
    int G = 64;             // programs per work item, at most (small classes use fewer)
    int wg_per_cu = 0;      // persistent workgroups per CU (0: occupancy limit)
    int concurrent = 0;     // depth classes on forked streams (2: and the depth <= 8
                            // class leaves one workgroup slot per CU to the others)
    int tile_lds = kTileLds;    // LDS bytes of an input window
    int tile_max = kMaxTiles;   // case tiles per program, at most
};

struct EvalPtrs {
    const uint2* code;
    const ProgMeta* meta;
    const int32_t* order;
    const int32_t* class_info;
    uint32_t* work_counter;
    const float* X;
    const float* y;
    float2* part;
    uint8_t* part_bad;
};

template <int MAXD, int K>
size_t eval_tile_floats(int n_vars, int tile_lds)
{
    // every dataset's window fits the budget; a single sub-tile of a dataset
    // with very many variables may need more
    const size_t one = (size_t)(n_vars + 1) * 64 * K;
    const size_t budget = (size_t)tile_lds / sizeof(float);
    return one > budget ? one : budget;
}

template <int MAXD, int K, int FIT>
size_t eval_lds_bytes(int n_vars, int G, int tile_lds)
{
    const size_t acc = FIT == kFitCorr     ? (size_t)G * sizeof(CorrPart)
                       : FIT == kFitReward ? (size_t)G * sizeof(long long)
                                           : (size_t)G * (sizeof(float2) + sizeof(uint32_t));
    return eval_tile_floats<MAXD, K>(n_vars, tile_lds) * sizeof(float) + acc;
}

// Whether a call runs the interpreter built for the whole command table
// (its op mask reaches beyond the benchmark set).
inline bool pb_ext(uint32_t allowed) { return (allowed & ~GP_BASE_OPS) != 0u; }

// Grid size of one class kernel (LDS attribute set outside any capture).
template <int MAXD, int K, int FIT, bool EXT>
int eval_grid(int n_vars, int G, const Tuning& tu, int cus, int* grid, size_t* lds_out,
              int* refill = nullptr)
{
    const int wg_per_cu = tu.wg_per_cu;
    const size_t lds = eval_lds_bytes<MAXD, K, FIT>(n_vars, G, tu.tile_lds);
    if (lds > 64 * 1024) {
        GP_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_eval<MAXD, K, FIT, EXT>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    }
    int per_cu = 0;
    GP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_eval<MAXD, K, FIT, EXT>, kWG, lds));
    if (per_cu < 1) return set_error(GP_E_TOO_LARGE, "n_vars=%d needs %zu bytes of LDS per workgroup", n_vars, lds);
    if (wg_per_cu > 0 && wg_per_cu < per_cu) per_cu = wg_per_cu;
    // overlapped classes: the depth <= 8 class (launched first) runs one
    // workgroup per CU below its limit, so that the registers and LDS left
    // over hold a deeper class's workgroup from the start instead of its
    // whole run waiting for the first class to drain (and k_eval gives the
    // deeper classes' wavefronts issue priority)
    if (MAXD == 8 && tu.concurrent == 2 && per_cu > 1) {
        --per_cu;
        // the slot comes back once the deeper classes are done: a second
        // launch of one workgroup per CU on the stream of the last of them
        // joins the same work queue
        if (refill) *refill = cus;
    }
    *grid = cus * per_cu;
    *lds_out = lds;
    return GP_OK;
}

struct EvalLaunch {
    int32_t stride = 1;
    int32_t target_items = 1;   // work items per class worth keeping large groups for
    int grid[kClasses] = {0, 0, 0};
    int refill0 = 0;            // workgroups of the depth <= 8 class's second launch
    size_t lds[kClasses] = {0, 0, 0};
    Layout layout;
};

// Programs per work item at most (the LDS accumulators' capacity): the
// tuning's value, capped in correlation mode (larger per-program sums).
int group_capacity(const Problem& pb, const Tuning& tu)
{
    return pb.fit == kFitCorr && tu.G > kCorrMaxG ? kCorrMaxG : tu.G;
}

template <int FIT, bool EXT>
int eval_grids(const Problem& pb, const Tuning& tu, int G, int cus, EvalLaunch* el)
{
    int rc;
    if ((rc = eval_grid<8, 4, FIT, EXT>(pb.max_vars, G, tu, cus, &el->grid[0], &el->lds[0],
                                        &el->refill0)) != GP_OK) return rc;
    if ((rc = eval_grid<16, kK1, FIT, EXT>(pb.max_vars, G, tu, cus, &el->grid[1], &el->lds[1])) != GP_OK) return rc;
    return eval_grid<32, 2, FIT, EXT>(pb.max_vars, G, tu, cus, &el->grid[2], &el->lds[2]);
}

template <int FIT>
int eval_grids(const Problem& pb, const Tuning& tu, int G, int cus, EvalLaunch* el)
{
    return pb_ext(pb.allowed) ? eval_grids<FIT, true>(pb, tu, G, cus, el)
                              : eval_grids<FIT, false>(pb, tu, G, cus, el);
}

int configure_eval(const Problem& pb, const Tuning& tu, EvalLaunch* el)
{
    int cus = 0;
    int rc = device_cus(&cus);
    if (rc != GP_OK) return rc;
    el->stride = 1;
    for (int c = 0; c < kClasses; ++c) {
        // tile counts grow with n_cases, so the largest dataset sizes the
        // partial buffer
        const int32_t t = max_tiles(pb.max_cases, class_k(c, pb.max_vars), tu.tile_max);
        if (t > el->stride) el->stride = t;
    }
    el->target_items = 4 * 6 * cus;     // ~4 items per workgroup slot
    const int G = group_capacity(pb, tu);
    if (pb.fit == kFitCorr) rc = eval_grids<kFitCorr>(pb, tu, G, cus, el);
    else if (pb.fit == kFitReward) rc = eval_grids<kFitReward>(pb, tu, G, cus, el);
    else rc = eval_grids<kFitMse>(pb, tu, G, cus, el);
    if (rc != GP_OK) return rc;
    el->layout = make_layout(pb.n_programs, pb.n_nodes, el->stride, pb.n_ds, pb.n_req, pb.fit);
    return GP_OK;
}

// Dataset/segment tables, validation, staging and the stable (depth class,
// length) partition.
int enqueue_tables(const Problem& pb, const Tuning& tu, const Staged& st, hipStream_t stream)
{
    hipLaunchKernelGGL(k_tables, dim3(1), dim3(256), 0, stream, pb.ds_dev, pb.n_ds, pb.one,
                       pb.req_dev, pb.n_req, pb.one_req, pb.n_programs, pb.n_nodes, pb.max_vars,
                       pb.max_cases, pb.need_out, tu.tile_lds, tu.tile_max, st.ds, st.req,
                       st.seg_ds, st.seg_start, st.bad);
    GP_HIP_TRY(hipGetLastError());
    return GP_OK;
}

// tables_ready: the dataset and request tables in `st` are already those
// of this problem and tuning (a plan derives them once, when captured:
// its tables are kernel arguments, fixed for its life).
int enqueue_stage(const Problem& pb, const Tuning& tu, const Staged& st, int32_t target_items,
                  hipStream_t stream, bool tables_ready = false)
{
    const int32_t n_blk = (int32_t)((pb.n_programs + kBucketBlock - 1) / kBucketBlock);
    int rc;
    if (!tables_ready && (rc = enqueue_tables(pb, tu, st, stream)) != GP_OK) return rc;
    const int32_t lpt = pb.n_req == 1 ? 1 : 0;
    hipLaunchKernelGGL(k_validate, dim3(n_blk), dim3(kBucketBlock), 0, stream, pb.n_programs,
                       pb.allowed, st.ds, st.req, st.seg_start, pb.n_req, st.bad, lpt, n_blk,
                       st.meta, st.cls, st.pds, st.blk_counts, st.blk_slen, st.code, st.restage);
    GP_HIP_TRY(hipGetLastError());
    SegOut so{pb.n_req == 1 ? 1 : 0, group_capacity(pb, tu), target_items, st.seg_ds, st.ds,
              st.seg_cnt, st.seg_pos, st.item_pre, st.class_g};
    hipLaunchKernelGGL(k_class_scan, dim3(1), dim3(1024), 0, stream, st.blk_counts, st.blk_slen,
                       n_blk, pb.n_nodes, st.blk_base, st.blk_code, st.class_info, st.counters,
                       st.overflow, so);
    GP_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_stage, dim3(n_blk), dim3(kBucketBlock), 0, stream, pb.n_programs, st.ds,
                       st.req, st.seg_start, st.pds, n_blk, st.blk_code, st.blk_base, st.overflow,
                       st.restage, pb.allowed, st.cls, st.meta, st.code, st.order);
    GP_HIP_TRY(hipGetLastError());
    return GP_OK;
}

// One class kernel of the evaluation (EXT: the interpreter for the whole
// command table, picked by the op mask).
template <int MD, int KK, int FIT>
void launch_eval(bool ext, dim3 g, size_t lds, hipStream_t sc, const Staged& st, int c,
                 const EvalConst& ea)
{
    if (ext)
        hipLaunchKernelGGL((k_eval<MD, KK, FIT, true>), g, dim3(kWG), lds, sc, st.code, st.meta,
                           st.order, st.class_info, st.counters + c, st.ds, st.seg_ds, st.seg_cnt,
                           st.seg_pos, st.item_pre, st.class_g, st.part, st.part_bad, st.part_corr,
                           ea);
    else
        hipLaunchKernelGGL((k_eval<MD, KK, FIT, false>), g, dim3(kWG), lds, sc, st.code, st.meta,
                           st.order, st.class_info, st.counters + c, st.ds, st.seg_ds, st.seg_cnt,
                           st.seg_pos, st.item_pre, st.class_g, st.part, st.part_bad, st.part_corr,
                           ea);
}

// The whole evaluation as stream work (no allocation, no synchronization:
// safe to capture into a graph).
int enqueue_eval(const Problem& pb, const Tuning& tu, const EvalLaunch& el, const Staged& st,
                 SideStreams& side, hipStream_t stream, CallEvents& ce, bool tables_ready = false)
{
    int rc;
    if ((rc = ce.mark(0, stream)) != GP_OK) return rc;
    if ((rc = enqueue_stage(pb, tu, st, el.target_items, stream, tables_ready)) != GP_OK) return rc;
    if (pb.n_req > 1) {
        hipLaunchKernelGGL(k_seg_tables, dim3(1), dim3(256), 0, stream, st.order, st.class_info,
                           st.seg_start, pb.n_req, st.bad, st.seg_ds, st.ds, group_capacity(pb, tu),
                           el.target_items, st.seg_cnt, st.seg_pos, st.item_pre, st.class_g);
        GP_HIP_TRY(hipGetLastError());
    }

    EvalConst ea{};
    ea.G = group_capacity(pb, tu);
    ea.part_stride = (int32_t)pb.n_programs;      // tile stride of the partials
    ea.max_vars = pb.max_vars;
    ea.n_seg = pb.n_req;
    ea.reward_power = pb.reward_power;
    ea.reward_M = (float)pb.max_score;
    // group-major items in the depth <= 8 class pay when that class has the
    // GPU to itself; overlapped with the other classes, tile-major is faster
    ea.group_major = tu.concurrent ? 0 : 1;
    if (tu.concurrent) {
        GP_HIP_TRY(hipEventRecord(side.fork, stream));
        for (auto& x : side.s) GP_HIP_TRY(hipStreamWaitEvent(x, side.fork, 0));
    }
    const bool ext = pb_ext(pb.allowed);
    for (int c = 0; c < kClasses; ++c) {
        if ((rc = ce.mark(1 + c, stream)) != GP_OK) return rc;
        const hipStream_t sc = (tu.concurrent && c > 0) ? side.s[c - 1] : stream;
        ea.cls = c;
        const dim3 g(el.grid[c]);
#define GP_LAUNCH_EVAL(MD, KK)                                                                 \
        do {                                                                                   \
            if (pb.fit == kFitCorr)                                                            \
                launch_eval<MD, KK, kFitCorr>(ext, g, el.lds[c], sc, st, c, ea);               \
            else if (pb.fit == kFitReward)                                                     \
                launch_eval<MD, KK, kFitReward>(ext, g, el.lds[c], sc, st, c, ea);             \
            else                                                                               \
                launch_eval<MD, KK, kFitMse>(ext, g, el.lds[c], sc, st, c, ea);                \
        } while (0)
        if (c == 0) {
            ea.tile_floats = (int32_t)eval_tile_floats<8, 4>(pb.max_vars, tu.tile_lds);
            GP_LAUNCH_EVAL(8, 4);
        } else if (c == 1) {
            ea.tile_floats = (int32_t)eval_tile_floats<16, kK1>(pb.max_vars, tu.tile_lds);
            GP_LAUNCH_EVAL(16, kK1);
        } else {
            ea.tile_floats = (int32_t)eval_tile_floats<32, 2>(pb.max_vars, tu.tile_lds);
            GP_LAUNCH_EVAL(32, 2);
        }
#undef GP_LAUNCH_EVAL
        GP_HIP_TRY(hipGetLastError());
    }
    if (el.refill0 > 0 && tu.concurrent == 2) {
        // the depth <= 8 class takes back its slot after the depth <= 16
        // class (same work counter: the items are shared, each taken once)
        ea.cls = 0;
        ea.tile_floats = (int32_t)eval_tile_floats<8, 4>(pb.max_vars, tu.tile_lds);
        const dim3 g(el.refill0);
        const int c = 0;
        const hipStream_t sc = side.s[0];
        if (pb.fit == kFitCorr) launch_eval<8, 4, kFitCorr>(ext, g, el.lds[c], sc, st, c, ea);
        else if (pb.fit == kFitReward) launch_eval<8, 4, kFitReward>(ext, g, el.lds[c], sc, st, c, ea);
        else launch_eval<8, 4, kFitMse>(ext, g, el.lds[c], sc, st, c, ea);
        GP_HIP_TRY(hipGetLastError());
    }
    if (tu.concurrent) {
        for (int i = 0; i < 2; ++i) {
            GP_HIP_TRY(hipEventRecord(side.join[i], side.s[i]));
            GP_HIP_TRY(hipStreamWaitEvent(stream, side.join[i], 0));
        }
    }
    ReduceArgs ra{};
    ra.meta = st.meta; ra.cls = st.cls; ra.pds = st.pds; ra.reqs = st.req;
    ra.seg_start = st.seg_start; ra.ds = st.ds;
    ra.part = st.part; ra.part_bad = st.part_bad; ra.part_corr = st.part_corr;
    ra.n_programs = pb.n_programs; ra.part_stride = (int32_t)pb.n_programs;
    ra.max_score = pb.max_score;
    ra.restage = st.restage;
    if ((rc = ce.mark(4, stream)) != GP_OK) return rc;
    if (pb.fit == kFitCorr)
        hipLaunchKernelGGL(k_reduce_corr, dim3((unsigned)((pb.n_programs + 255) / 256)), dim3(256),
                           0, stream, ra);
    else if (pb.fit == kFitReward)
        hipLaunchKernelGGL(k_reduce_reward, dim3((unsigned)((pb.n_programs + 255) / 256)),
                           dim3(256), 0, stream, ra);
    else
        hipLaunchKernelGGL(k_reduce, dim3((unsigned)((pb.n_programs + 255) / 256)), dim3(256), 0,
                           stream, ra);
    GP_HIP_TRY(hipGetLastError());
    if ((rc = ce.mark(5, stream)) != GP_OK) return rc;
    return GP_OK;
}

template <int MAXD, int K, bool EXT>
int launch_predict(const EvalPtrs& p, float* out, int64_t ld_out, const EvalConst& args,
                   hipStream_t stream, int cus)
{
    const size_t lds = (size_t)args.n_vars * 64 * K * sizeof(float);
    if (lds > 64 * 1024) {
        GP_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_predict<MAXD, K, EXT>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    }
    int per_cu = 0;
    GP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_predict<MAXD, K, EXT>, kWG, lds));
    if (per_cu < 1) return set_error(GP_E_TOO_LARGE, "n_vars=%d needs %zu bytes of LDS per workgroup", args.n_vars, lds);
    hipLaunchKernelGGL((k_predict<MAXD, K, EXT>), dim3(cus * per_cu), dim3(kWG), lds, stream, p.code,
                       p.meta, p.order, p.class_info, p.work_counter, p.X, out, ld_out, args);
    GP_HIP_TRY(hipGetLastError());
    return GP_OK;
}

// ----------------------------------------------------------------- autotune
// In-process cache of tuned scheduling knobs, optionally mirrored in a
// text file named by GPEVAL_TUNE_CACHE (one "key G wg_per_cu concurrent"
// line per entry).  Keys describe the workload shape, not its values.
std::mutex g_tune_mutex;
std::map<std::string, Tuning> g_tune;
bool g_tune_loaded = false;

std::string tune_key(const Problem& pb)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    char name[64] = {0};
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) snprintf(name, sizeof name, "%s", prop.gcnArchName);
    for (char* c = name; *c; ++c) if (*c == ' ' || *c == ':') *c = '_';
    const double mean_len = pb.n_programs ? (double)pb.n_nodes / (double)pb.n_programs : 0.0;
    int lp = 0;
    while ((int64_t(1) << (lp + 1)) <= pb.n_programs) ++lp;
    int lc = 0;
    while ((int64_t(1) << (lc + 1)) <= pb.max_cases) ++lc;
    char buf[160];
    snprintf(buf, sizeof buf, "%s/cases2^%d/vars%d/progs2^%d/len%d/reqs%d", name, lc,
             pb.max_vars, lp, (int)(mean_len + 0.5), pb.n_req);
    return buf;
}

void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = getenv("GPEVAL_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char key[200];
    Tuning t;
    while (fscanf(f, "%199s %d %d %d %d %d", key, &t.G, &t.wg_per_cu, &t.concurrent, &t.tile_lds,
                  &t.tile_max) == 6)
        g_tune[key] = t;
    fclose(f);
}

void tune_store_locked(const std::string& key, const Tuning& t)
{
    g_tune[key] = t;
    const char* path = getenv("GPEVAL_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d %d %d\n", key.c_str(), t.G, t.wg_per_cu, t.concurrent, t.tile_lds,
            t.tile_max);
    fclose(f);
}

}  // namespace

// ================================================================== plans
struct gp_plan {
    Problem pb;
    Tuning tu;
    EvalLaunch el;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    Staged st;
    SideStreams side;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
    double tuned_ms = 0.0;
    int tune_trials = 0;
};

namespace {

void plan_release_graph(gp_plan* p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

// (Re)size the plan's workspace and capture its graph.
int plan_build(gp_plan* p)
{
    int rc = configure_eval(p->pb, p->tu, &p->el);
    if (rc != GP_OK) return rc;
    if (p->ws_bytes < p->el.layout.total) {
        if (p->ws) {
            GP_HIP_TRY(hipDeviceSynchronize());
            GP_HIP_TRY(hipFree(p->ws));
            p->ws = nullptr;
            p->ws_bytes = 0;
        }
        if (hipMalloc(&p->ws, p->el.layout.total) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(GP_E_NO_MEMORY, "plan workspace of %zu bytes", p->el.layout.total);
        }
        p->ws_bytes = p->el.layout.total;
    }
    p->st = carve(p->ws, p->el.layout);
    // replays of a previous graph may still read the workspace
    if (p->exec) GP_HIP_TRY(hipDeviceSynchronize());
    plan_release_graph(p);
    // the plan's tables (kernel arguments only) once, outside the graph
    if ((rc = enqueue_tables(p->pb, p->tu, p->st, p->cap)) != GP_OK) return rc;
    GP_HIP_TRY(hipStreamSynchronize(p->cap));
    GP_HIP_TRY(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    CallEvents none;
    (void)none.begin(false);
    rc = enqueue_eval(p->pb, p->tu, p->el, p->st, p->side, p->cap, none, true);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(p->cap, &g);
    if (rc != GP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (ec != hipSuccess) return set_error(GP_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ec));
    p->graph = g;
    GP_HIP_TRY(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    return GP_OK;
}

// Median of `runs` timed runs of one configuration (after one warm-up when
// `warm`), or a negative value when it does not fit the plan's workspace.
int time_config(gp_plan* p, const Tuning& t, hipStream_t stream, hipEvent_t e0, hipEvent_t e1,
                float* ms_out, int runs = 5, bool warm = true)
{
    *ms_out = -1.f;
    EvalLaunch el;
    int rc = configure_eval(p->pb, t, &el);
    if (rc != GP_OK) return rc;
    if (el.layout.total > p->ws_bytes) return GP_OK;
    const Staged st = carve(p->ws, el.layout);
    CallEvents none;
    (void)none.begin(false);
    float ms[8];
    runs = std::min(std::max(runs, 1), 8);
    if (warm && (rc = enqueue_eval(p->pb, t, el, st, p->side, stream, none)) != GP_OK) return rc;
    for (int r = 0; r < runs; ++r) {
        GP_HIP_TRY(hipEventRecord(e0, stream));
        if ((rc = enqueue_eval(p->pb, t, el, st, p->side, stream, none)) != GP_OK) return rc;
        GP_HIP_TRY(hipEventRecord(e1, stream));
        GP_HIP_TRY(hipEventSynchronize(e1));
        GP_HIP_TRY(hipEventElapsedTime(&ms[r], e0, e1));
    }
    std::sort(ms, ms + runs);
    *ms_out = ms[runs / 2];
    return GP_OK;
}

// Time candidate knobs on the real inputs and keep the fastest: coordinate
// descent over five axes (programs per work item, workgroups per CU, depth
// classes on forked streams, the LDS budget of an input window, the cap on
// case tiles per program), each axis tried in turn with the others at their
// best so far, two sweeps, each candidate the median of five runs; then the
// three fastest candidates are timed again in turns (five rounds, one run
// each per round, so drift hits them alike) and the lowest median wins.
// The tile axes set a program's summation order, so the chosen plan is
// deterministic for its problem shape (the tuning is cached by it) but may
// differ from gp_eval in the last bits.
int plan_autotune(gp_plan* p, hipStream_t stream)
{
    const std::string key = tune_key(p->pb);
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        tune_load_locked();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            p->tu = it->second;
            return GP_OK;
        }
    }
    hipEvent_t e0, e1;
    GP_HIP_TRY(hipEventCreate(&e0));
    GP_HIP_TRY(hipEventCreate(&e1));
    const int kAxes = 5;
    const std::vector<int> values[kAxes] = {{32, 64, 128}, {0, 3, 4}, {0, 1, 2},
                                            {12 * 1024, 24 * 1024, 40 * 1024}, {2, 8, 32}};
    auto field = [](Tuning& t, int a) -> int& {
        return a == 0 ? t.G : a == 1 ? t.wg_per_cu : a == 2 ? t.concurrent
                                                            : a == 3 ? t.tile_lds : t.tile_max;
    };
    Tuning best = p->tu;
    float best_ms = 1e30f;
    int rc = time_config(p, best, stream, e0, e1, &best_ms);
    if (rc == GP_OK && best_ms < 0.f) best_ms = 1e30f;
    int tried = 1;
    std::vector<std::pair<float, Tuning>> seen;
    if (best_ms < 1e30f) seen.push_back({best_ms, best});
    for (int sweep = 0; sweep < 2 && rc == GP_OK; ++sweep) {
        for (int a = 0; a < kAxes && rc == GP_OK; ++a) {
            for (int v : values[a]) {
                Tuning t = best;
                if (field(t, a) == v) continue;
                field(t, a) = v;
                float ms = -1.f;
                if ((rc = time_config(p, t, stream, e0, e1, &ms)) != GP_OK) break;
                ++tried;
                if (ms >= 0.f) seen.push_back({ms, t});
                if (ms >= 0.f && ms < best_ms) {
                    best_ms = ms;
                    best = t;
                }
            }
        }
    }
    // run-off among the three fastest distinct candidates
    if (rc == GP_OK && seen.size() > 1) {
        std::stable_sort(seen.begin(), seen.end(),
                         [](const std::pair<float, Tuning>& x, const std::pair<float, Tuning>& y) {
                             return x.first < y.first;
                         });
        auto same = [](const Tuning& x, const Tuning& y) {
            return x.G == y.G && x.wg_per_cu == y.wg_per_cu && x.concurrent == y.concurrent &&
                   x.tile_lds == y.tile_lds && x.tile_max == y.tile_max;
        };
        std::vector<Tuning> top;
        for (const auto& c : seen) {
            bool dup = false;
            for (const auto& u : top) dup = dup || same(u, c.second);
            if (!dup) top.push_back(c.second);
            if (top.size() == 3) break;
        }
        std::vector<std::vector<float>> smp(top.size());
        for (int round = 0; round < 5 && rc == GP_OK; ++round)
            for (size_t i = 0; i < top.size() && rc == GP_OK; ++i) {
                float ms = -1.f;
                if ((rc = time_config(p, top[i], stream, e0, e1, &ms, 1, round == 0)) == GP_OK)
                    smp[i].push_back(ms);
            }
        if (rc == GP_OK) {
            for (size_t i = 0; i < top.size(); ++i) {
                std::sort(smp[i].begin(), smp[i].end());
                const float med = smp[i][smp[i].size() / 2];
                if (i == 0 || med < best_ms) {
                    best_ms = med;
                    best = top[i];
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != GP_OK) return rc;
    p->tu = best;
    p->tuned_ms = best_ms;
    p->tune_trials = tried;
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    tune_store_locked(key, best);
    return GP_OK;
}

Problem make_problem(const gp_problem* d)
{
    Problem pb{};
    pb.one_req.nodes = d->nodes; pb.one_req.offsets = d->offsets; pb.one_req.consts = d->consts;
    pb.one_req.n_programs = d->n_programs; pb.one_req.n_nodes = d->n_nodes;
    pb.one_req.n_consts = d->n_consts;
    pb.one_req.out_fitness = d->out_fitness; pb.one_req.out_status = d->out_status;
    pb.one_req.dataset = 0;
    pb.req_dev = nullptr; pb.n_req = 1;
    pb.one.X = d->X; pb.one.y = d->y; pb.one.ld_x = d->ld_x; pb.one.n_cases = d->n_cases;
    pb.one.tax_on_length = d->tax_on_length; pb.one.n_vars = d->n_vars; pb.one.reserved = 0;
    pb.ds_dev = nullptr; pb.n_ds = 1;
    pb.n_programs = d->n_programs; pb.n_nodes = d->n_nodes;
    pb.max_vars = d->n_vars; pb.max_cases = d->n_cases;
    pb.allowed = d->allowed_op_mask ? d->allowed_op_mask : GP_BASE_OPS;
    pb.need_out = 1;
    return pb;
}

int eval_problem(const Problem& pb, hipStream_t stream)
{
    int rc = check_problem(pb);
    if (rc != GP_OK || pb.n_programs == 0) return rc;
    Tuning tu;
    EvalLaunch el;
    if ((rc = configure_eval(pb, tu, &el)) != GP_OK) return rc;
    Workspace* w = nullptr;
    if ((rc = get_workspace(stream, el.layout.total, &w)) != GP_OK) return rc;
    const Staged st = carve(w->ptr, el.layout);
    CallEvents ce;
    if ((rc = ce.begin(true)) != GP_OK) return rc;
    if ((rc = enqueue_eval(pb, tu, el, st, w->side, stream, ce)) != GP_OK) return rc;
    ce.commit();
    return GP_OK;
}

// ------------------------------------------------- no-allocation form
// gp_eval_noalloc keeps its workspace in one fixed device array per GPU
// instead of memory the library allocates.  In host code `scratch` names a
// host-side stand-in, never the device memory: its device address is taken
// with hipGetSymbolAddress once per device (with that device current, each
// GPU holding its own copy) and only that address reaches kernels.  Every
// kernel of the call initializes what it reads (counters, flags, partials),
// so no clearing is needed between calls; calls that overlap in time on one
// GPU share the array and race.
constexpr size_t kScratchBytes = GP_NOALLOC_WORKSPACE_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// This device's scratch address; the first call on a device takes it and
// also caches the device's CU count (the only set-up that may touch host
// containers).
int scratch_for_device(void** out)
{
    int dev = 0;
    GP_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices)
        return set_error(GP_E_INVALID_ARG, "device %d: the fixed workspace covers devices 0..%d", dev,
                         kMaxScratchDevices - 1);
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return set_error(GP_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        }
        int cus = 0;
        const int rc = device_cus(&cus);
        if (rc != GP_OK) return rc;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GP_OK;
}

// gp_eval's work on the fixed array: every depth class on the caller's
// stream (no side streams), no timing events, no allocation.
int eval_problem_noalloc(const Problem& pb, hipStream_t stream)
{
    int rc = check_problem(pb);
    if (rc != GP_OK || pb.n_programs == 0) return rc;
    void* base = nullptr;
    if ((rc = scratch_for_device(&base)) != GP_OK) return rc;
    Tuning tu;
    tu.concurrent = 0;
    EvalLaunch el;
    if ((rc = configure_eval(pb, tu, &el)) != GP_OK) return rc;
    if (el.layout.total > kScratchBytes)
        return set_error(GP_E_TOO_LARGE, "the call needs %zu bytes of workspace; the fixed array holds %zu",
                         el.layout.total, kScratchBytes);
    const Staged st = carve(base, el.layout);
    SideStreams unused;
    CallEvents ce;
    if ((rc = ce.begin(false)) != GP_OK) return rc;
    return enqueue_eval(pb, tu, el, st, unused, stream, ce);
}

// ------------------------------------------------- Monte-Carlo ranking
// The paper's ranking without a sort (Sec. "Monte-Carlo Ranking", Table 2):
// a random sample of the population's fitness values estimates the
// percentiles, then one pass places every individual in its percentile
// band and gives the band's expected number of children.
//
// key(v): larger is better; NaN (a program that could not be scored) is
// the worst value and ties with -inf (an invalid MSE of +inf).
__device__ __forceinline__ double rank_key(double v, int higher_is_better)
{
    if (v != v) return -__builtin_inf();
    return higher_is_better ? v : -v;
}

// SplitMix64 (Steele, Lea, Flood 2014): the k-th output of the sequence
// started at `seed`, computed directly from the counter.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

constexpr int kMaxRankSample = 1024;

// One workgroup: draw the sample (index k = high 64 bits of h_k * n), read
// the keys, sort them ascending by counting (ties by sample position, so
// the order is a function of the keys only), store them.
__global__ __launch_bounds__(1024) void k_rank_sample(const double* __restrict__ fitness,
                                                      int64_t n, int32_t higher, uint64_t seed,
                                                      int32_t S, double* __restrict__ sorted)
{
    __shared__ double keys[kMaxRankSample];
    const int t = threadIdx.x;
    if (t < S) {
        const uint64_t h = splitmix64_at(seed, (uint64_t)t);
        const int64_t idx = (int64_t)__umul64hi(h, (uint64_t)n);
        keys[t] = rank_key(fitness[idx], higher);
    }
    __syncthreads();
    if (t < S) {
        const double v = keys[t];
        int pos = 0;
        for (int j = 0; j < S; ++j) {
            const double u = keys[j];
            pos += (u < v) || (u == v && j < t);
        }
        sorted[pos] = v;
    }
}

// Expected children per percentile band (Table 2), band b = 10 b ... 10 b + 9.
__constant__ float kChildrenByBand[10] = {0.01f, 0.03f, 0.06f, 0.15f, 0.25f,
                                          0.5f, 1.0f, 1.5f, 2.5f, 4.0f};

// One thread per individual: the percentile is 100 x (sampled keys strictly
// below its key) / S, rounded down; the band is that percentile's tens digit
// (90 and above is the top band).
__global__ __launch_bounds__(256) void k_rank_assign(const double* __restrict__ fitness, int64_t n,
                                                     int32_t higher, int32_t S,
                                                     const double* __restrict__ sorted,
                                                     int32_t* __restrict__ out_band,
                                                     float* __restrict__ out_children)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = rank_key(fitness[i], higher);
    int lo = 0, hi = S;                         // first sorted key not below v
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sorted[mid] < v) lo = mid + 1; else hi = mid;
    }
    const int pct = (int)((100LL * lo) / S);
    const int band = pct >= 90 ? 9 : pct / 10;
    out_band[i] = band * 10;
    if (out_children) out_children[i] = kChildrenByBand[band];
}

}  // namespace

// ================================================================ C ABI
extern "C" {

const char* gp_last_error(void) { return g_last_error.c_str(); }

int gp_version(void) { return GPEVAL_VERSION; }

int gp_validate(const uint32_t* nodes, const int64_t* offsets, int64_t n_programs,
                int64_t n_consts, int32_t n_vars, uint32_t allowed_op_mask,
                int32_t* status, int32_t* max_depth, int64_t* first_bad)
{
    if (n_programs < 0 || n_consts < 0 || n_vars < 0)
        return set_error(GP_E_INVALID_ARG, "negative size");
    if (n_programs > 0 && (!offsets)) return set_error(GP_E_INVALID_ARG, "offsets is NULL");
    const uint32_t allowed = allowed_op_mask ? allowed_op_mask : GP_ALL_OPS;
    int64_t bad_at = -1;
    for (int64_t p = 0; p < n_programs; ++p) {
        const int64_t s = offsets[p], e = offsets[p + 1];
        int st = GP_PROG_OK, md = 0;
        if (s < 0 || e < s) st = GP_PROG_BAD_OFFSETS;
        else if (e == s) st = GP_PROG_EMPTY;
        else if (!nodes) st = GP_PROG_BAD_OFFSETS;
        else {
            GclCheck gc;
            for (int64_t k = s; k < e && st == GP_PROG_OK; ++k)
                st = gc.step(nodes[k] & 0xFFu, nodes[k] >> 8, allowed, n_vars, n_consts);
            if (st == GP_PROG_OK) st = gc.finish();
            md = gc.maxd;
        }
        if (status) status[p] = st;
        if (max_depth) max_depth[p] = md;
        if (st != GP_PROG_OK && bad_at < 0) bad_at = p;
    }
    if (first_bad) *first_bad = bad_at;
    if (bad_at >= 0) return set_error(GP_E_BAD_PROGRAM, "program %lld is invalid", (long long)bad_at);
    return GP_OK;
}

int gp_eval(const uint32_t* nodes, const int64_t* offsets, int64_t n_programs,
            int64_t n_nodes, const float* consts, int64_t n_consts,
            const float* X, int32_t n_vars, int64_t ld_x,
            const float* y, int64_t n_cases,
            double tax_on_length, uint32_t allowed_op_mask,
            double* out_fitness, int32_t* out_status, hipStream_t stream)
{
    const gp_problem d{nodes, offsets, n_programs, n_nodes, consts, n_consts, X, n_vars, ld_x,
                       y, n_cases, tax_on_length, allowed_op_mask, out_fitness, out_status};
    return eval_problem(make_problem(&d), stream);
}

int gp_eval_noalloc(const uint32_t* nodes, const int64_t* offsets, int64_t n_programs,
                    int64_t n_nodes, const float* consts, int64_t n_consts,
                    const float* X, int32_t n_vars, int64_t ld_x,
                    const float* y, int64_t n_cases,
                    double tax_on_length, uint32_t allowed_op_mask,
                    double* out_fitness, int32_t* out_status, hipStream_t stream)
{
    const gp_problem d{nodes, offsets, n_programs, n_nodes, consts, n_consts, X, n_vars, ld_x,
                       y, n_cases, tax_on_length, allowed_op_mask, out_fitness, out_status};
    return eval_problem_noalloc(make_problem(&d), stream);
}

int gp_eval_correlation(const uint32_t* nodes, const int64_t* offsets, int64_t n_programs,
                        int64_t n_nodes, const float* consts, int64_t n_consts,
                        const float* X, int32_t n_vars, int64_t ld_x,
                        const float* y, int64_t n_cases, double max_score,
                        uint32_t allowed_op_mask, double* out_score, int32_t* out_status,
                        hipStream_t stream)
{
    if (!std::isfinite(max_score)) return set_error(GP_E_INVALID_ARG, "max_score is not finite");
    const gp_problem d{nodes, offsets, n_programs, n_nodes, consts, n_consts, X, n_vars, ld_x,
                       y, n_cases, 0.0, allowed_op_mask, out_score, out_status};
    Problem pb = make_problem(&d);
    pb.fit = kFitCorr;
    pb.max_score = max_score;
    return eval_problem(pb, stream);
}

int gp_eval_reward(const uint32_t* nodes, const int64_t* offsets, int64_t n_programs,
                   int64_t n_nodes, const float* consts, int64_t n_consts,
                   const float* X, int32_t n_vars, int64_t ld_x,
                   const float* y, int64_t n_cases, double max_score, int32_t power,
                   uint32_t allowed_op_mask, double* out_reward, int32_t* out_status,
                   hipStream_t stream)
{
    if (!(std::fabs(max_score) <= GP_MAX_REWARD_SCORE) || max_score != std::trunc(max_score))
        return set_error(GP_E_INVALID_ARG, "max_score is not an integer of magnitude <= 2^24");
    if (power != 1 && power != 2 && power != 3 && power != 8)
        return set_error(GP_E_INVALID_ARG, "power %d is not 1, 2, 3 or 8", (int)power);
    const gp_problem d{nodes, offsets, n_programs, n_nodes, consts, n_consts, X, n_vars, ld_x,
                       y, n_cases, 0.0, allowed_op_mask, out_reward, out_status};
    Problem pb = make_problem(&d);
    pb.fit = kFitReward;
    pb.max_score = max_score;
    pb.reward_power = power;
    return eval_problem(pb, stream);
}

int gp_mc_rank(const double* fitness, int64_t n, int32_t higher_is_better, uint64_t seed,
               int32_t sample_size, int32_t* out_band, float* out_children,
               double* out_sample_keys, hipStream_t stream)
{
    if (n < 0) return set_error(GP_E_INVALID_ARG, "n < 0");
    if (sample_size < 1 || sample_size > kMaxRankSample)
        return set_error(GP_E_INVALID_ARG, "sample_size must be 1..%d", kMaxRankSample);
    if (n == 0) return GP_OK;
    if (!fitness || !out_band) return set_error(GP_E_INVALID_ARG, "NULL fitness or out_band");
    double* sorted = out_sample_keys;
    if (!sorted) {
        Workspace* w = nullptr;
        const int rc = get_workspace(stream, (size_t)sample_size * sizeof(double), &w);
        if (rc != GP_OK) return rc;
        sorted = static_cast<double*>(w->ptr);
    }
    const int32_t hb = higher_is_better ? 1 : 0;
    hipLaunchKernelGGL(k_rank_sample, dim3(1), dim3(kMaxRankSample), 0, stream, fitness, n, hb,
                       seed, sample_size, sorted);
    GP_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_rank_assign, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       fitness, n, hb, sample_size, sorted, out_band, out_children);
    GP_HIP_TRY(hipGetLastError());
    return GP_OK;
}

int gp_eval_batched(const gp_request* requests_dev, int32_t n_requests,
                    const gp_dataset* datasets_dev, int32_t n_datasets,
                    int64_t total_programs, int64_t total_nodes,
                    int32_t max_n_vars, int64_t max_n_cases, uint32_t allowed_op_mask,
                    hipStream_t stream)
{
    if (!requests_dev) return set_error(GP_E_INVALID_ARG, "requests_dev is NULL");
    Problem pb{};
    pb.req_dev = requests_dev; pb.n_req = n_requests;
    pb.ds_dev = datasets_dev; pb.n_ds = n_datasets;
    pb.n_programs = total_programs; pb.n_nodes = total_nodes;
    pb.max_vars = max_n_vars; pb.max_cases = max_n_cases;
    pb.allowed = allowed_op_mask ? allowed_op_mask : GP_BASE_OPS;
    pb.need_out = 1;
    return eval_problem(pb, stream);
}

int gp_predict(const uint32_t* nodes, const int64_t* offsets, int64_t n_programs,
               int64_t n_nodes, const float* consts, int64_t n_consts,
               const float* X, int32_t n_vars, int64_t ld_x, int64_t n_cases,
               uint32_t allowed_op_mask, float* out, int64_t ld_out, int32_t* out_status,
               hipStream_t stream)
{
    int rc = check_common(n_programs, n_nodes, n_consts, n_vars, ld_x, n_cases);
    if (rc != GP_OK) return rc;
    if (n_programs == 0) return GP_OK;
    if (!offsets || !out) return set_error(GP_E_INVALID_ARG, "NULL offsets or out");
    if (ld_out < n_cases) return set_error(GP_E_INVALID_ARG, "ld_out < n_cases");
    if ((rc = check_pointers(nodes, n_nodes, consts, n_consts, X, n_vars)) != GP_OK) return rc;
    // work items (program, sub-tile) are counted in 32 bits
    if ((double)n_programs * (double)((n_cases + 511) / 512) > 2.0e9)
        return set_error(GP_E_TOO_LARGE, "n_programs * n_cases too large for one gp_predict call");
    int cus = 0;
    if ((rc = device_cus(&cus)) != GP_OK) return rc;
    Problem pb{};
    pb.one_req.nodes = nodes; pb.one_req.offsets = offsets; pb.one_req.consts = consts;
    pb.one_req.n_programs = n_programs; pb.one_req.n_nodes = n_nodes;
    pb.one_req.n_consts = n_consts; pb.one_req.out_status = out_status;
    pb.n_req = 1;
    pb.one.X = X; pb.one.y = reinterpret_cast<const float*>(out);   // any non-null: unused
    pb.one.ld_x = ld_x; pb.one.n_cases = n_cases; pb.one.tax_on_length = 0.0;
    pb.one.n_vars = n_vars;
    pb.n_ds = 1;
    pb.n_programs = n_programs; pb.n_nodes = n_nodes;
    pb.max_vars = n_vars; pb.max_cases = n_cases;
    pb.allowed = allowed_op_mask ? allowed_op_mask : GP_ALL_OPS;
    pb.need_out = 0;
    const Layout L = make_layout(n_programs, n_nodes, 0, 1, 1);
    Workspace* w = nullptr;
    if ((rc = get_workspace(stream, L.total, &w)) != GP_OK) return rc;
    const Staged st = carve(w->ptr, L);
    if ((rc = enqueue_stage(pb, Tuning(), st, 1, stream)) != GP_OK) return rc;
    EvalPtrs ep{st.code, st.meta, st.order, st.class_info, nullptr, X, nullptr, nullptr, nullptr};
    EvalConst ea{};
    ea.ld_x = ld_x; ea.n_cases = n_cases; ea.n_vars = n_vars;
    for (int c = 0; c < kClasses; ++c) {
        ea.cls = c;
        ep.work_counter = st.counters + c;
        const bool ext = pb_ext(pb.allowed);
        if (c == 0) rc = ext ? launch_predict<8, 4, true>(ep, out, ld_out, ea, stream, cus)
                             : launch_predict<8, 4, false>(ep, out, ld_out, ea, stream, cus);
        else if (c == 1) rc = ext ? launch_predict<16, kK1, true>(ep, out, ld_out, ea, stream, cus)
                                  : launch_predict<16, kK1, false>(ep, out, ld_out, ea, stream, cus);
        else rc = ext ? launch_predict<32, 2, true>(ep, out, ld_out, ea, stream, cus)
                      : launch_predict<32, 2, false>(ep, out, ld_out, ea, stream, cus);
        if (rc != GP_OK) return rc;
    }
    hipLaunchKernelGGL(k_fill_invalid, dim3((unsigned)n_programs), dim3(256), 0, stream, st.cls,
                       n_cases, out, ld_out);
    GP_HIP_TRY(hipGetLastError());
    return GP_OK;
}

int gp_plan_create(gp_plan** plan, const gp_problem* problem, const gp_tuning* tuning,
                   int autotune, hipStream_t stream)
{
    if (!plan || !problem) return set_error(GP_E_INVALID_ARG, "NULL plan or problem");
    *plan = nullptr;
    const Problem pb = make_problem(problem);
    int rc = check_problem(pb);
    if (rc != GP_OK) return rc;
    if (pb.n_programs == 0) return set_error(GP_E_INVALID_ARG, "a plan needs n_programs >= 1");
    gp_plan* p = new gp_plan();
    p->pb = pb;
    if (tuning) {
        if (tuning->programs_per_item < 0 || tuning->programs_per_item > 128 || tuning->wg_per_cu < 0 ||
            tuning->tile_lds_bytes < 0 || (tuning->tile_lds_bytes > 0 && (tuning->tile_lds_bytes < 4096 ||
                                                                         tuning->tile_lds_bytes > 65536)) ||
            tuning->max_tiles < 0 || tuning->max_tiles > kMaxTiles ||
            tuning->concurrent_classes < 0 || tuning->concurrent_classes > 2) {
            delete p;
            return set_error(GP_E_INVALID_ARG, "tuning out of range");
        }
        if (tuning->programs_per_item > 0) p->tu.G = tuning->programs_per_item;
        p->tu.wg_per_cu = tuning->wg_per_cu;
        p->tu.concurrent = tuning->concurrent_classes;
        if (tuning->tile_lds_bytes > 0) p->tu.tile_lds = tuning->tile_lds_bytes;
        if (tuning->max_tiles > 0) p->tu.tile_max = tuning->max_tiles;
    }
    if (hipGetDevice(&p->device) != hipSuccess ||
        hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess ||
        p->side.create() != GP_OK) {
        gp_plan_destroy(p);
        return set_error(GP_E_HIP, "plan stream setup failed");
    }
    // workspace for the largest candidate configuration (the most programs
    // per item and the most tiles per program)
    EvalLaunch el;
    Tuning big = p->tu;
    big.G = 128;
    big.tile_max = kMaxTiles;
    if ((rc = configure_eval(pb, big, &el)) != GP_OK ||
        hipMalloc(&p->ws, el.layout.total) != hipSuccess) {
        (void)hipGetLastError();
        gp_plan_destroy(p);
        return rc != GP_OK ? rc : set_error(GP_E_NO_MEMORY, "plan workspace");
    }
    p->ws_bytes = el.layout.total;
    if (autotune && (rc = plan_autotune(p, stream)) != GP_OK) {
        gp_plan_destroy(p);
        return rc;
    }
    if ((rc = plan_build(p)) != GP_OK) {
        gp_plan_destroy(p);
        return rc;
    }
    *plan = p;
    return GP_OK;
}

int gp_plan_launch(gp_plan* plan, hipStream_t stream)
{
    if (!plan || !plan->exec) return set_error(GP_E_INVALID_ARG, "plan is not built");
    GP_HIP_TRY(hipGraphLaunch(plan->exec, stream));
    return GP_OK;
}

int gp_plan_update(gp_plan* plan, const gp_problem* problem)
{
    if (!plan || !problem) return set_error(GP_E_INVALID_ARG, "NULL plan or problem");
    const Problem pb = make_problem(problem);
    int rc = check_problem(pb);
    if (rc != GP_OK) return rc;
    if (pb.n_programs == 0) return set_error(GP_E_INVALID_ARG, "a plan needs n_programs >= 1");
    plan->pb = pb;
    return plan_build(plan);
}

int gp_plan_get_tuning(const gp_plan* plan, gp_tuning* out)
{
    if (!plan || !out) return set_error(GP_E_INVALID_ARG, "NULL plan or out");
    out->programs_per_item = plan->tu.G;
    out->wg_per_cu = plan->tu.wg_per_cu;
    out->concurrent_classes = plan->tu.concurrent;
    out->tile_lds_bytes = plan->tu.tile_lds;
    out->max_tiles = plan->tu.tile_max;
    return GP_OK;
}

void gp_plan_destroy(gp_plan* plan)
{
    if (!plan) return;
    if (plan->cap) (void)hipStreamSynchronize(plan->cap);
    (void)hipDeviceSynchronize();
    plan_release_graph(plan);
    plan->side.destroy();
    if (plan->cap) (void)hipStreamDestroy(plan->cap);
    if (plan->ws) (void)hipFree(plan->ws);
    delete plan;
}

int gp_timing_enable(int on)
{
    g_timing.on = on != 0;
    return GP_OK;
}

int gp_timing_reset(void)
{
    for (auto& evs : g_timing.pending)
        for (auto& e : evs) (void)hipEventDestroy(e);
    g_timing.pending.clear();
    for (double& m : g_timing.ms) m = 0.0;
    g_timing.calls = 0;
    return GP_OK;
}

int gp_timing_read(double* ms, int64_t* n_calls)
{
    int rc = GP_OK;
    for (auto& evs : g_timing.pending) {
        if (hipEventSynchronize(evs[GP_TIMING_PHASES - 1]) != hipSuccess) {
            rc = set_error(GP_E_HIP, "hipEventSynchronize failed");
            break;
        }
        float t = 0.f;
        for (int i = 0; i + 1 < GP_TIMING_PHASES; ++i) {
            if (hipEventElapsedTime(&t, evs[i], evs[i + 1]) == hipSuccess) g_timing.ms[i] += t;
        }
        if (hipEventElapsedTime(&t, evs[0], evs[GP_TIMING_PHASES - 1]) == hipSuccess)
            g_timing.ms[GP_TIMING_PHASES - 1] += t;
        g_timing.calls += 1;
        for (auto& e : evs) (void)hipEventDestroy(e);
    }
    g_timing.pending.clear();
    if (ms)
        for (int i = 0; i < GP_TIMING_PHASES; ++i) ms[i] = g_timing.ms[i];
    if (n_calls) *n_calls = g_timing.calls;
    return rc;
}

int gp_workspace_size(int64_t n_programs, int64_t n_nodes, int32_t n_requests,
                      int32_t n_datasets, int32_t max_n_vars, int64_t max_n_cases,
                      size_t* bytes)
{
    if (!bytes) return set_error(GP_E_INVALID_ARG, "bytes is NULL");
    if (n_programs < 0 || n_nodes < 0 || n_requests < 1 || n_datasets < 1 || max_n_vars < 0 ||
        max_n_cases < 1)
        return set_error(GP_E_INVALID_ARG, "sizes out of range");
    int32_t stride = 1;
    for (int c = 0; c < kClasses; ++c) {
        const int32_t t = max_tiles(max_n_cases, class_k(c, max_n_vars), kMaxTiles);
        if (t > stride) stride = t;
    }
    const size_t need = make_layout(n_programs, n_nodes, stride, n_datasets, n_requests).total;
    *bytes = need + need / 4;      // the growth slack get_workspace adds
    return GP_OK;
}

}  // extern "C"

// Drops the cached workspace of one stream (the server calls it before it
// destroys its streams).  Not exported.
__attribute__((visibility("hidden"))) void gp_internal_release_stream_workspace(hipStream_t stream)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_ws_mutex);
    auto it = g_ws.find(std::make_pair(dev, stream));
    if (it == g_ws.end()) return;
    (void)hipStreamSynchronize(stream);
    if (it->second.ptr) (void)hipFree(it->second.ptr);
    it->second.side.destroy();
    g_ws.erase(it);
}

extern "C" {

void gp_release_workspaces(void)
{
    std::lock_guard<std::mutex> lk(g_ws_mutex);
    for (auto& kv : g_ws) {
        (void)hipStreamSynchronize(kv.first.second);
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
        kv.second.side.destroy();
    }
    g_ws.clear();
}

}  // extern "C"
