// gpeval.hip -- gfx950 kernels and C ABI of the batched fitness evaluator.
//
// Path of one gp_eval call (all on the caller's stream):
//   k_prepare        one thread per program: validate (GCL stack discipline,
//                    32-element limit, opcode/operand ranges, allowed ops),
//                    stage each node as 8 bytes {op | read-slot | write-slot,
//                    var index or constant bits}, record length, maximum
//                    depth and depth class.
//   k_class_count /  stable partition of program ids by depth class
//   k_class_scan /   (max depth <= 8, <= 16, <= 32), so each class runs a
//   k_class_scatter  kernel whose register stack is only as deep as needed.
//   k_eval<MAXD,K>   persistent workgroups pull (program group, case tile)
//                    items from an atomic counter; the case tile's inputs
//                    are staged in LDS; each wavefront runs one program at a
//                    time over K cases per lane with the value stack in
//                    VGPRs; residual, scaled square and compensated (TwoSum)
//                    accumulation are fused; wave shuffles then LDS reduce
//                    to one {hi, lo, bad} partial per (program, tile).
//   k_reduce         one thread per program: fp64 sum of its tile partials
//                    in fixed order, unscaling, tax, classification.
//
// Semantics follow the paper's GCL section (RPN stack machine, 32-element
// stack, command table operand order) and the protected-operator readings
// stated in gpeval.h.  One program per wavefront keeps the opcode stream
// wave-uniform (the paper's divergence argument, Sec. "Avoiding Thread
// Divergence", moved from a block to a wavefront).

#include "gpeval.h"

#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
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
constexpr int kMaxTiles = 32;            // case tiles per program (cap)
constexpr uint32_t kNoSlot = 0xFFu;      // staged write slot: nothing to save
constexpr int kBucketBlock = 1024;       // programs per partition block

// Per-program record written by k_prepare.
struct ProgMeta {
    int64_t start;      // first node (original and staged code share it)
    int32_t len;        // node count (the length taxed)
    int32_t slen;       // staged instruction count (<= len)
};
static_assert(sizeof(ProgMeta) == 16, "ProgMeta layout");

// Staged-only opcodes (superinstructions).  A leaf directly followed by a
// binary op folds into "top = top OP leaf"; a leaf directly followed by a
// unary op folds into "save top; top = f(leaf)".  The leaf's load and the
// op still run for every case: only the push/pop and one dispatch go.
constexpr uint32_t kOpBinVar = 12;      // 12..15: ADD..DIV, leaf = X[var]
constexpr uint32_t kOpBinConst = 16;    // 16..19: ADD..DIV, leaf = constant
constexpr uint32_t kOpUnVar = 20;       // 20..25: SIN..ABS of X[var]
constexpr uint32_t kOpUnConst = 26;     // 26..31: SIN..ABS of a constant

__host__ __device__ inline int depth_class(int maxd)
{
    return maxd <= 8 ? 0 : (maxd <= 16 ? 1 : 2);
}

// Cases per lane for a depth class: deeper stacks hold fewer cases per
// lane so that the register stack (MAXD * K VGPRs) stays bounded.  (8 cases
// per lane for the shallow class measured slower on gfx950: occupancy drops
// from 5 to 3 waves per SIMD and LDS input reads are exposed.)  Depends only
// on the class and the dataset, never on the rest of the population.
int class_k(int c, int n_vars)
{
    if (c == 0) return 4;
    return c == 1 ? 4 : 2;
}

// Tile geometry for one class: a tile is `passes` consecutive sub-tiles of
// 256*K cases; a work item covers one tile of G programs.  Up to 32 tiles
// per program keep enough work items for small depth classes (larger
// tiles were measured slower: too few items to fill 256 CUs).  Depends
// only on (n_cases, K), so a program's summation order never depends on
// the rest of the population.
struct TileShape {
    int32_t sub;        // cases per sub-tile (256 * K)
    int32_t passes;     // sub-tiles per tile
    int32_t n_tiles;    // tiles covering n_cases
};

TileShape tile_shape(int64_t n_cases, int k)
{
    TileShape t;
    t.sub = kWG * k;
    int64_t n_sub = (n_cases + t.sub - 1) / t.sub;
    int64_t passes = (n_sub + kMaxTiles - 1) / kMaxTiles;
    if (passes < 1) passes = 1;
    t.passes = (int32_t)passes;
    t.n_tiles = (int32_t)((n_sub + passes - 1) / passes);
    return t;
}

// Power-of-two pre-scale s = 2^-e with 4^e >= n: every scaled partial sum
// of squared residuals is then <= MSE, so it overflows fp32 only when the
// MSE itself is beyond FLT_MAX.
int scale_exponent(int64_t n)
{
    int e = 0;
    while ((int64_t(1) << (2 * e)) < n) ++e;
    return e;
}

// ------------------------------------------------------------- k_prepare
// Stack slots are stored pre-scaled: element `slot` of a class with maximum
// depth MAXD lives at index slot * (32 / MAXD) of each 32-float VGPR chunk,
// so the kernel uses a 5-bit field directly (always inside the chunk).
__host__ __device__ constexpr int class_depth(int c) { return c == 0 ? 8 : (c == 1 ? 16 : 32); }

__global__ __launch_bounds__(256) void k_prepare(
    const uint32_t* __restrict__ nodes, const int64_t* __restrict__ offsets,
    int64_t n_programs, int64_t n_nodes, const float* __restrict__ consts,
    int64_t n_consts, int32_t n_vars, uint32_t allowed,
    uint2* __restrict__ code, ProgMeta* __restrict__ meta,
    uint8_t* __restrict__ cls, int32_t* __restrict__ out_status)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_programs) return;
    const int64_t s = offsets[p], e = offsets[p + 1];
    int status = GP_PROG_OK;
    int depth = 0, maxd = 0;
    // pass 1: validate (GCL stack discipline, operand ranges, allowed ops)
    if (s < 0 || e < s || e > n_nodes || e - s > INT32_MAX) {
        status = GP_PROG_BAD_OFFSETS;
    } else if (e == s) {
        status = GP_PROG_EMPTY;
    } else {
        for (int64_t k = s; k < e; ++k) {
            const uint32_t w = nodes[k];
            const uint32_t op = w & 0xFFu, arg = w >> 8;
            if (op >= GP_N_OPS || !((allowed >> op) & 1u)) { status = GP_PROG_BAD_OP; break; }
            if (op == GP_LOAD && (int64_t)arg >= (int64_t)n_vars) { status = GP_PROG_BAD_VAR; break; }
            if (op == GP_CONST && (int64_t)arg >= n_consts) { status = GP_PROG_BAD_CONST; break; }
            const int need = op <= GP_CONST ? 0 : (op <= GP_DIV ? 2 : 1);
            if (depth < need) { status = GP_PROG_UNDERFLOW; break; }
            depth += op <= GP_CONST ? 1 : (op <= GP_DIV ? -1 : 0);
            if (depth > GP_MAX_STACK) { status = GP_PROG_TOO_DEEP; break; }
            if (depth > maxd) maxd = depth;
        }
        if (status == GP_PROG_OK && depth != 1) status = GP_PROG_FINAL_DEPTH;
    }
    const int c = status == GP_PROG_OK ? depth_class(maxd) : -1;
    // pass 2: stage 8-byte instructions {op | read index << 8 | write index
    // << 16, variable index or constant bits}, folding a leaf into the op
    // that directly follows it
    int64_t sk = s;                              // next staged slot
    if (c >= 0) {
        const uint32_t J = 32u / (uint32_t)class_depth(c);
        const uint32_t dummy = 32u - J;          // slot MAXD-1: never live
        depth = 0;
        for (int64_t k = s; k < e; ++k) {
            const uint32_t w = nodes[k];
            const uint32_t op = w & 0xFFu, arg = w >> 8;
            uint2 cw;
            if (op <= GP_CONST) {
                const uint32_t payload = op == GP_LOAD ? arg : __float_as_uint(consts[arg]);
                // the old top (element depth-1) would move into slot depth-1
                const uint32_t wr = depth >= 1 ? (uint32_t)(depth - 1) * J : dummy;
                const uint32_t nx = k + 1 < e ? (nodes[k + 1] & 0xFFu) : 0xFFu;
                if (depth >= 1 && nx >= GP_ADD && nx <= GP_DIV) {
                    // top = top OP leaf: no push, no pop
                    cw.x = (op == GP_LOAD ? kOpBinVar : kOpBinConst) + (nx - GP_ADD);
                    cw.y = payload;
                    ++k;                         // the binary node is consumed
                } else if (nx >= GP_SIN && nx < GP_N_OPS) {
                    cw.x = ((op == GP_LOAD ? kOpUnVar : kOpUnConst) + (nx - GP_SIN)) | (wr << 16);
                    cw.y = payload;
                    ++depth;
                    ++k;                         // the unary node is consumed
                } else {
                    cw.x = op | (wr << 16);
                    cw.y = payload;
                    ++depth;
                }
            } else if (op <= GP_DIV) {
                // second from top (element depth-2) is read from slot depth-2
                cw.x = op | (((uint32_t)(depth - 2) * J) << 8);
                cw.y = 0;
                --depth;
            } else {
                cw.x = op;
                cw.y = 0;
            }
            code[sk++] = cw;
        }
    }
    ProgMeta m;
    m.start = s;
    m.len = (int32_t)(status == GP_PROG_BAD_OFFSETS ? 0 : e - s);
    m.slen = (int32_t)(sk - s);
    meta[p] = m;
    cls[p] = c >= 0 ? (uint8_t)c : (uint8_t)0xFF;
    if (out_status) out_status[p] = status;
}

// --------------------------------------------------- depth-class partition
// blk_counts[c * n_blk + b] = programs of class c in block b.
__global__ __launch_bounds__(kBucketBlock) void k_class_count(
    const uint8_t* __restrict__ cls, int64_t n_programs, int32_t n_blk,
    int32_t* __restrict__ blk_counts)
{
    __shared__ int cnt[kClasses];
    if (threadIdx.x < kClasses) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * kBucketBlock + threadIdx.x;
    if (p < n_programs) {
        const int c = cls[p];
        if (c < kClasses) atomicAdd(&cnt[c], 1);
    }
    __syncthreads();
    if (threadIdx.x < kClasses) blk_counts[threadIdx.x * n_blk + blockIdx.x] = cnt[threadIdx.x];
}

// One workgroup: exclusive scan of blk_counts in class-major order into
// blk_base; class_info[2c] = first position of class c, [2c+1] = its size;
// also clears the per-class work counters of k_eval.
__global__ __launch_bounds__(1024) void k_class_scan(
    const int32_t* __restrict__ blk_counts, int32_t n_blk,
    int32_t* __restrict__ blk_base, int32_t* __restrict__ class_info,
    uint32_t* __restrict__ work_counters)
{
    __shared__ int part[1024];
    const int total = kClasses * n_blk;
    const int chunk = (total + 1023) / 1024;
    const int t = threadIdx.x;
    const int lo = t * chunk, hi = min(total, lo + chunk);
    int sum = 0;
    for (int i = lo; i < hi; ++i) sum += blk_counts[i];
    part[t] = sum;
    __syncthreads();
    // inclusive Hillis-Steele scan of the 1024 chunk sums
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - sum;
    for (int i = lo; i < hi; ++i) {
        blk_base[i] = run;
        run += blk_counts[i];
    }
    if (t < kClasses) {
        // class t starts after every program of the classes before it
        int start = 0, size = 0;
        for (int i = 0; i < t * n_blk; ++i) start += blk_counts[i];
        for (int i = t * n_blk; i < (t + 1) * n_blk; ++i) size += blk_counts[i];
        class_info[2 * t] = start;
        class_info[2 * t + 1] = size;
        work_counters[t] = 0u;
    }
}

// Stable scatter: order[blk_base[c, b] + rank of p among class-c programs
// of block b] = p.
__global__ __launch_bounds__(kBucketBlock) void k_class_scatter(
    const uint8_t* __restrict__ cls, int64_t n_programs, int32_t n_blk,
    const int32_t* __restrict__ blk_base, int32_t* __restrict__ order)
{
    constexpr int kW = kBucketBlock / 64;
    __shared__ int wcnt[kW][kClasses];
    const int64_t p = (int64_t)blockIdx.x * kBucketBlock + threadIdx.x;
    const int c = p < n_programs ? (int)cls[p] : 0xFF;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int rank = 0;
    for (int cc = 0; cc < kClasses; ++cc) {
        const uint64_t m = __ballot(c == cc);
        if (lane == 0) wcnt[wave][cc] = __popcll(m);
        if (c == cc) rank = __popcll(m & below);
    }
    __syncthreads();
    if (c < kClasses) {
        for (int w = 0; w < wave; ++w) rank += wcnt[w][c];
        order[blk_base[c * n_blk + blockIdx.x] + rank] = (int32_t)p;
    }
}

// ------------------------------------------------------------ evaluation
// Scalars of one class launch (pointers travel as restrict-qualified kernel
// parameters so that uniform loads of programs and metadata become scalar
// memory loads).
struct EvalConst {
    int64_t ld_x;
    int64_t n_cases;
    int32_t cls;
    int32_t n_vars;
    int32_t G;              // programs per work item
    int32_t passes;
    int32_t n_tiles;
    int32_t part_stride;
    float scale;            // 2^-e
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

// ------------------------------------------------------------------ sin/cos
// Constants from gen_sin_poly.py: minimax odd polynomial for sin on
// |r| <= pi/2 + 0.01 (relative error 5.7e-10 before fp32 evaluation) and a
// three-part fp32 split of pi for Cody-Waite reduction.  Measured against
// correctly rounded results: <= 1.75 ulp for |x| <= 2^17, including inputs
// next to multiples of pi; larger or non-finite inputs take the library
// path (which carries a Payne-Hanek reduction).
constexpr float kSinC0 = -1.666666716e-01f;
constexpr float kSinC1 = 8.333351463e-03f;
constexpr float kSinC2 = -1.984328410e-04f;
constexpr float kSinC3 = 2.763883458e-06f;
constexpr float kSinC4 = -2.573010249e-08f;
constexpr float kPiA = 3.141592741e+00f;
constexpr float kPiB = -8.742277657e-08f;
constexpr float kPiC = -3.430249020e-15f;
constexpr float kInvPi = 3.183098733e-01f;
constexpr float kTrigFastLimit = 131072.0f;

// sin(r) for |r| <= pi/2 (+ margin)
__device__ __forceinline__ float sin_poly(float r)
{
    const float u = r * r;
    float q = fmaf(u, kSinC4, kSinC3);
    q = fmaf(u, q, kSinC2);
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

// sin x = (-1)^k sin(x - k pi), k = rint(x / pi)
__device__ __forceinline__ float sin_fast(float x)
{
    const float k = rintf(x * kInvPi);
    const float s = sin_poly(reduce_pi(x, k));
    const int ki = (int)k;
    return __int_as_float(__float_as_int(s) ^ (ki << 31));
}

// cos x = -(-1)^k sin(x - (k + 1/2) pi), k = rint(x / pi - 1/2)
__device__ __forceinline__ float cos_fast(float x)
{
    const float k = rintf(fmaf(x, kInvPi, -0.5f));
    const float s = sin_poly(reduce_pi(x, k + 0.5f));
    const int ki = (int)k;
    return __int_as_float(__float_as_int(s) ^ ((ki + 1) << 31));
}

// --------------------------------------------------------- sqrt|a|, ln|a|
// sqrt|a| with the hardware square root (faithful, <= 1 ulp); magnitudes
// below 2^-100 are scaled by 2^64 first (and the root by 2^-32 after), so
// no denormal reaches the instruction.
__device__ __forceinline__ float sqrt_abs(float a)
{
    const float x = fabsf(a);
    const bool tiny = x < 0x1p-100f;
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

// The value stack below the top lives in VGPR arrays of 32 floats ("chunks"):
// chunk c holds cases [c*J, (c+1)*J) of every slot, element index
// slot*J + (case mod J), J = 32 / MAXD.  A uniform dynamic index into a
// 32-element vector compiles to GPR-index-mode moves (smaller vectors would
// be expanded into compare/select chains).  `ix` is the staged, pre-scaled
// slot index (5 bits, so always inside the chunk).
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
                out[j] = fabsf(b[j]) <= 0.001f ? 1.f : a[j] / b[j];                \
            break;                                                                 \
        }                                                                          \
    } while (0)
#define GP_BINARY(bop, a, top) GP_BINARY_AB(bop, a, top, top)

// Runs one staged program on K cases per lane; xl points at this lane's
// first case of the LDS input tile.  A sub-tile's cases are laid out case-
// major: case j of lane t is element j*256 + t of a variable's row (row
// stride SUB), so each of the K reads of a LOAD is a conflict-free,
// lane-contiguous LDS access.  The top of the stack is returned in tos[].
template <int MAXD, int K, int SUB>
__device__ __forceinline__ void run_program(const uint2* __restrict__ pc,
                                            const uint2* __restrict__ pend,
                                            const float* __restrict__ xl, float (&tos)[K])
{
    constexpr int J = 32 / MAXD;                  // cases per 32-float chunk
    static_assert(K % J == 0 && K / J <= 4, "chunking");
    float c0[32], c1[32], c2[32], c3[32];
#pragma unroll
    for (int j = 0; j < K; ++j) tos[j] = 0.f;

    // the staging buffer has one padding node after the last
    // program, so fetching one node ahead never leaves it
    uint2 w_next = *pc;
    do {
        const uint2 w = w_next;
        ++pc;
        w_next = *pc;
        const uint32_t op = w.x & 0xFFu;
        const uint32_t rd = (w.x >> 8) & 31u;
        const uint32_t wr = (w.x >> 16) & 31u;
        if (op <= GP_CONST) {
            // leaf: the old top moves into the stack (slot MAXD-1
            // never holds a live element, so a push onto an empty
            // stack writes there), the new value becomes the top
#pragma unroll
            for (int j = 0; j < K; ++j) GP_CHUNK_PUT(wr, j, tos[j]);
            if (op == GP_LOAD) {
                const float* xp = xl + (size_t)w.y * SUB;
#pragma unroll
                for (int j = 0; j < K; ++j) tos[j] = xp[j * kWG];
            } else {
                const float c = __uint_as_float(w.y);
#pragma unroll
                for (int j = 0; j < K; ++j) tos[j] = c;
            }
        } else if (op <= GP_DIV) {
            // binary: a = second from top (stack slot rd), b = top
            float sv[K];
#pragma unroll
            for (int j = 0; j < K; ++j) sv[j] = GP_CHUNK_GET(rd, j);
            GP_BINARY(op, sv, tos);
        } else if (op >= kOpBinVar && op < kOpUnVar) {
            // top = top OP leaf
            float lv[K];
            if (op < kOpBinConst) {
                const float* xp = xl + (size_t)w.y * SUB;
#pragma unroll
                for (int j = 0; j < K; ++j) lv[j] = xp[j * kWG];
            } else {
                const float c = __uint_as_float(w.y);
#pragma unroll
                for (int j = 0; j < K; ++j) lv[j] = c;
            }
            const uint32_t bop = GP_ADD + ((op - kOpBinVar) & 3u);
            GP_BINARY_AB(bop, tos, lv, tos);
        } else {
            uint32_t uop = op;
            if (op >= kOpUnVar) {
                // f(leaf): the old top is saved first
#pragma unroll
                for (int j = 0; j < K; ++j) GP_CHUNK_PUT(wr, j, tos[j]);
                if (op < kOpUnConst) {
                    const float* xp = xl + (size_t)w.y * SUB;
#pragma unroll
                    for (int j = 0; j < K; ++j) tos[j] = xp[j * kWG];
                    uop = op - kOpUnVar + GP_SIN;
                } else {
                    const float c = __uint_as_float(w.y);
#pragma unroll
                    for (int j = 0; j < K; ++j) tos[j] = c;
                    uop = op - kOpUnConst + GP_SIN;
                }
            }
            // unary: replaces the top
            switch (uop) {
            case GP_SIN:
            case GP_COS: {
                // fast path for |x| <= 2^17; the library function (with a
                // large-argument reduction) for the rest
                bool big = false;
#pragma unroll
                for (int j = 0; j < K; ++j) big |= !(fabsf(tos[j]) <= kTrigFastLimit);
                if (__builtin_expect(__ballot(big) != 0ull, 0)) {
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        const float x = tos[j];
                        if (fabsf(x) <= kTrigFastLimit)
                            tos[j] = uop == GP_SIN ? sin_fast(x) : cos_fast(x);
                        else
                            tos[j] = uop == GP_SIN ? sinf(x) : cosf(x);
                    }
                } else if (uop == GP_SIN) {
#pragma unroll
                    for (int j = 0; j < K; ++j) tos[j] = sin_fast(tos[j]);
                } else {
#pragma unroll
                    for (int j = 0; j < K; ++j) tos[j] = cos_fast(tos[j]);
                }
                break;
            }
            case GP_EXP:
#pragma unroll
                for (int j = 0; j < K; ++j) tos[j] = expf(tos[j]);
                break;
            case GP_LOG:
#pragma unroll
                for (int j = 0; j < K; ++j) tos[j] = log_protected(tos[j]);
                break;
            case GP_SQRT:
#pragma unroll
                for (int j = 0; j < K; ++j) tos[j] = sqrt_abs(tos[j]);
                break;
            default:
#pragma unroll
                for (int j = 0; j < K; ++j) tos[j] = fabsf(tos[j]);
                break;
            }
        }
    } while (pc != pend);

}

template <int MAXD, int K>
__global__ __launch_bounds__(kWG) void k_eval(
    const uint2* __restrict__ code, const ProgMeta* __restrict__ meta,
    const int32_t* __restrict__ order, const int32_t* __restrict__ class_info,
    uint32_t* __restrict__ work_counter, const float* __restrict__ X,
    const float* __restrict__ y, float2* __restrict__ part,
    uint8_t* __restrict__ part_bad, EvalConst a)
{
    static_assert(K == 2 || K == 4 || K == 8, "cases per lane");
    static_assert(MAXD == 8 || MAXD == 16 || MAXD == 32, "stack class");
    constexpr int J = 32 / MAXD;                  // cases per 32-float chunk
    static_assert(K % J == 0 && K / J <= 4, "chunking");
    constexpr int SUB = kWG * K;                  // cases per sub-tile
    extern __shared__ float lds[];
    float* xt = lds;                              // [n_vars][SUB]
    float2* wpart = reinterpret_cast<float2*>(lds + (size_t)a.n_vars * SUB);  // [G][kWaves]
    uint32_t* wbad = reinterpret_cast<uint32_t*>(wpart + a.G * kWaves);        // [G]
    __shared__ uint32_t s_item;

    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int lo = tid;                           // this lane's first case in a sub-tile
    const int start = class_info[2 * a.cls];
    const int count = class_info[2 * a.cls + 1];
    const int n_groups = (count + a.G - 1) / a.G;
    const uint32_t n_items = (uint32_t)n_groups * (uint32_t)a.n_tiles;
    int64_t staged = -1;                          // sub-tile currently in LDS

    for (;;) {
        if (tid == 0) s_item = atomicAdd(work_counter, 1u);
        if (tid < a.G) wbad[tid] = 0u;
        __syncthreads();
        const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= n_items) break;
        const int tile = (int)(item / (uint32_t)n_groups);
        const int grp = (int)(item % (uint32_t)n_groups);
        const int g0 = grp * a.G;
        const int gn = min(a.G, count - g0);

        for (int pass = 0; pass < a.passes; ++pass) {
            const int64_t sub_idx = (int64_t)tile * a.passes + pass;
            const int64_t base = sub_idx * SUB;
            if (base >= a.n_cases) break;
            if (sub_idx != staged) {
                __syncthreads();
                for (int i = tid; i < a.n_vars * SUB; i += kWG) {
                    const int v = i / SUB, c = i - v * SUB;
                    const int64_t gi = base + c;
                    xt[i] = gi < a.n_cases ? X[(int64_t)v * a.ld_x + gi] : 0.f;
                }
                staged = sub_idx;
                __syncthreads();
            }
            float yv[K];
            bool live[K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int64_t gi = base + lo + j * kWG;
                live[j] = gi < a.n_cases;
                yv[j] = live[j] ? y[gi] : 0.f;
            }

            for (int g = 0; g < gn; ++g) {
                const int pid = order[start + g0 + g];
                const ProgMeta m = meta[pid];
                float tos[K];
                run_program<MAXD, K, SUB>(code + m.start, code + m.start + m.slen, xt + lo, tos);

                // fused residual, validity and scaled compensated square sum
                float hi = 0.f, lo_ = 0.f;
                bool bad = false;
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    if (live[j]) {
                        const float f = tos[j];
                        bad |= !__builtin_isfinite(f);
                        const float r = (f - yv[j]) * a.scale;
                        float s, e;
                        two_sum(hi, r * r, s, e);
                        hi = s;
                        lo_ += e;
                    }
                }
                // wavefront tree: every lane ends with the same pair
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) {
                    const float h2 = __shfl_xor(hi, off);
                    const float l2 = __shfl_xor(lo_, off);
                    acc_pair(hi, lo_, h2, l2);
                }
                const bool wave_bad = __ballot(bad) != 0ull;
                if (lane == 0) {
                    float2 v = make_float2(hi, lo_);
                    if (pass > 0) {
                        float2 o = wpart[g * kWaves + wave];
                        float h = o.x, l = o.y;
                        acc_pair(h, l, v.x, v.y);
                        v = make_float2(h, l);
                    }
                    wpart[g * kWaves + wave] = v;
                }
                if (wave_bad && lane == 0) atomicOr(&wbad[g], 1u);
            }
            __syncthreads();
        }
        // combine the wavefronts in fixed order and store the tile partial
        if (tid < gn) {
            const int pid = order[start + g0 + tid];
            float h = wpart[tid * kWaves].x, l = wpart[tid * kWaves].y;
#pragma unroll
            for (int w = 1; w < kWaves; ++w) acc_pair(h, l, wpart[tid * kWaves + w].x, wpart[tid * kWaves + w].y);
            const int64_t slot = (int64_t)pid * a.part_stride + tile;
            part[slot] = make_float2(h, l);
            part_bad[slot] = (uint8_t)(wbad[tid] != 0u);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ k_predict
// Per-case outputs f_p(x_i) of the programs of one depth class: persistent
// workgroups pull (program, sub-tile) items; each lane writes its K values.
template <int MAXD, int K>
__global__ __launch_bounds__(kWG) void k_predict(
    const uint2* __restrict__ code, const ProgMeta* __restrict__ meta,
    const int32_t* __restrict__ order, const int32_t* __restrict__ class_info,
    uint32_t* __restrict__ work_counter, const float* __restrict__ X,
    float* __restrict__ out, int64_t ld_out, EvalConst a)
{
    constexpr int SUB = kWG * K;
    extern __shared__ float lds[];
    float* xt = lds;                              // [n_vars][SUB]
    __shared__ uint32_t s_item;
    const int tid = threadIdx.x;
    const int lo = tid;
    const int start = class_info[2 * a.cls];
    const int count = class_info[2 * a.cls + 1];
    const int64_t n_sub = (a.n_cases + SUB - 1) / SUB;
    const uint64_t n_items = (uint64_t)count * (uint64_t)n_sub;
    int64_t staged = -1;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(work_counter, 1u);
        __syncthreads();
        const uint64_t item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (item >= n_items) break;
        const int64_t sub = (int64_t)(item / (uint64_t)count);
        const int g = (int)(item % (uint64_t)count);
        const int64_t base = sub * SUB;
        if (sub != staged) {
            for (int i = tid; i < a.n_vars * SUB; i += kWG) {
                const int v = i / SUB, c = i - v * SUB;
                const int64_t gi = base + c;
                xt[i] = gi < a.n_cases ? X[(int64_t)v * a.ld_x + gi] : 0.f;
            }
            staged = sub;
            __syncthreads();
        }
        const int pid = order[start + g];
        const ProgMeta m = meta[pid];
        float tos[K];
        run_program<MAXD, K, SUB>(code + m.start, code + m.start + m.slen, xt + lo, tos);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int64_t gi = base + lo + j * kWG;
            if (gi < a.n_cases) out[(int64_t)pid * ld_out + gi] = tos[j];
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
    if (cls[p] < kClasses) return;
    for (int64_t i = threadIdx.x; i < n_cases; i += 256) out[p * ld_out + i] = __builtin_nanf("");
}

// ------------------------------------------------------------ k_reduce
struct ReduceArgs {
    const ProgMeta* meta;
    const uint8_t* cls;
    const float2* part;
    const uint8_t* part_bad;
    double* out;
    int64_t n_programs;
    int32_t part_stride;
    int32_t n_tiles[kClasses];
    double unscale;         // 4^e / n_cases
    double tax;
};

__global__ __launch_bounds__(256) void k_reduce(ReduceArgs a)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n_programs) return;
    const int c = a.cls[p];
    if (c >= kClasses) { a.out[p] = __builtin_nan(""); return; }
    const ProgMeta m = a.meta[p];
    const int nt = a.n_tiles[c];
    double s = 0.0;
    bool bad = false;
    for (int t = 0; t < nt; ++t) {
        const float2 v = a.part[p * a.part_stride + t];
        s += (double)v.x + (double)v.y;
        bad |= a.part_bad[p * a.part_stride + t] != 0;
    }
    const double mse = s * a.unscale;
    a.out[p] = (bad || !(mse <= (double)FLT_MAX)) ? __builtin_inf() : mse + a.tax * (double)m.len;
}

// ----------------------------------------------------------- workspaces
struct Workspace {
    void* ptr = nullptr;
    size_t bytes = 0;
};

std::mutex g_ws_mutex;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

struct Layout {
    size_t code, meta, cls, order, blk_counts, blk_base, class_info, counters, part, part_bad, total;
};

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

Layout make_layout(int64_t n_programs, int64_t n_nodes, int32_t part_stride)
{
    Layout L;
    const int64_t n_blk = (n_programs + kBucketBlock - 1) / kBucketBlock;
    size_t off = 0;
    L.code = off;       off = align_up(off + (size_t)(n_nodes + 1) * sizeof(uint2));
    L.meta = off;       off = align_up(off + (size_t)n_programs * sizeof(ProgMeta));
    L.cls = off;        off = align_up(off + (size_t)n_programs);
    L.order = off;      off = align_up(off + (size_t)n_programs * 4);
    L.blk_counts = off; off = align_up(off + (size_t)kClasses * n_blk * 4);
    L.blk_base = off;   off = align_up(off + (size_t)kClasses * n_blk * 4);
    L.class_info = off; off = align_up(off + 2 * kClasses * 4);
    L.counters = off;   off = align_up(off + kClasses * 4);
    L.part = off;       off = align_up(off + (size_t)n_programs * part_stride * sizeof(float2));
    L.part_bad = off;   off = align_up(off + (size_t)n_programs * part_stride);
    L.total = off;
    return L;
}

int get_workspace(hipStream_t stream, size_t bytes, void** out)
{
    int dev = 0;
    GP_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_ws_mutex);
    Workspace& w = g_ws[std::make_pair(dev, stream)];
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
    *out = w.ptr;
    return GP_OK;
}

struct DeviceInfo {
    int cus = 0;
    int occ[kClasses] = {0, 0, 0};
};
std::mutex g_dev_mutex;
std::map<int, DeviceInfo> g_dev;

template <int MAXD, int K>
size_t eval_lds_bytes(int n_vars, int G)
{
    return (size_t)n_vars * kWG * K * sizeof(float) + (size_t)G * kWaves * sizeof(float2) +
           (size_t)G * sizeof(uint32_t);
}

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
int launch_eval(const EvalPtrs& p, const EvalConst& args, hipStream_t stream, int cus)
{
    const size_t lds = eval_lds_bytes<MAXD, K>(args.n_vars, args.G);
    if (lds > 64 * 1024) {
        GP_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_eval<MAXD, K>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    }
    int per_cu = 0;
    GP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_eval<MAXD, K>, kWG, lds));
    if (per_cu < 1) return set_error(GP_E_TOO_LARGE, "n_vars=%d needs %zu bytes of LDS per workgroup", args.n_vars, lds);
    const int grid = cus * per_cu;
    hipLaunchKernelGGL((k_eval<MAXD, K>), dim3(grid), dim3(kWG), lds, stream, p.code, p.meta,
                       p.order, p.class_info, p.work_counter, p.X, p.y, p.part, p.part_bad, args);
    GP_HIP_TRY(hipGetLastError());
    return GP_OK;
}

// ---------------------------------------------------------------- timing
struct Timing {
    bool on = false;
    // events of calls not yet read: kPhases + 1 boundaries per call
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
    int begin()
    {
        on = g_timing.on;
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

template <int MAXD, int K>
int launch_predict(const EvalPtrs& p, float* out, int64_t ld_out, const EvalConst& args,
                   hipStream_t stream, int cus)
{
    const size_t lds = (size_t)args.n_vars * kWG * K * sizeof(float);
    if (lds > 64 * 1024) {
        GP_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_predict<MAXD, K>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    }
    int per_cu = 0;
    GP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_predict<MAXD, K>, kWG, lds));
    if (per_cu < 1) return set_error(GP_E_TOO_LARGE, "n_vars=%d needs %zu bytes of LDS per workgroup", args.n_vars, lds);
    hipLaunchKernelGGL((k_predict<MAXD, K>), dim3(cus * per_cu), dim3(kWG), lds, stream, p.code,
                       p.meta, p.order, p.class_info, p.work_counter, p.X, out, ld_out, args);
    GP_HIP_TRY(hipGetLastError());
    return GP_OK;
}

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

// Device views of one call's workspace.
struct Staged {
    uint2* code;
    ProgMeta* meta;
    uint8_t* cls;
    int32_t* order;
    int32_t* class_info;
    uint32_t* counters;
    float2* part;
    uint8_t* part_bad;
};

// Validation, staging and the stable depth-class partition, on `stream`.
int stage_population(const uint32_t* nodes, const int64_t* offsets, int64_t n_programs,
                     int64_t n_nodes, const float* consts, int64_t n_consts, int32_t n_vars,
                     uint32_t allowed_op_mask, int32_t* out_status, int32_t part_stride,
                     hipStream_t stream, Staged* st)
{
    const uint32_t allowed = allowed_op_mask ? allowed_op_mask : GP_ALL_OPS;
    const Layout L = make_layout(n_programs, n_nodes, part_stride);
    void* wsv = nullptr;
    int rc = get_workspace(stream, L.total, &wsv);
    if (rc != GP_OK) return rc;
    char* ws = static_cast<char*>(wsv);
    st->code = reinterpret_cast<uint2*>(ws + L.code);
    st->meta = reinterpret_cast<ProgMeta*>(ws + L.meta);
    st->cls = reinterpret_cast<uint8_t*>(ws + L.cls);
    st->order = reinterpret_cast<int32_t*>(ws + L.order);
    int32_t* blk_counts = reinterpret_cast<int32_t*>(ws + L.blk_counts);
    int32_t* blk_base = reinterpret_cast<int32_t*>(ws + L.blk_base);
    st->class_info = reinterpret_cast<int32_t*>(ws + L.class_info);
    st->counters = reinterpret_cast<uint32_t*>(ws + L.counters);
    st->part = reinterpret_cast<float2*>(ws + L.part);
    st->part_bad = reinterpret_cast<uint8_t*>(ws + L.part_bad);

    const int32_t n_blk = (int32_t)((n_programs + kBucketBlock - 1) / kBucketBlock);
    const unsigned grid_p = (unsigned)((n_programs + 255) / 256);
    hipLaunchKernelGGL(k_prepare, dim3(grid_p), dim3(256), 0, stream, nodes, offsets, n_programs,
                       n_nodes, consts, n_consts, n_vars, allowed, st->code, st->meta, st->cls,
                       out_status);
    GP_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_class_count, dim3(n_blk), dim3(kBucketBlock), 0, stream, st->cls,
                       n_programs, n_blk, blk_counts);
    GP_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_class_scan, dim3(1), dim3(1024), 0, stream, blk_counts, n_blk, blk_base,
                       st->class_info, st->counters);
    GP_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_class_scatter, dim3(n_blk), dim3(kBucketBlock), 0, stream, st->cls,
                       n_programs, n_blk, blk_base, st->order);
    GP_HIP_TRY(hipGetLastError());
    return GP_OK;
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
        int st = GP_PROG_OK, depth = 0, md = 0;
        if (s < 0 || e < s) st = GP_PROG_BAD_OFFSETS;
        else if (e == s) st = GP_PROG_EMPTY;
        else if (!nodes) st = GP_PROG_BAD_OFFSETS;
        else {
            for (int64_t k = s; k < e; ++k) {
                const uint32_t op = nodes[k] & 0xFFu, arg = nodes[k] >> 8;
                if (op >= GP_N_OPS || !((allowed >> op) & 1u)) { st = GP_PROG_BAD_OP; break; }
                if (op == GP_LOAD && (int64_t)arg >= (int64_t)n_vars) { st = GP_PROG_BAD_VAR; break; }
                if (op == GP_CONST && (int64_t)arg >= n_consts) { st = GP_PROG_BAD_CONST; break; }
                const int need = op <= GP_CONST ? 0 : (op <= GP_DIV ? 2 : 1);
                const int delta = op <= GP_CONST ? 1 : (op <= GP_DIV ? -1 : 0);
                if (depth < need) { st = GP_PROG_UNDERFLOW; break; }
                depth += delta;
                if (depth > GP_MAX_STACK) { st = GP_PROG_TOO_DEEP; break; }
                if (depth > md) md = depth;
            }
            if (st == GP_PROG_OK && depth != 1) st = GP_PROG_FINAL_DEPTH;
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
    int rc = check_common(n_programs, n_nodes, n_consts, n_vars, ld_x, n_cases);
    if (rc != GP_OK) return rc;
    if (n_programs == 0) return GP_OK;
    if (!offsets || !out_fitness || !y) return set_error(GP_E_INVALID_ARG, "NULL offsets, y or out_fitness");
    if ((rc = check_pointers(nodes, n_nodes, consts, n_consts, X, n_vars)) != GP_OK) return rc;
    if (!std::isfinite(tax_on_length)) return set_error(GP_E_INVALID_ARG, "tax_on_length is not finite");

    int cus = 0;
    if ((rc = device_cus(&cus)) != GP_OK) return rc;
    TileShape ts[kClasses];
    int32_t stride = 1;
    for (int c = 0; c < kClasses; ++c) {
        ts[c] = tile_shape(n_cases, class_k(c, n_vars));
        if (ts[c].n_tiles > stride) stride = ts[c].n_tiles;
    }
    CallEvents ce;
    if ((rc = ce.begin()) != GP_OK) return rc;
    if ((rc = ce.mark(0, stream)) != GP_OK) return rc;
    Staged st;
    rc = stage_population(nodes, offsets, n_programs, n_nodes, consts, n_consts, n_vars,
                          allowed_op_mask, out_status, stride, stream, &st);
    if (rc != GP_OK) return rc;

    const int e = scale_exponent(n_cases);
    EvalPtrs ep{st.code, st.meta, st.order, st.class_info, nullptr, X, y, st.part, st.part_bad};
    EvalConst ea{};
    ea.ld_x = ld_x; ea.n_cases = n_cases; ea.n_vars = n_vars; ea.G = 8;
    ea.part_stride = stride;
    ea.scale = ldexpf(1.0f, -e);
    for (int c = 0; c < kClasses; ++c) {
        if ((rc = ce.mark(1 + c, stream)) != GP_OK) return rc;
        ea.cls = c;
        ep.work_counter = st.counters + c;
        ea.passes = ts[c].passes;
        ea.n_tiles = ts[c].n_tiles;
        if (c == 0) rc = launch_eval<8, 4>(ep, ea, stream, cus);
        else if (c == 1) rc = launch_eval<16, 4>(ep, ea, stream, cus);
        else rc = launch_eval<32, 2>(ep, ea, stream, cus);
        if (rc != GP_OK) return rc;
    }

    ReduceArgs ra{};
    ra.meta = st.meta; ra.cls = st.cls; ra.part = st.part; ra.part_bad = st.part_bad;
    ra.out = out_fitness;
    ra.n_programs = n_programs; ra.part_stride = stride;
    for (int c = 0; c < kClasses; ++c) ra.n_tiles[c] = ts[c].n_tiles;
    ra.unscale = ldexp(1.0, 2 * e) / (double)n_cases;
    ra.tax = tax_on_length;
    if ((rc = ce.mark(4, stream)) != GP_OK) return rc;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((n_programs + 255) / 256)), dim3(256), 0, stream, ra);
    GP_HIP_TRY(hipGetLastError());
    if ((rc = ce.mark(5, stream)) != GP_OK) return rc;
    ce.commit();
    return GP_OK;
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
    Staged st;
    rc = stage_population(nodes, offsets, n_programs, n_nodes, consts, n_consts, n_vars,
                          allowed_op_mask, out_status, 0, stream, &st);
    if (rc != GP_OK) return rc;
    EvalPtrs ep{st.code, st.meta, st.order, st.class_info, nullptr, X, nullptr, nullptr, nullptr};
    EvalConst ea{};
    ea.ld_x = ld_x; ea.n_cases = n_cases; ea.n_vars = n_vars;
    for (int c = 0; c < kClasses; ++c) {
        ea.cls = c;
        ep.work_counter = st.counters + c;
        if (c == 0) rc = launch_predict<8, 4>(ep, out, ld_out, ea, stream, cus);
        else if (c == 1) rc = launch_predict<16, 4>(ep, out, ld_out, ea, stream, cus);
        else rc = launch_predict<32, 2>(ep, out, ld_out, ea, stream, cus);
        if (rc != GP_OK) return rc;
    }
    hipLaunchKernelGGL(k_fill_invalid, dim3((unsigned)n_programs), dim3(256), 0, stream, st.cls,
                       n_cases, out, ld_out);
    GP_HIP_TRY(hipGetLastError());
    return GP_OK;
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

void gp_release_workspaces(void)
{
    std::lock_guard<std::mutex> lk(g_ws_mutex);
    for (auto& kv : g_ws) {
        if (kv.second.ptr) {
            (void)hipStreamSynchronize(kv.first.second);
            (void)hipFree(kv.second.ptr);
        }
    }
    g_ws.clear();
}

}  // extern "C"
