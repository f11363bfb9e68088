// staging.h -- the interpreter's staged program format and the staging
// walk: validation with the instruction count (check_program) and emission
// (stage_walk), and their short forms for op masks within the benchmark set
// (check_program_base, stage_walk_base).  Included by gpeval.hip for the
// device passes (k_validate, k_stage) and by a host test harness, so the
// count, the emission and the meaning of the staged words can be checked
// without a GPU.
//
// The includer provides, before this header: gpeval.h, uint2 and
// make_uint2, __float_as_uint, the LDS float type lds_f32, kHeldConsts and
// kBucketBlock, the folding functions binary_value(op, a, b) and
// unary_value(op, x) for the benchmark set, and GP_STAGING_FN (the
// qualifier of the two walks: __device__ in the library).
#pragma once

// Staged instruction flags (see k_stage).  A leaf directly followed by a
// binary op folds into "top = top OP leaf"; a leaf directly followed by a
// unary op folds into "save top; top = f(leaf)".  The leaf's load and the
// op still run for every case: only the push/pop and one dispatch go.
constexpr uint32_t kFPush = 1u;
constexpr uint32_t kFUn = 2u;
constexpr uint32_t kFSBin = 4u;
constexpr uint32_t kFLBin = 8u;
constexpr uint32_t kFLast = 0x80000000u;  // the program's last instruction (sign bit)
constexpr uint32_t kFConst = 32u;       // the leaf is a constant
// Cell moves (DUP, SWAP, DEL, COPY, PASTE; full command table only):
// slot field = cell read, payload = cell written | (compaction source << 8)
// | (compaction target << 16), all pre-scaled; the selector says which
// parts run, in this order: tmp = read cell; write cell = top; top = tmp;
// compaction target = compaction source.
constexpr uint32_t kFMove = 16u;
constexpr uint32_t kMvRead = 1u, kMvWrite = 2u, kMvTop = 4u, kMvCompact = 8u;

__host__ __device__ inline uint2 staged_word(uint32_t flags, uint32_t sel, uint32_t slot,
                                             uint32_t payload)
{
    return make_uint2(flags | (sel << 8) | (slot << 16), payload);
}

__host__ __device__ inline int depth_class(int maxd)
{
    return maxd <= 8 ? 0 : (maxd <= 16 ? 1 : 2);
}

// Op kinds of the command table.  Unary selectors: the benchmark set's six
// (SIN..ABS) first, then SQUARE..SQRT_RAW; binary selectors ADD..DIV, POW.
// (bit tables over the 28 opcodes: one shift per test)
constexpr uint32_t kBinaryOps = 0x3Cu | (1u << GP_POW);                    // ADD..DIV, POW
constexpr uint32_t kUnaryOps = 0xFC0u | (((1u << 10) - 1u) << GP_SQUARE);  // SIN..ABS, SQUARE..SQRT_RAW
__host__ __device__ constexpr bool op_is_binary(uint32_t op)
{
    return op < 32u && ((kBinaryOps >> op) & 1u);
}
__host__ __device__ constexpr bool op_is_unary(uint32_t op)
{
    return op < 32u && ((kUnaryOps >> op) & 1u);
}
__host__ __device__ constexpr uint32_t bop_sel(uint32_t op) { return op == GP_POW ? 4u : op - GP_ADD; }
__host__ __device__ constexpr uint32_t uop_sel(uint32_t op)
{
    return op <= GP_ABS ? op - GP_SIN : op - GP_SQUARE + 6u;
}
constexpr uint32_t kUnSquare = 6u;      // first selector beyond the benchmark set
constexpr uint32_t kBinPow = 4u;

// The GCL stack and variable discipline, one node at a time; the host
// validator and the device staging passes share it, so both accept the
// same programs.  Held variables fill the storage cells from the top:
// variable k sits `pos` cells below the top cell; a PASTE frees its cell
// and the variable in the lowest held cell moves into it, so the held
// variables always occupy the top `live` cells.
struct GclCheck {
    int depth = 0, live = 0, maxd = 0;
    uint32_t held = 0u;                 // bit k: variable k holds a value
    uint64_t pos = 0ull;                // 4 bits per variable

    __host__ __device__ int var_pos(uint32_t k) const { return (int)((pos >> (4u * k)) & 15ull); }
    __host__ __device__ void set_pos(uint32_t k, int p)
    {
        pos = (pos & ~(15ull << (4u * k))) | ((uint64_t)p << (4u * k));
    }
    // COPY @k of a free variable: its cell position.
    __host__ __device__ int copy(uint32_t k)
    {
        held |= 1u << k;
        set_pos(k, live);
        return live++;
    }
    // PASTE @k of a held variable: the position of the variable that moves
    // into k's freed cell, or -1.
    __host__ __device__ int paste(uint32_t k)
    {
        const int p = var_pos(k);
        held &= ~(1u << k);
        --live;
        if (p == live) return -1;
        for (uint32_t m = 0; m < GP_GCL_VARS; ++m)
            if (((held >> m) & 1u) && var_pos(m) == live) set_pos(m, p);
        return live;
    }
    // Applies one node; returns its GP_PROG_* status (checks in the order
    // op, operand range, underflow, pairing, depth).
    __host__ __device__ int step(uint32_t op, uint32_t arg, uint32_t allowed, int32_t n_vars,
                                 int64_t n_consts)
    {
        if (op < GP_DUP) {
            // the benchmark set: leaves push, binary ops pop one, unary ops
            // keep the depth
            if (!((allowed >> op) & 1u)) return GP_PROG_BAD_OP;
            if (op == GP_LOAD && (int64_t)arg >= (int64_t)n_vars) return GP_PROG_BAD_VAR;
            if (op == GP_CONST && (int64_t)arg >= n_consts) return GP_PROG_BAD_CONST;
            if (depth < (op <= GP_CONST ? 0 : (op <= GP_DIV ? 2 : 1))) return GP_PROG_UNDERFLOW;
            depth += op <= GP_CONST ? 1 : (op <= GP_DIV ? -1 : 0);
        } else {
            if (op >= GP_N_OPS || !((allowed >> op) & 1u)) return GP_PROG_BAD_OP;
            const int need = op == GP_SWAP || op == GP_POW ? 2 : (op == GP_PASTE ? 0 : 1);
            if (depth < need) return GP_PROG_UNDERFLOW;
            if (op == GP_COPY) {
                if (arg >= GP_GCL_VARS || ((held >> arg) & 1u)) return GP_PROG_BAD_PAIR;
                copy(arg);
            } else if (op == GP_PASTE) {
                if (arg >= GP_GCL_VARS || !((held >> arg) & 1u)) return GP_PROG_BAD_PAIR;
                paste(arg);
            }
            if (op == GP_PASTE || op == GP_DUP) ++depth;
            else if (op == GP_POW || op == GP_DEL) --depth;
        }
        if (depth + live > GP_MAX_STACK) return GP_PROG_TOO_DEEP;
        if (depth + live > maxd) maxd = depth + live;
        return GP_PROG_OK;
    }
    __host__ __device__ int finish() const
    {
        return depth != 1 ? GP_PROG_FINAL_DEPTH : (live != 0 ? GP_PROG_BAD_PAIR : GP_PROG_OK);
    }
};

// Emits the staged instructions of one valid program (k_validate counts
// them with the same rules as it validates).  Constants are held back on a
// shadow stack and folded: an operator whose operands are all held-back
// constants is computed here, once, with the interpreter's own scalar
// arithmetic (the same bits every case would get), and only its value
// travels on.  Held-back constants always sit on top of the runtime stack;
// they are pushed ("flushed") before a variable or a moved cell is pushed
// above them, combined with the runtime top as "top = top OP c", or pushed
// at the end when the whole program is constant.  A variable directly
// followed by an operator folds into it (top OP x, or save + f(x)).  DUP,
// SWAP, DEL, COPY and PASTE become one cell move each (no more instructions
// than nodes); held variables take the cells from the top down (GclCheck).
// What is folded depends only on the node kinds, never on values, so
// counting and emitting agree.
template <class Nodes, class Consts>
GP_STAGING_FN int64_t stage_walk(Nodes nodes, int64_t s, int64_t e, Consts consts, uint32_t J,
                              uint32_t row_bytes, uint2* __restrict__ out, int64_t cap,
                              lds_f32* pvs)
{
    // held-back constant i of this thread is pvs[i * kBucketBlock] (LDS:
    // a per-lane index into a register array would become a select chain)
#define pv(i) pvs[(i) * kBucketBlock]
    // never writes past the range k_validate sized (`cap` entries)
    auto put = [&](int64_t i, uint2 v) {
        if (i < cap) out[i] = v;
    };
    // A push onto an empty stack saves the meaningless old top in cell 0:
    // no element sits there below depth 2, and after a push depth + held
    // variables <= MAXD keeps every held variable above it.
    const uint32_t dummy = 0u;
    // cell (pre-scaled) of the held variable at position q from the top
    auto vcell = [&](int q) { return 32u - J * (uint32_t)(q + 1); };
    GclCheck gc;
    int rt = 0;                                  // runtime stack depth
    int np = 0;                                  // held-back constants
    int64_t n = 0;                               // emitted instructions
    for (int64_t k = s; k < e; ++k) {
        const uint32_t w = nodes(k);
        const uint32_t op = w & 0xFFu, arg = w >> 8;
        // held-back constants become runtime elements, bottom up
        auto flush = [&]() {
            for (int i = 0; i < np; ++i) {
                const uint32_t wr = rt >= 1 ? (uint32_t)(rt - 1) * J : dummy;
                put(n, staged_word(kFPush | kFConst, 0u, wr, __float_as_uint(pv(i))));
                ++n;
                ++rt;
            }
            np = 0;
        };
        // one flush site: before a variable, a move or a command that is
        // not folded (the commands beyond the set; POW over two held
        // constants), and when the held run is full
        if ((op == GP_CONST && np == kHeldConsts) || op == GP_LOAD ||
            (op >= GP_DUP && (op != GP_POW || np >= 2)))
            flush();
        if (op == GP_CONST) {
            pv(np & (kHeldConsts - 1)) = consts(arg);
            ++np;
            continue;
        }
        if (op == GP_LOAD) {
            const uint32_t payload = arg * row_bytes;
            const uint32_t nx = k + 1 < e ? (nodes(k + 1) & 0xFFu) : 0xFFu;
            const uint32_t wr = rt >= 1 ? (uint32_t)(rt - 1) * J : dummy;
            if (op_is_binary(nx)) {
                // top = top OP x (the binary op has a runtime element below)
                put(n, staged_word(kFLBin, bop_sel(nx), 0u, payload));
                ++k;
            } else if (op_is_unary(nx)) {
                put(n, staged_word(kFPush | kFUn, uop_sel(nx), wr, payload));
                ++rt;
                ++k;
            } else {
                put(n, staged_word(kFPush, 0u, wr, payload));
                ++rt;
            }
            ++n;
            continue;
        }
        if (op_is_binary(op)) {
            const uint32_t bop = bop_sel(op);
            if (np >= 2) {
                --np;
                pv(np - 1) = binary_value(op, pv(np - 1), pv(np));
            } else if (np == 1) {
                // top = top OP c: the runtime top is the left operand
                --np;
                put(n, staged_word(kFLBin | kFConst, bop, 0u, __float_as_uint(pv(0))));
                ++n;
            } else {
                // second from top (element rt-2) is read from slot rt-2
                put(n, staged_word(kFSBin, bop, (uint32_t)(rt - 2) * J, 0u));
                ++n;
                --rt;
            }
            continue;
        }
        if (op_is_unary(op)) {
            if (np >= 1) {
                pv(np - 1) = unary_value(op, pv(np - 1));
            } else {
                put(n, staged_word(kFUn, uop_sel(op), 0u, 0u));
                ++n;
            }
            continue;
        }
        // cell moves
        const uint32_t wr = rt >= 1 ? (uint32_t)(rt - 1) * J : dummy;
        if (op == GP_DUP) {
            put(n++, staged_word(kFMove, kMvWrite, 0u, wr));
            ++rt;
        } else if (op == GP_SWAP) {
            const uint32_t c2 = (uint32_t)(rt - 2) * J;
            put(n++, staged_word(kFMove, kMvRead | kMvWrite | kMvTop, c2, c2));
        } else if (op == GP_DEL) {
            // the element below becomes the top; deleting the only element
            // moves nothing
            if (rt >= 2) put(n++, staged_word(kFMove, kMvRead | kMvTop, (uint32_t)(rt - 2) * J, 0u));
            --rt;
        } else if (op == GP_COPY) {
            const int q = gc.copy(arg);
            put(n++, staged_word(kFMove, kMvWrite, 0u, vcell(q)));
        } else {
            // PASTE: the variable becomes the top (the old top saved unless
            // the stack was empty); the lowest held variable moves into the
            // freed cell
            const int q = gc.var_pos(arg);
            const int from = gc.paste(arg);
            uint32_t sel = kMvRead | kMvTop | (rt >= 1 ? kMvWrite : 0u);
            uint32_t pay = wr;
            if (from >= 0) {
                sel |= kMvCompact;
                pay |= (vcell(from) << 8) | (vcell(q) << 16);
            }
            put(n++, staged_word(kFMove, sel, vcell(q), pay));
            ++rt;
        }
    }
    // a constant program: its value is pushed
    for (int i = 0; i < np; ++i) {
        const uint32_t wr = rt >= 1 ? (uint32_t)(rt - 1) * J : dummy;
        put(n, staged_word(kFPush | kFConst, 0u, wr, __float_as_uint(pv(i))));
        ++n;
        ++rt;
    }
    if (n > 0 && n <= cap) out[n - 1].x |= kFLast;
    return n;
#undef pv
}

// Validation of one program (GclCheck: stack and variable discipline,
// operand ranges, allowed ops) and the count of staged instructions, by
// the same rules stage_walk emits them: held-back constants (np), a
// variable folding into the operator after it, one instruction per cell
// move (none for DEL of the only element).
template <class Nodes>
GP_STAGING_FN void check_program(Nodes nodes, int64_t s, int64_t e, uint32_t allowed,
                              int32_t n_vars, int64_t n_consts, int& status, int& maxd,
                              int64_t& n_staged)
{
    GclCheck gc;
    int64_t n_st = 0;
    int np = 0;
    bool taken = false;
    for (int64_t k = s; k < e; ++k) {
        const uint32_t w = nodes(k);
        const uint32_t op = w & 0xFFu, arg = w >> 8;
        const int depth0 = gc.depth;
        status = gc.step(op, arg, allowed, n_vars, n_consts);
        if (status != GP_PROG_OK) break;
        if (op == GP_CONST) {
            if (np == kHeldConsts) { n_st += np; np = 0; }   // pushed, as in staging
            ++np;
        } else if (op == GP_LOAD) {
            n_st += np + 1;                   // flush, then the variable
            np = 0;
            const uint32_t nx = k + 1 < e ? (nodes(k + 1) & 0xFFu) : 0xFFu;
            taken = op_is_binary(nx) || op_is_unary(nx);
        } else if (taken) {
            taken = false;                    // folded into the variable
        } else if (op_is_binary(op)) {
            if (np >= 2 && op == GP_POW) { n_st += np; np = 0; }   // pushed, not folded
            if (np >= 2) --np;
            else if (np == 1) { np = 0; ++n_st; }
            else ++n_st;
        } else if (op_is_unary(op)) {
            if (op > GP_ABS) { n_st += np; np = 0; }               // pushed, not folded
            if (np == 0) ++n_st;
        } else {
            n_st += np;                       // flush, then the cell move
            np = 0;
            if (op != GP_DEL || depth0 >= 2) ++n_st;
        }
    }
    maxd = gc.maxd;
    if (status == GP_PROG_OK) status = gc.finish();
    n_staged = n_st + np;
}


// ------------------------------------------------ the benchmark set alone
// When the op mask stays within GP_BASE_OPS no command beyond the set can
// pass validation, so the walks need neither the variable discipline nor
// the cell moves.  These two take the same decisions as check_program and
// stage_walk for such masks (the host harness compares them word for word)
// with a loop a fraction of the size: one thread walks each program, and
// the loop body is what the walk costs per node.

// check_program for a mask within GP_BASE_OPS: the same checks in the same
// order (op, operand range, underflow, depth), the same count.
template <class Nodes>
GP_STAGING_FN void check_program_base(Nodes nodes, int64_t s, int64_t e, uint32_t allowed,
                                      int32_t n_vars, int64_t n_consts, int& status, int& maxd,
                                      int64_t& n_staged)
{
    // every lane of a wavefront walks a different program, so the step is
    // written as selects (no branch per node kind): all lanes run the same
    // instructions whatever their node is
    int depth = 0, md = 0, np = 0, st = GP_PROG_OK;
    int64_t n_st = 0;
    bool taken = false;
    uint32_t w = s < e ? nodes(s) : 0u;
    for (int64_t k = s; k < e; ++k) {
        const uint32_t op = w & 0xFFu, arg = w >> 8;
        const uint32_t wn = k + 1 < e ? nodes(k + 1) : 0xFFu;   // next word, read early
        const bool leaf = op <= GP_CONST;
        const bool bin = op - GP_ADD < 4u;                        // ADD..DIV
        const bool un = op - GP_SIN < 6u;                         // SIN..ABS
        const int need = leaf ? 0 : (bin ? 2 : 1);
        const int eff = leaf ? 1 : (bin ? -1 : 0);
        const bool ok_op = op < 32u && ((allowed >> (op & 31u)) & 1u);
        // the checks in check_program's order: the first failing one names it
        int code = depth + eff > GP_MAX_STACK ? GP_PROG_TOO_DEEP : GP_PROG_OK;
        code = depth < need ? GP_PROG_UNDERFLOW : code;
        code = op == GP_CONST && (int64_t)arg >= n_consts ? GP_PROG_BAD_CONST : code;
        code = op == GP_LOAD && (int64_t)arg >= (int64_t)n_vars ? GP_PROG_BAD_VAR : code;
        code = ok_op ? code : GP_PROG_BAD_OP;
        if (code != GP_PROG_OK) {
            st = code;
            break;
        }
        depth += eff;
        md = depth > md ? depth : md;
        // staged words, as stage_walk emits them: a full run of held
        // constants is pushed before the next is held; a variable pushes
        // the held ones, then itself; an operator folded into the variable
        // before it adds nothing; a binary op over fewer than two held
        // constants is one word, a unary op on the runtime top is one word
        const bool cst = op == GP_CONST, var = op == GP_LOAD;
        const bool cap = cst && np == kHeldConsts;
        const bool run_bin = bin && !taken, run_un = un && !taken;
        n_st += (cap ? np : 0) + (var ? np + 1 : 0) + (run_bin && np <= 1 ? 1 : 0) +
                (run_un && np == 0 ? 1 : 0);
        np = cst ? (cap ? 1 : np + 1) : (var ? 0 : (run_bin ? (np >= 2 ? np - 1 : 0) : np));
        const uint32_t nx = wn & 0xFFu;
        taken = var && nx >= GP_ADD && nx <= GP_ABS;
        w = wn;
    }
    maxd = md;
    if (st == GP_PROG_OK && depth != 1) st = GP_PROG_FINAL_DEPTH;
    status = st;
    n_staged = n_st + np;
}

// stage_walk for a program that check_program_base accepted.  The reader
// gives op(k), arg(k) (a variable's index) and cval(k) (a constant node's
// value), so the device can hand it node words and constant values already
// gathered into LDS.  Emits the same words as stage_walk.
template <class Reader>
GP_STAGING_FN int64_t stage_walk_base(Reader rd, int64_t s, int64_t e, uint32_t J,
                                      uint32_t row_bytes, uint2* __restrict__ out, int64_t cap,
                                      lds_f32* pvs)
{
#define pv(i) pvs[(i) * kBucketBlock]
    auto put = [&](int64_t i, uint2 v) {
        if (i < cap) out[i] = v;
    };
    int rt = 0, np = 0;
    int64_t n = 0;
    auto flush = [&]() {
        for (int i = 0; i < np; ++i) {
            const uint32_t wr = rt >= 1 ? (uint32_t)(rt - 1) * J : 0u;
            put(n, staged_word(kFPush | kFConst, 0u, wr, __float_as_uint(pv(i))));
            ++n;
            ++rt;
        }
        np = 0;
    };
    for (int64_t k = s; k < e; ++k) {
        const uint32_t op = rd.op(k);
        const uint32_t nx = k + 1 < e ? rd.op(k + 1) : 0xFFu;
        if (op == GP_CONST) {
            if (np == kHeldConsts) flush();
            pv(np) = rd.cval(k);
            ++np;
        } else if (op == GP_LOAD) {
            flush();
            const uint32_t payload = rd.arg(k) * row_bytes;
            const uint32_t wr = rt >= 1 ? (uint32_t)(rt - 1) * J : 0u;
            if (nx >= GP_ADD && nx <= GP_DIV) {
                put(n, staged_word(kFLBin, nx - GP_ADD, 0u, payload));
                ++k;
            } else if (nx >= GP_SIN && nx <= GP_ABS) {
                put(n, staged_word(kFPush | kFUn, nx - GP_SIN, wr, payload));
                ++rt;
                ++k;
            } else {
                put(n, staged_word(kFPush, 0u, wr, payload));
                ++rt;
            }
            ++n;
        } else if (op <= GP_DIV) {
            if (np >= 2) {
                --np;
                pv(np - 1) = binary_value(op, pv(np - 1), pv(np));
            } else if (np == 1) {
                np = 0;
                put(n, staged_word(kFLBin | kFConst, op - GP_ADD, 0u, __float_as_uint(pv(0))));
                ++n;
            } else {
                put(n, staged_word(kFSBin, op - GP_ADD, (uint32_t)(rt - 2) * J, 0u));
                ++n;
                --rt;
            }
        } else if (np >= 1) {
            pv(np - 1) = unary_value(op, pv(np - 1));
        } else {
            put(n, staged_word(kFUn, op - GP_SIN, 0u, 0u));
            ++n;
        }
    }
    flush();
    if (n > 0 && n <= cap) out[n - 1].x |= kFLast;
    return n;
#undef pv
}
