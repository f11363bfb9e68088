// staging.h -- the interpreter's staged program format and the staging
// walk: validation with the instruction count (check_program) and emission
// (stage_walk), and for op masks within the benchmark set both in one
// shorter pass (stage_check_base).  Included by gpeval.hip for the
// device passes (k_validate, k_stage) and by a host test harness, so the
// count, the emission and the meaning of the staged words can be checked
// without a GPU.
//
// The includer provides, before this header: gpeval.h, uint2 and
// make_uint2, __float_as_uint, the LDS float type lds_f32, kHeldConsts and
// kBucketBlock, the folding functions binary_value(op, a, b) and
// unary_value(op, x) for the benchmark set, and GP_STAGING_FN (the
// qualifier of the walks: __device__ in the library).
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
// | (compaction target << 16); the selector says which parts run, in this
// order: tmp = read cell; write cell = top; top = tmp; compaction target =
// compaction source.
constexpr uint32_t kFMove = 16u;
constexpr uint32_t kMvRead = 1u, kMvWrite = 2u, kMvTop = 4u, kMvCompact = 8u;

// Cell numbers (slot fields and move payloads, 5 bits each) do not depend
// on the depth class, so a program is staged before its class is known:
// stack element i is cell i, the held variable q places below the top of
// the cell space is cell 31 - q.  A class of maximum depth MAXD keeps cell
// c at register index (c * J) mod 32 of its 32-float chunks, J = 32 / MAXD:
// element i at i * J, that variable at 32 - J * (q + 1).
// A variable leaf's payload is its input row's byte offset in the
// interpreter's window at four cases per lane (row stride 256 * 4 bytes);
// a class with two cases per lane halves it.
constexpr uint32_t kVarPayload = 1024u;
// The cell written by a push onto an empty stack: no element sits there
// below depth 2, and after a push depth + held variables <= MAXD keeps
// every held variable above it.
constexpr uint32_t kDummyCell = 0u;

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
GP_STAGING_FN int64_t stage_walk(Nodes nodes, int64_t s, int64_t e, Consts consts,
                              uint2* __restrict__ out, int64_t cap, lds_f32* pvs)
{
    // held-back constant i of this thread is pvs[i * kBucketBlock] (LDS:
    // a per-lane index into a register array would become a select chain)
#define pv(i) pvs[(i) * kBucketBlock]
    // never writes past the range k_validate sized (`cap` entries)
    auto put = [&](int64_t i, uint2 v) {
        if (i < cap) out[i] = v;
    };
    // cell of the held variable at position q from the top
    auto vcell = [&](int q) { return 31u - (uint32_t)q; };
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
                const uint32_t wr = rt >= 1 ? (uint32_t)(rt - 1) : kDummyCell;
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
            const uint32_t payload = arg * kVarPayload;
            const uint32_t nx = k + 1 < e ? (nodes(k + 1) & 0xFFu) : 0xFFu;
            const uint32_t wr = rt >= 1 ? (uint32_t)(rt - 1) : kDummyCell;
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
                put(n, staged_word(kFSBin, bop, (uint32_t)(rt - 2), 0u));
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
        const uint32_t wr = rt >= 1 ? (uint32_t)(rt - 1) : kDummyCell;
        if (op == GP_DUP) {
            put(n++, staged_word(kFMove, kMvWrite, 0u, wr));
            ++rt;
        } else if (op == GP_SWAP) {
            const uint32_t c2 = (uint32_t)(rt - 2);
            put(n++, staged_word(kFMove, kMvRead | kMvWrite | kMvTop, c2, c2));
        } else if (op == GP_DEL) {
            // the element below becomes the top; deleting the only element
            // moves nothing
            if (rt >= 2) put(n++, staged_word(kFMove, kMvRead | kMvTop, (uint32_t)(rt - 2), 0u));
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
        const uint32_t wr = rt >= 1 ? (uint32_t)(rt - 1) : kDummyCell;
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
// pass validation, so the walk needs neither the variable discipline nor
// the cell moves, and it validates and emits in one pass: one thread walks
// each program, and the loop body is what the walk costs per node.
//
// Its reader gives, for node k: op(k), the opcode (0xFF for any opcode
// from 32 up), or kOpBadConst for a constant whose index is out of range;
// pay(k), the node's payload word (a
// variable's index, or what cval turns into a constant's value); and
// cval(k, pay(k)), a constant's value (asked for constants in range only).
// The walk reads op(k), pay(k) and op(k + 1) together at each step, so one
// memory round trip serves the step.
constexpr uint32_t kOpBadConst = 0xFEu;

// check_program and stage_walk in one pass, for a mask within
// GP_BASE_OPS: the same checks in the same order (op, operand range,
// underflow, depth at each node, then the final depth), the same maximum
// depth and, for a valid program, the same words, stored to out[0, n) with
// n returned (the staged count).  At most e - s words are stored, whatever
// the program; for an invalid one they mean nothing.  A variable folds the
// operator after it into its own word, so that operator is checked with it.
template <class Reader>
GP_STAGING_FN int64_t stage_check_base(Reader rd, int64_t s, int64_t e, uint32_t allowed,
                                       int32_t n_vars, uint2* __restrict__ out, lds_f32* pvs,
                                       int& status, int& maxd)
{
#define pv(i) pvs[(i) * kBucketBlock]
    int rt = 0, np = 0, md = 0, st = GP_PROG_OK;
    int64_t n = 0;
    // each word is stored as it is made; the last one is stored again at
    // the end, with kFLast
    uint2 last = make_uint2(0u, 0u);
    auto put = [&](uint2 v) {
        out[n] = v;
        last = v;
        ++n;
    };
    // one node's checks at depth d: the last test that fails names the
    // status, so they run from the least to the most important
    auto check = [&](uint32_t oc, uint32_t arg, int d) {
        const uint32_t op = oc == kOpBadConst ? (uint32_t)GP_CONST : oc;
        const bool leaf = op <= GP_CONST;
        const bool bin = op - GP_ADD < 4u;                    // ADD..DIV
        const int need = leaf ? 0 : (bin ? 2 : 1);
        const int eff = leaf ? 1 : (bin ? -1 : 0);
        const bool ok_op = op < 32u && ((allowed >> (op & 31u)) & 1u);
        int code = d + eff > GP_MAX_STACK ? GP_PROG_TOO_DEEP : GP_PROG_OK;
        code = d < need ? GP_PROG_UNDERFLOW : code;
        code = oc == kOpBadConst ? GP_PROG_BAD_CONST : code;
        code = op == GP_LOAD && (int64_t)arg >= (int64_t)n_vars ? GP_PROG_BAD_VAR : code;
        return ok_op ? code : GP_PROG_BAD_OP;
    };
    // held-back constants become runtime elements, bottom up
    auto flush = [&]() {
        for (int i = 0; i < np; ++i) {
            const uint32_t wr = rt >= 1 ? (uint32_t)(rt - 1) : kDummyCell;
            put(staged_word(kFPush | kFConst, 0u, wr, __float_as_uint(pv(i))));
            ++rt;
        }
        np = 0;
    };
    float top = 0.f;                             // pv(np - 1) while np >= 1
    for (int64_t k = s; k < e; ++k) {
        const uint32_t op = rd.op(k);
        const uint32_t pay = rd.pay(k);
        const uint32_t nx = k + 1 < e ? rd.op(k + 1) : 0xFFu;
        const uint32_t arg = op == GP_LOAD ? pay : 0u;
        int code = check(op, arg, rt + np);
        if (code != GP_PROG_OK) {
            st = code;
            break;
        }
        if (op == GP_CONST) {
            if (np == kHeldConsts) flush();
            top = rd.cval(k, pay);
            pv(np) = top;
            ++np;
            md = rt + np > md ? rt + np : md;
        } else if (op == GP_LOAD) {
            flush();
            md = rt + 1 > md ? rt + 1 : md;
            const bool fb = nx - GP_ADD < 4u, fu = nx - GP_SIN < 6u;
            if (fb || fu) {
                // the operator after the variable, at the depth rt + 1 the
                // push left (within the limit, as the push was checked):
                // only its mask bit and, for a binary op, underflow remain
                code = !((allowed >> nx) & 1u) ? GP_PROG_BAD_OP
                                               : (fb && rt == 0 ? GP_PROG_UNDERFLOW : GP_PROG_OK);
                if (code != GP_PROG_OK) {
                    st = code;
                    break;
                }
                ++k;
            }
            const uint32_t payload = arg * kVarPayload;
            const uint32_t wr = rt >= 1 ? (uint32_t)(rt - 1) : kDummyCell;
            if (fb) {
                // top = top OP x: the push and the pop cancel
                put(staged_word(kFLBin, nx - GP_ADD, 0u, payload));
            } else {
                put(staged_word(fu ? kFPush | kFUn : kFPush, fu ? nx - GP_SIN : 0u, wr, payload));
                ++rt;
            }
        } else if (op <= GP_DIV) {
            if (np >= 2) {
                --np;
                top = binary_value(op, pv(np - 1), top);
                pv(np - 1) = top;
            } else if (np == 1) {
                // top = top OP c: the runtime top is the left operand
                np = 0;
                put(staged_word(kFLBin | kFConst, op - GP_ADD, 0u, __float_as_uint(top)));
            } else {
                // second from top (element rt-2) is read from cell rt-2
                put(staged_word(kFSBin, op - GP_ADD, (uint32_t)(rt - 2), 0u));
                --rt;
            }
        } else if (np >= 1) {
            top = unary_value(op, top);
            pv(np - 1) = top;
        } else {
            put(staged_word(kFUn, op - GP_SIN, 0u, 0u));
        }
    }
    if (st == GP_PROG_OK && rt + np != 1) st = GP_PROG_FINAL_DEPTH;
    if (st == GP_PROG_OK) {
        flush();                                 // a constant program: its value is pushed
        out[n - 1] = make_uint2(last.x | kFLast, last.y);
    }
    status = st;
    maxd = md;
    return n;
#undef pv
}
