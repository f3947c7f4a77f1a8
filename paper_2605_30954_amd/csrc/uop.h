// Internal instruction format of the interpreter ("uops").
//
// A postfix program is rewritten on the device, once per call, into a uop
// stream for an accumulator + register-stack machine:
//   * `acc` holds the value of the subtree evaluated last,
//   * S[0..D) hold pending left/right operands (pushed subtrees),
//   * a terminal operand (variable or constant) is folded into the uop of the
//     operator that consumes it, so terminals never occupy a stack slot.
// The operands of each binary node are evaluated in Sethi-Ullman order (the
// operand subtree that needs more stack slots first), which bounds the stack
// depth by the number of binary levels.  Evaluation order does not change any
// result: each subtree is computed by the same operations on the same inputs.
//
// One uop = uint2 {hdr, payload}; payload carries a constant's float bits.
// The header is laid out for the interpreters' scalar dispatch: every
// decision they take is a single-bit test (s_bitcmp + branch), and the
// operand fields need no further decoding.  The END uop's header is exactly
// UOP_END (no flag set), so the loop test is one compare.
//   hdr[0:4)   op (UOP_*)
//   hdr[4]     CHEAP: op is ADD, SUB, RSUB or MUL
//   hdr[5]     PUSHC: the pushed value (PUSH) holds a constant
//   hdr[6]     LDV: load prefix is a variable (acc <- x[var1] before the op)
//   hdr[7]     LDC: load prefix is a constant (acc <- c); the load prefix is
//              the first leaf of a subtree
//   hdr[8]     PUSH: push acc into S[push slot] before the load
//   hdr[9]     TPRE: the src operand is the uop's first variable (x[var1])
//   hdr[10]    SC: the src operand is a constant (the payload)
//   hdr[11]    SP: the src operand pops S[arg2]
//   hdr[12]    TX2: the src operand is a second variable (x[arg2]; LDV is set)
//   The uop reads a variable iff LDV or TPRE is set; var1 is the first one.
//   hdr[13]    adjoint: the acc operand's subtree contains a constant
//   hdr[14]    adjoint: the src operand contains a constant
//   hdr[15:18) push slot
//   hdr[18:24) var1
//   hdr[24:32) arg2: the constant's ordinal (SC or LDC), the src variable
//              when both operands are variables, or the popped slot
// At most one of {src, load} is a constant, so one payload suffices.
#pragma once
#include <cstddef>
#include <cstdint>

namespace gg {

enum UopOp : uint32_t {
  UOP_NOP = 0,  // acc unchanged (a lone terminal program)
  // binary, cheap; src may be a scalar constant
  UOP_ADD = 1,   // acc + src
  UOP_SUB = 2,   // acc - src
  UOP_RSUB = 3,  // src - acc
  UOP_MUL = 4,   // acc * src
  // binary, protected
  UOP_DIV = 5,   // div_p(acc, src)
  UOP_RDIV = 6,  // div_p(src, acc)
  UOP_POW = 7,   // pow_p(acc, src)
  UOP_RPOW = 8,  // pow_p(src, acc)
  // unary on acc
  UOP_SIN = 9,
  UOP_COS = 10,
  UOP_SQ = 11,
  UOP_SQRT = 12,
  UOP_EXP = 13,
  UOP_LOG = 14,
  UOP_END = 15,
  UOP_NUM = 16
};

enum : uint32_t { SRC_NONE = 0, SRC_VAR = 1, SRC_CONST = 2, SRC_POP = 3 };
enum : uint32_t { LD_NONE = 0, LD_VAR = 1, LD_CONST = 2 };

constexpr uint32_t U_CHEAP = 1u << 4;
constexpr uint32_t U_PUSHC = 1u << 5;
constexpr uint32_t U_LDV = 1u << 6;
constexpr uint32_t U_LDC = 1u << 7;
constexpr uint32_t HDR_PUSH = 1u << 8;
constexpr uint32_t U_TPRE = 1u << 9;
constexpr uint32_t U_SC = 1u << 10;
constexpr uint32_t U_SP = 1u << 11;
constexpr uint32_t U_TX2 = 1u << 12;
constexpr uint32_t U_SV = U_TPRE | U_TX2;   // src is a variable
constexpr uint32_t U_V1 = U_LDV | U_TPRE;   // the uop reads a first variable
constexpr uint32_t HDR_ADJ_ACC = 1u << 13;
constexpr uint32_t HDR_ADJ_SRC = 1u << 14;
constexpr uint32_t UOP_END_HDR = uint32_t(UOP_END);

__host__ __device__ constexpr inline uint32_t uop_op(uint32_t h) { return h & 15u; }
__host__ __device__ constexpr inline uint32_t uop_push_slot(uint32_t h) { return (h >> 15) & 7u; }
__host__ __device__ constexpr inline uint32_t uop_var1(uint32_t h) { return (h >> 18) & 63u; }
__host__ __device__ constexpr inline uint32_t uop_arg2(uint32_t h) { return h >> 24; }
__host__ __device__ constexpr inline uint32_t uop_src(uint32_t h) {
  return (h & U_SV) ? SRC_VAR : (h & U_SC) ? SRC_CONST : (h & U_SP) ? SRC_POP : SRC_NONE;
}
__host__ __device__ constexpr inline uint32_t uop_load(uint32_t h) {
  return (h & U_LDV) ? LD_VAR : (h & U_LDC) ? LD_CONST : LD_NONE;
}
// src operand: variable index, constant ordinal or popped slot
__host__ __device__ constexpr inline uint32_t uop_src_arg(uint32_t h) {
  return (h & U_TPRE) ? uop_var1(h) : uop_arg2(h);
}
// load operand: variable index or constant ordinal
__host__ __device__ constexpr inline uint32_t uop_load_arg(uint32_t h) {
  return (h & U_LDV) ? uop_var1(h) : uop_arg2(h);
}

__host__ __device__ constexpr inline uint32_t make_hdr(uint32_t op, uint32_t src, uint32_t srcarg,
                                                       uint32_t load, uint32_t loadarg) {
  const uint32_t flags = (op >= UOP_ADD && op <= UOP_MUL ? U_CHEAP : 0u) |
                         (load == LD_VAR ? U_LDV : 0u) |
                         (load == LD_CONST ? U_LDC : 0u) |
                         (src == SRC_VAR ? (load == LD_VAR ? U_TX2 : U_TPRE) : 0u) |
                         (src == SRC_CONST ? U_SC : 0u) | (src == SRC_POP ? U_SP : 0u);
  const uint32_t var1 = load == LD_VAR ? loadarg : src == SRC_VAR ? srcarg : 0u;
  const uint32_t arg2 = (src == SRC_CONST || src == SRC_POP) ? srcarg
                        : load == LD_CONST                   ? loadarg
                        : (src == SRC_VAR && load == LD_VAR) ? srcarg
                                                             : 0u;
  return op | flags | ((var1 & 63u) << 18) | ((arg2 & 255u) << 24);
}
__host__ __device__ constexpr inline uint32_t with_push(uint32_t h, uint32_t slot, bool has_const) {
  return h | HDR_PUSH | (has_const ? U_PUSHC : 0u) | ((slot & 7u) << 15);
}

// Adjoint tape rule: how many per-row factors a uop stores in the forward
// sweep so that the reverse sweep can propagate adjoints.  d acc-operand is
// needed when that operand's subtree holds a constant and the partial is not
// a constant itself (+, - and a product with a constant factor need no tape);
// d src is needed when the src operand holds a constant.
__host__ __device__ constexpr inline int tape_acc(uint32_t h) {
  return !(h & HDR_ADJ_ACC) ? 0
         : (uop_op(h) == UOP_NOP || uop_op(h) == UOP_ADD || uop_op(h) == UOP_SUB ||
            uop_op(h) == UOP_RSUB)
             ? 0
         : (uop_op(h) == UOP_MUL && uop_src(h) == SRC_CONST) ? 0
                                                             : 1;
}
__host__ __device__ constexpr inline int tape_src(uint32_t h) {
  return !(h & HDR_ADJ_SRC) ? 0
         : (uop_op(h) == UOP_MUL || uop_op(h) == UOP_DIV || uop_op(h) == UOP_RDIV ||
            uop_op(h) == UOP_POW || uop_op(h) == UOP_RPOW)
             ? 1
             : 0;
}

// Per-individual metadata written by the compile kernel.
struct ProgMeta {
  int32_t n_uops;   // including the END uop
  int32_t status;   // 0 ok, 2 malformed
  int32_t slots;    // stack slots needed
  int32_t n_tape;   // adjoint tape entries per row
  int32_t n_const;  // constants used
  int32_t cost;     // estimated VALU work per row (planning)
  float mu;         // shift for the moment sums (mean prediction on the first rows)
  int32_t n_merge;  // uops whose two operands both hold constants
};
// ProgMeta as 32-bit words, for kernels that fetch it one word per lane
constexpr int kMetaWords = 8;
constexpr int kMetaStatus = 1, kMetaNConst = 4, kMetaMu = 6;
static_assert(sizeof(ProgMeta) == kMetaWords * 4, "ProgMeta is 8 words");
static_assert(offsetof(ProgMeta, status) == kMetaStatus * 4 && offsetof(ProgMeta, n_const) == kMetaNConst * 4 &&
                  offsetof(ProgMeta, mu) == kMetaMu * 4,
              "ProgMeta word offsets");

}  // namespace gg
