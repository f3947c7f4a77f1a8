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
//   hdr[0:5)   op (UOP_*)
//   hdr[5:7)   src kind: 0 none (unary), 1 variable, 2 constant, 3 pop S[slot]
//   hdr[7:9)   load prefix: 0 none, 1 variable, 2 constant (acc <- terminal
//              before the operator runs; used for the first leaf of a subtree)
//   hdr[9]     push acc into S[push slot] before the load
//   hdr[10:14) push slot
//   hdr[14]    adjoint: the acc operand's subtree contains a constant
//   hdr[15]    adjoint: the src operand contains a constant
//   hdr[16:24) src operand: variable index | constant ordinal | pop slot
//   hdr[24:32) load operand: variable index | constant ordinal
// At most one of {src, load} is a constant, so one payload suffices.
#pragma once
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

constexpr uint32_t HDR_PUSH = 1u << 9;
constexpr uint32_t HDR_ADJ_ACC = 1u << 14;
constexpr uint32_t HDR_ADJ_SRC = 1u << 15;

__host__ __device__ constexpr inline uint32_t uop_op(uint32_t h) { return h & 31u; }
__host__ __device__ constexpr inline uint32_t uop_src(uint32_t h) { return (h >> 5) & 3u; }
__host__ __device__ constexpr inline uint32_t uop_load(uint32_t h) { return (h >> 7) & 3u; }
__host__ __device__ constexpr inline uint32_t uop_push_slot(uint32_t h) { return (h >> 10) & 15u; }
__host__ __device__ constexpr inline uint32_t uop_src_arg(uint32_t h) { return (h >> 16) & 255u; }
__host__ __device__ constexpr inline uint32_t uop_load_arg(uint32_t h) { return h >> 24; }

__host__ __device__ constexpr inline uint32_t make_hdr(uint32_t op, uint32_t src, uint32_t srcarg,
                                                       uint32_t load, uint32_t loadarg) {
  return op | (src << 5) | (load << 7) | (srcarg << 16) | (loadarg << 24);
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

// VGPR pairs that hold a program of up to L_max tokens in registers (at most
// L_max + 1 uops including END; lane l of pair e holds uop e*64 + l).
__host__ __device__ constexpr inline int uop_pairs(int L_max) {
  return L_max + 1 <= 64 ? 1 : L_max + 1 <= 128 ? 2 : L_max + 1 <= 256 ? 4 : 8;
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
  int32_t pad;
};

}  // namespace gg
