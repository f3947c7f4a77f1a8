// Host-side program codec: genotype <-> postfix, and validation.
//
// Encoding follows Section 3.2 ("Data Structure of Individuals") and Fig. 1:
// the active nodes of a heap-ordered template are written in post-order
// (left subtree, right subtree, node), introns are skipped, constants are
// appended to the constant list in the order the traversal meets them, and the
// program is padded with END to a fixed stride (the padding to L_max that turns
// a population into one dense array).
#include <cstdint>
#include <cstring>
#include <vector>

#include "errors.h"
#include "gpgomea_eval.h"
#include "gpgomea_ops.h"

namespace gg {

std::string& last_error() {
  thread_local std::string msg;
  return msg;
}

static inline int sym_arity(int s) {
  if (s >= GPGOMEA_SYM_ADD && s <= GPGOMEA_SYM_DIV) return 2;
  if (s == GPGOMEA_SYM_POW) return 2;
  if (s >= GPGOMEA_SYM_SIN && s <= GPGOMEA_SYM_LOG) return 1;
  return 0;
}
static inline bool sym_terminal(int s) { return s == GPGOMEA_SYM_CONST || s >= GPGOMEA_SYM_VAR0; }

static inline int slot_depth(int s) {
  int d = 0;
  for (unsigned v = unsigned(s) + 1; v > 1; v >>= 1) ++d;
  return d;
}

// Encode one genotype.  Returns 0 or an E_PROGRAM code (message set).
static int encode_one(const int8_t* g, const float* gc, int T, int height, int8_t* ops, int L_max,
                      float* cs, int C_max, int* out_len, int* out_nc) {
  struct Frame {
    int slot, next;
  };
  std::vector<Frame> st;
  st.reserve(64);
  st.push_back({0, 0});
  int L = 0, C = 0;
  while (!st.empty()) {
    Frame& f = st.back();
    const int sym = g[f.slot];
    const int ar = sym_arity(sym);
    if (ar == 0 && !sym_terminal(sym))
      return fail(GPGOMEA_E_PROGRAM, "active slot %d holds no symbol (%d)", f.slot, sym);
    if (ar > 0 && slot_depth(f.slot) >= height)
      return fail(GPGOMEA_E_PROGRAM, "operator %d is active at leaf slot %d", sym, f.slot);
    if (f.next < ar) {
      const int child = 2 * f.slot + 1 + f.next;
      f.next++;
      if (child >= T) return fail(GPGOMEA_E_PROGRAM, "active slot %d outside the template", child);
      st.push_back({child, 0});
      continue;
    }
    if (L >= L_max) return fail(GPGOMEA_E_PROGRAM, "program longer than L_max=%d", L_max);
    ops[L++] = int8_t(sym);
    if (sym == GPGOMEA_SYM_CONST) {
      if (C >= C_max) return fail(GPGOMEA_E_PROGRAM, "more than C_max=%d constants", C_max);
      std::memcpy(&cs[C++], &gc[f.slot], sizeof(float));  // bit pattern preserved
    }
    st.pop_back();
  }
  *out_len = L;
  *out_nc = C;
  return GPGOMEA_OK;
}

// Parse one postfix program into child links.  kids[2*i], kids[2*i+1] are the
// token indices of token i's operands (-1 if none).  Returns the root token or
// -1 (message set); `nconst` receives the number of constants.
static int parse_one(const int8_t* ops, int L_max, int F, int C_max, std::vector<int>& kids,
                     int* nconst) {
  std::vector<int> st;
  st.reserve(64);
  kids.assign(2 * size_t(L_max), -1);
  int C = 0, t = 0;
  for (; t < L_max; ++t) {
    const int s = ops[t];
    if (s == GPGOMEA_SYM_END) break;
    const int ar = sym_arity(s);
    if (ar == 0) {
      if (s == GPGOMEA_SYM_CONST) {
        if (++C > C_max) return fail(GPGOMEA_E_PROGRAM, "more than C_max=%d constants", C_max), -1;
      } else if (s >= GPGOMEA_SYM_VAR0) {
        if (s - GPGOMEA_SYM_VAR0 >= F) return fail(GPGOMEA_E_PROGRAM, "variable %d >= F=%d", s - GPGOMEA_SYM_VAR0, F), -1;
      } else {
        return fail(GPGOMEA_E_PROGRAM, "unknown symbol %d at token %d", s, t), -1;
      }
    } else {
      if (int(st.size()) < ar) return fail(GPGOMEA_E_PROGRAM, "stack underflow at token %d", t), -1;
      for (int c = ar - 1; c >= 0; --c) {
        kids[2 * size_t(t) + c] = st.back();
        st.pop_back();
      }
    }
    st.push_back(t);
  }
  if (st.size() != 1) return fail(GPGOMEA_E_PROGRAM, "program leaves %d values", int(st.size())), -1;
  *nconst = C;
  return st[0];
}

}  // namespace gg

using namespace gg;

extern "C" int gpgomea_encode(const int8_t* genes, const float* gene_consts, int32_t M, int32_t T,
                              int32_t height, const int8_t* heights, int8_t* ops, int32_t L_max,
                              float* consts, int32_t C_max, int16_t* len, int16_t* nconst,
                              int32_t* bad_index) {
  if (bad_index) *bad_index = -1;
  if (!genes || !gene_consts || !ops || !consts) return fail(GPGOMEA_E_ARG, "NULL pointer");
  if (M < 0 || T < 1 || L_max < 1 || C_max < 0 || L_max > GPGOMEA_MAX_LEN)
    return fail(GPGOMEA_E_SHAPE, "bad shape M=%d T=%d L_max=%d C_max=%d", M, T, L_max, C_max);
  for (int32_t i = 0; i < M; ++i) {
    const int h = heights ? heights[i] : height;
    const int Ti = (1 << (h + 1)) - 1;
    if (h < 0 || h > 8 || Ti > T) {
      if (bad_index) *bad_index = i;
      return fail(GPGOMEA_E_SHAPE, "individual %d: height %d does not fit T=%d", i, h, T);
    }
    int8_t* o = ops + size_t(i) * L_max;
    float* c = consts + size_t(i) * C_max;
    std::memset(o, 0xff, size_t(L_max));
    if (C_max) std::memset(c, 0, size_t(C_max) * sizeof(float));
    int L = 0, C = 0;
    const int rc = encode_one(genes + size_t(i) * T, gene_consts + size_t(i) * T, Ti, h, o, L_max,
                              c, C_max, &L, &C);
    if (rc != GPGOMEA_OK) {
      if (bad_index) *bad_index = i;
      return rc;
    }
    if (len) len[i] = int16_t(L);
    if (nconst) nconst[i] = int16_t(C);
  }
  return GPGOMEA_OK;
}

extern "C" int gpgomea_decode(const int8_t* ops, const float* consts, int32_t M, int32_t L_max,
                              int32_t C_max, int32_t height, int8_t* genes, float* gene_consts,
                              int32_t* bad_index) {
  if (bad_index) *bad_index = -1;
  if (!ops || !consts || !genes || !gene_consts) return fail(GPGOMEA_E_ARG, "NULL pointer");
  if (M < 0 || L_max < 1 || L_max > GPGOMEA_MAX_LEN || C_max < 0 || height < 0 || height > 8)
    return fail(GPGOMEA_E_SHAPE, "bad shape");
  const int T = (1 << (height + 1)) - 1;
  std::vector<int> kids, slot(size_t(L_max), -1), cidx(size_t(L_max), -1), order;
  for (int32_t i = 0; i < M; ++i) {
    const int8_t* o = ops + size_t(i) * L_max;
    int8_t* g = genes + size_t(i) * T;
    float* gc = gene_consts + size_t(i) * T;
    std::memset(g, 0xff, size_t(T));
    std::memset(gc, 0, size_t(T) * sizeof(float));
    int nc = 0;
    const int root = parse_one(o, L_max, GPGOMEA_MAX_FEATURES, C_max, kids, &nc);
    if (root < 0) {
      if (bad_index) *bad_index = i;
      return GPGOMEA_E_PROGRAM;
    }
    // constant ordinals follow token order
    for (int t = 0, c = 0; t <= root; ++t) cidx[t] = (o[t] == GPGOMEA_SYM_CONST) ? c++ : -1;
    // place from the root downwards (a parent's token comes after its operands)
    slot[root] = 0;
    for (int t = root; t >= 0; --t) {
      if (slot[t] < 0) continue;
      const int s = slot[t];
      if (s >= T) {
        if (bad_index) *bad_index = i;
        return fail(GPGOMEA_E_PROGRAM, "individual %d is taller than height %d", i, height);
      }
      g[s] = o[t];
      if (cidx[t] >= 0) std::memcpy(&gc[s], &consts[size_t(i) * C_max + cidx[t]], sizeof(float));
      for (int c = 0; c < 2; ++c) {
        const int k = kids[2 * size_t(t) + c];
        if (k >= 0) slot[k] = 2 * s + 1 + c;
      }
    }
    for (int t = 0; t <= root; ++t) slot[t] = -1;
  }
  return GPGOMEA_OK;
}

extern "C" int gpgomea_validate(const int8_t* ops, int32_t M, int32_t L_max, int32_t C_max,
                                int32_t F, int32_t max_height, int8_t* status_out,
                                int32_t* first_bad) {
  if (first_bad) *first_bad = -1;
  if (!ops) return fail(GPGOMEA_E_ARG, "NULL pointer");
  if (M < 0 || L_max < 1 || L_max > GPGOMEA_MAX_LEN || C_max < 0 || F < 1 ||
      F > GPGOMEA_MAX_FEATURES || max_height < -1)
    return fail(GPGOMEA_E_SHAPE, "bad shape");
  std::vector<int> kids, ht(size_t(L_max), 0);
  int bad = 0;
  std::string keep = last_error();
  for (int32_t i = 0; i < M; ++i) {
    const int8_t* o = ops + size_t(i) * L_max;
    int nc = 0;
    const int root = parse_one(o, L_max, F, C_max, kids, &nc);
    bool ok = root >= 0;
    if (ok && max_height >= 0) {
      // operands precede their operator, so one forward pass gives every height
      for (int t = 0; t <= root; ++t) {
        const int a = kids[2 * size_t(t)], b = kids[2 * size_t(t) + 1];
        ht[t] = a < 0 ? 0 : 1 + (b < 0 ? ht[a] : (ht[a] > ht[b] ? ht[a] : ht[b]));
      }
      ok = ht[root] <= max_height;
    }
    if (status_out) status_out[i] = ok ? 0 : 2;
    if (!ok && first_bad && *first_bad < 0) *first_bad = i;
    bad += !ok;
  }
  last_error() = keep;
  return bad;
}
