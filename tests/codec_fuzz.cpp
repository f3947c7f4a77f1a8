// Host-side exercise of the library's codec (csrc/codec.cpp) for a build with
// AddressSanitizer and UndefinedBehaviorSanitizer: seeded random genotypes
// (valid ones, and ones with unknown symbols, active operators at leaf slots,
// too many constants), encode -> decode -> encode round trips, and random
// byte programs through validate.  Built and run by tests/test_codec_sanitizers.py
// with g++; prints "ok <cases>" and exits 0, or reports the first mismatch.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "gpgomea_eval.h"
#include "gpgomea_ops.h"

int main() {
  std::mt19937_64 rng(12345);
  auto uni = [&](int lo, int hi) { return int(lo + rng() % uint64_t(hi - lo + 1)); };
  long cases = 0, trips = 0;
  for (int it = 0; it < 4000; ++it) {
    const int H = uni(0, 8), T = (1 << (H + 1)) - 1, M = uni(1, 6);
    const int F = uni(1, 12), L_max = uni(1, GPGOMEA_MAX_LEN), C_max = uni(0, GPGOMEA_MAX_CONSTS);
    std::vector<int8_t> genes(size_t(M) * T), heights(M);
    std::vector<float> gc(size_t(M) * T);
    const bool mixed = uni(0, 1);
    for (int i = 0; i < M; ++i) {
      heights[i] = int8_t(mixed ? uni(0, H) : H);
      for (int s = 0; s < T; ++s) {
        const int r = uni(0, 99);
        int8_t g;
        if (r < 45) g = int8_t(uni(0, GPGOMEA_NUM_OPS - 1));
        else if (r < 70) g = int8_t(GPGOMEA_SYM_CONST);
        else if (r < 97) g = int8_t(GPGOMEA_SYM_VAR0 + uni(0, F - 1));
        else g = int8_t(uni(-128, 127));  // anything, valid or not
        genes[size_t(i) * T + s] = g;
        gc[size_t(i) * T + s] = float(uni(-1000, 1000)) / 7.0f;
      }
    }
    std::vector<int8_t> ops(size_t(M) * L_max);
    std::vector<float> cs(size_t(M) * (C_max > 0 ? C_max : 1));
    std::vector<int16_t> len(M), nc(M);
    int32_t bad = -2;
    const int rc = gpgomea_encode(genes.data(), gc.data(), M, T, mixed ? 0 : H, mixed ? heights.data() : nullptr,
                                  ops.data(), L_max, cs.data(), C_max, len.data(), nc.data(), &bad);
    ++cases;
    if (rc == GPGOMEA_OK && !mixed) {
      // round trip: decode to a fresh template, encode again, same program
      std::vector<int8_t> g2(size_t(M) * T);
      std::vector<float> c2(size_t(M) * T);
      int32_t bad2 = -2;
      const int rd = gpgomea_decode(ops.data(), cs.data(), M, L_max, C_max, H, g2.data(), c2.data(), &bad2);
      if (rd == GPGOMEA_OK) {
        ++trips;
        std::vector<int8_t> ops2(size_t(M) * L_max);
        std::vector<float> cs2(cs.size());
        std::vector<int16_t> len2(M), nc2(M);
        const int re = gpgomea_encode(g2.data(), c2.data(), M, T, H, nullptr, ops2.data(), L_max, cs2.data(),
                                      C_max, len2.data(), nc2.data(), &bad2);
        if (re != GPGOMEA_OK || ops2 != ops || std::memcmp(cs2.data(), cs.data(), cs.size() * 4) != 0 ||
            len2 != len || nc2 != nc) {
          std::printf("round trip mismatch at case %d\n", it);
          return 1;
        }
      }
      // (the encoder does not know F: a stray byte may name any variable)
      std::vector<int8_t> st(M);
      int32_t first = 0;
      if (gpgomea_validate(ops.data(), M, L_max, C_max, GPGOMEA_MAX_FEATURES, H, st.data(), &first) != 0 ||
          first != -1) {
        std::printf("validate refused an encoded batch at case %d\n", it);
        return 1;
      }
      for (int i = 0; i < M; ++i)
        if (st[i] != 0) {
          std::printf("encoded program %d invalid at case %d\n", i, it);
          return 1;
        }
    }
    // random bytes through validate
    std::vector<int8_t> rb(size_t(M) * L_max), st(M);
    for (auto& b : rb) b = int8_t(uni(0, 3) ? uni(-1, 80) : uni(-128, 127));
    int32_t first = 0;
    const int nbad = gpgomea_validate(rb.data(), M, L_max, C_max, F, int32_t(uni(-1, 8)), st.data(), &first);
    if (nbad < 0 || (nbad == 0) != (first == -1) || (first >= 0 && st[size_t(first)] != 2)) {
      std::printf("validate counts disagree at case %d\n", it);
      return 1;
    }
    ++cases;
  }
  std::printf("ok %ld cases, %ld round trips\n", cases, trips);
  return 0;
}
