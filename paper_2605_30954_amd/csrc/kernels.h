// Host-side launchers of the device kernels (internal interface between the
// C ABI and the kernel translation units).  Every launcher only enqueues on
// `stream` and returns the hipError_t of the launch.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "uop.h"

namespace gg {

// Layout of the dataset statistics block in the workspace (doubles).
enum : int {
  ST_YBAR = 0,  // mean of y
  ST_VY = 1,    // population variance of y
  ST_YT = 2,    // sum of (y - ybar) over all rows (rounding residue, ~0)
  ST_N = 3,
  ST_COUNT = 8
};
constexpr int kStatBlocks = 256;  // partial sums per statistics pass

// Launch parameters of the row-tiled kernels.
struct TileCfg {
  int K = 8;               // rows per lane per batch
  int D = 8;               // register stack slots (template)
  int W = 4;               // waves per block
  int R = 1024;            // rows per LDS tile (multiple of 64*K)
  int G = 16;              // individuals per group (fused forward)
  int NP = 1;              // VGPR pairs holding a program (uop_pairs(L_max))
  int tiles_per_span = 1;  // LDS tiles a block sweeps before writing partials
  int n_spans = 1;
  int n_groups = 1;
};

struct DataArgs {
  const float* X;
  int64_t ldx;
  int F;
  int64_t N;
  const float* y;
};

hipError_t launch_ystats(const float* y, int64_t N, double* stats, double* scratch, hipStream_t s);

// merges[i][m] (m < MT): constant ranges of the two operands of the m-th uop of
// program i whose operands both hold constants (loA | nA<<8 | loS<<16 | nS<<24)
hipError_t launch_compile(const int8_t* ops, int M, int L_max, const float* consts, int C_max,
                          int F, int Dmax, int U_stride, uint2* uops, ProgMeta* meta,
                          uint32_t* merges, int MT, hipStream_t s);

// mean prediction over the first rows -> meta[i].mu
hipError_t launch_probe(bool fp64, int K, int D, const uint2* uops, int U_stride, ProgMeta* meta,
                        int M, const DataArgs& d, hipStream_t s);

// fused batched forward: partial moment sums part[i][span][4]
hipError_t launch_fused_forward(bool fp64, const TileCfg& c, const uint2* uops, int U_stride,
                                const ProgMeta* meta, int M, const DataArgs& d,
                                const double* stats, double* part, bool want_sse, hipStream_t s);

// per-individual finalize of the fused partials
hipError_t launch_finalize(const ProgMeta* meta, int M, const double* part, int n_spans,
                           const double* stats, uint32_t flags, double* fitness, double* aux,
                           int8_t* status, double* ab, hipStream_t s);

// plain form: one launch per individual (call M times), last block finalizes
hipError_t launch_plain_forward(bool fp64, const TileCfg& c, int i, const uint2* uops,
                                int U_stride, const ProgMeta* meta, const DataArgs& d,
                                const double* stats, double* part, unsigned* ticket,
                                uint32_t flags, double* fitness, double* aux, int8_t* status,
                                double* ab, hipStream_t s);
int plain_blocks(const TileCfg& c, int64_t N);

// Adjoint launch plan.  Individuals are split into tiers (register tape of
// tc_a entries, register tape of tc_b entries, LDS tape); every tier cuts the
// rows into the same n_spans spans of span_rows rows.  A tier's n_groups is
// the number of group slots its grid holds per span.
struct AdjPlan {
  TileCfg path, reg, reg_b, wide;
  int n_spans = 1;
  int64_t span_rows = 0;
  int tc_a = 16, tc_b = 32;  // register tape entries of tiers A and B
  int lane_consts = 16;      // per-lane constant columns of the register tiers
  int tape_cap = 1;          // LDS tape entries per wave of tier C
  bool need_b = true;        // ... in tier B (or fall back to it from the path tier)
  bool need_wide = true;     // ... in tier C
  int nc_p = 12;             // path tier: programs with <= nc_p constants (0: none)
  bool need_a = true;        // some program of this shape may fall in tier A
};

// Tier lists: lists[tier * M + k], counts[tier], tier = 0 A, 1 B, 2 C, 3 path
// (after finalize); redo[M] (the path tier's fallback flags, or null) cleared.
hipError_t launch_adjoint_partition(const AdjPlan& a, const ProgMeta* meta, const double* ab, int M,
                                    int* lists, int* counts, int* redo, hipStream_t s);
// Plain form: counts[4i + tier] = 1 for individual i's tier, list0[0] = 0.
hipError_t launch_adjoint_tier_flags(const AdjPlan& a, const ProgMeta* meta, const double* ab, int M,
                                     int* counts, int* list0, hipStream_t s);
// gradient partials gpart[i][span][C_max] of the individuals list[0 .. *count);
// with redo (may be null), an individual that fell back from the path tier
// is redone only on the spans flagged in redo_span
hipError_t launch_adjoint_reg(const AdjPlan& a, int tier, const uint2* uops, int U_stride,
                              const ProgMeta* meta, int M, int C_max, const DataArgs& d,
                              const double* stats, const double* ab, double* gpart,
                              const int* list, const int* count, int* redo,
                              uint8_t* redo_span, hipStream_t s);
// path tier over lists[3][0 .. counts[3]); redo[i] is set for an individual
// with a partial that is not finite (zero redo[] before), redo_span[i][s] says
// which spans (written for every span of every individual of the tier), and
// the individual is appended to the list of tier B (or C) with its count
hipError_t launch_adjoint_path(const AdjPlan& a, const uint2* uops, int U_stride,
                               const ProgMeta* meta, int M, int C_max, const DataArgs& d,
                               const double* stats, const double* ab, double* gpart,
                               const uint32_t* merges, int MT, int* redo, uint8_t* redo_span,
                               int* lists, int* counts, hipStream_t s);
hipError_t launch_adjoint_lds(const AdjPlan& a, const uint2* uops, int U_stride,
                              const ProgMeta* meta, int M, int C_max, const DataArgs& d,
                              const double* stats, const double* ab, double* gpart,
                              const int* list, const int* count, int* redo, uint8_t* redo_span,
                              hipStream_t s);
hipError_t launch_grad_finalize(const ProgMeta* meta, int M, int C_max, const double* gpart,
                                int n_spans, const double* stats, const double* ab,
                                uint32_t flags, const int8_t* status, double* grad,
                                hipStream_t s);

int lds_limit_bytes();
int measure_op_costs(double* out, int n, int iters, hipStream_t s, float* scratch);
hipError_t launch_fill_u32(unsigned* p, int n, unsigned v, hipStream_t s);

// LDS bytes of one LDS-tape adjoint block (row tile, centred targets, W
// copies of the constant accumulators, W wave tapes of tape_cap entries x 64
// lanes x K rows).
inline size_t adjoint_lds_bytes(int F, int R, int G, int C_max, int W, int K, int tape_cap) {
  const size_t off =
      (size_t(F) * R * 4 + size_t(R) * 8 + size_t(W) * G * C_max * 8 + 15) & ~size_t(15);
  return off + size_t(W) * tape_cap * 64 * K * 4;
}
// LDS bytes of one register-tape adjoint block (row tile, centred targets,
// `copies` sets of constant accumulators, W waves x CC per-lane constant
// columns of 65 floats).
inline size_t adjoint_reg_lds_bytes(int F, int R, int G, int C_max, int W, int CC, int copies) {
  return size_t(F) * R * 4 + size_t(R) * 8 + size_t(copies) * G * C_max * 8 +
         size_t(W) * CC * 65 * 4;
}
// LDS bytes of one path-tier block (row tile, centred targets, constant
// accumulators, W waves x NC per-lane constant columns of 65 floats).
inline size_t adjoint_path_lds_bytes(int F, int R, int G, int C_max, int W, int NC) {
  return size_t(F) * R * 4 + size_t(R) * 8 + size_t(G) * C_max * 8 + size_t(W) * NC * 65 * 4;
}
inline size_t forward_lds_bytes(int F, int R, int G) {
  return size_t(F) * R * 4 + size_t(R) * 8 + size_t(G) * 4 * 8 + 16;
}

}  // namespace gg
