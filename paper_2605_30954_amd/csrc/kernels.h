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

// Seed of the adjoint, per individual, written by the finalize: the residual
// of row r is s0 + s1 p_r - y_r ((a, b) with linear scaling, (0, 1) without);
// the gradient kernels sum (residual * inv_scale) * dp/dc in binary32 terms and
// the gradient finalize multiplies by scale = 1 / inv_scale, a power of two
// near the root-mean-square residual (exact scaling: it only keeps the
// binary32 terms of heavy-tailed targets within range).
enum : int { AB_S0 = 0, AB_S1 = 1, AB_INV_SCALE = 2, AB_SCALE = 3, AB_WORDS = 4 };

// Launch parameters of the row-tiled kernels.
struct TileCfg {
  int K = 8;               // rows per lane per batch
  int D = 8;               // register stack slots (template)
  int W = 4;               // waves per block
  int R = 1024;            // rows per LDS tile (multiple of 64*K)
  int G = 16;              // individuals per group (fused forward)
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

// events[i][m] (m < ET): flush events of path forward mode, in uop order
// (see k_prep.hip); ET >= L_max - 1 never overflows
hipError_t launch_compile(const int8_t* ops, int M, int L_max, const float* consts, int C_max,
                          int F, int Dmax, int U_stride, uint2* uops, ProgMeta* meta,
                          uint2* events, int ET, hipStream_t s);

// mean prediction over the first rows -> meta[i].mu
hipError_t launch_probe(bool fp64, const uint2* uops, int U_stride, ProgMeta* meta, int M,
                        const DataArgs& d, hipStream_t s);

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

// ------------------------------------------------------------------ adjoint
// Work classes of the path-forward-mode adjoint (see k_adjoint.hip): 0..3
// shallow programs with at most 4, 8, 16, or more constants (chunks of 32),
// 4 deep programs (more than four stack slots); kAdjFallback and
// kAdjFallbackWide are the binary64 passes over the fallen-back entries'
// parts of 8 constants (at most 4 stack slots, or more).  The plain form
// runs the same class kernels, one individual per launch.
constexpr int kAdjClasses = 5;
constexpr int kAdjFallback = 5;
constexpr int kAdjFallbackWide = 6;
constexpr int kAdjChunks = 8;   // entries per individual at most (GPGOMEA_MAX_CONSTS / 32)
constexpr int kAdjChunkNC = 32;  // constants per entry of the chunked classes
constexpr int kAdjParts = 4;  // binary64 list items per entry (8 constants each)

// One class launch: the entries list[0 .. *count) over n_spans spans of
// span_rows rows, G entries per group, n_groups group slots per span (blocks
// loop over the groups of their slot).
struct AdjLaunch {
  int cls, K;
  const uint2* uops;
  int U_stride;
  const ProgMeta* meta;
  DataArgs d;
  const double* stats;
  const double* ab;
  double* gpart;
  int C_max, gstride, gi0;
  const int* list;
  const int* count;
  int R, G, n_groups, n_spans;
  int64_t span_rows;
  const uint2* events;
  int ET;
  int* redo;
  int32_t* redo_span;
  int rstride, ebase;
  int* fb_list;
  int* fb_count;
  int fb_stride;
  bool split;
  uint64_t* pool;  // bad-tile masks (tile_words words per slot), pool_cap slots
  int* pool_count;
  int pool_cap, tile_words;
};
// Tile-granular binary64 fallback: one bit per row tile of a span, at most
// 64 * kTileWords tiles per span (else the fallback redoes whole spans).
constexpr int kTileWords = 8;
// static LDS of the path kernels (tile masks and redo states of a group)
constexpr size_t kAdjStaticLds = 64 * kTileWords * 8 + 64 * 4 + 16;

// lists[c * lstride + k] (c < kAdjClasses), counts[c]; counts[kAdjClasses],
// counts[kAdjClasses + 1] = 0 (the fallback lists); redo[i * 8 + k] = 0
hipError_t launch_adjoint_partition(const ProgMeta* meta, const double* ab, int M, int lstride,
                                    int* lists, int* counts, int* redo, hipStream_t s);
// plain form: plist[8i + k] = 8i + k, pcount[i] = entries of i, pfb_count[2i], [2i + 1] = 0
hipError_t launch_adjoint_plain_lists(const ProgMeta* meta, const double* ab, int M, int* plist,
                                      int* pcount, int* pfb_count, int* redo, hipStream_t s);
hipError_t launch_adjoint_class(const AdjLaunch& L, hipStream_t s);
// grad[i][j] for i in [i0, i0 + M): 2 s1 / N * sum of gpart[((i - i0) * C_max + j) * gstride + span]
hipError_t launch_grad_finalize(const ProgMeta* meta, int i0, int M, int C_max, const double* gpart,
                                int gstride, int n_spans, const double* stats, const double* ab,
                                double* grad, hipStream_t s);
// The paper's two evaluation designs (comparators of the fused path): raw MSE
// of M programs, one workgroup (design 1) or nb workgroups plus an
// aggregation kernel (design 2) per program; part = M * nb doubles.
struct DesignArgs {
  const int8_t* ops;
  int M, L;
  const float* consts;
  int C, F;
  const float* X;
  int64_t ldx, N;
  const float* y;
  int block;
  double* fitness;
  int8_t* status;
};
hipError_t launch_design1(const DesignArgs& a, hipStream_t s);
hipError_t launch_design2(const DesignArgs& a, int nb, double* part, hipStream_t s);
// One Adam step on every program's constants (constants [M, C] in place,
// moments mom1/mom2 [M, C], best constants / fitness kept per program).
struct AdamParams {
  float lr, beta1, beta2, eps;
  float omb1, omb2;    // 1 - beta1, 1 - beta2 (formed in binary64 from the caller's values)
  float bias1, bias2;  // 1 - beta1^t, 1 - beta2^t (likewise)
};
hipError_t launch_adam_consts(float* consts, int M, int C, const double* grad, const double* fitness,
                              float* mom1, float* mom2, float* best_c, double* best_f,
                              const AdamParams& p, hipStream_t s);
// LDS bytes of one path-class block (row tile, centred targets, constant
// accumulators: one copy, or W with split)
size_t adjoint_path_lds_bytes(int F, int R, int G, int NC, int W, bool split);

int lds_limit_bytes();
int measure_op_costs(double* out, int n, int iters, hipStream_t s, float* scratch);
hipError_t launch_fill_u32(unsigned* p, int n, unsigned v, hipStream_t s);

// Programs per group of the forward kernel (its LDS table of the group's
// status and shift holds this many).
constexpr int kFwdMaxG = 128;

inline size_t forward_lds_bytes(int F, int R, int G) {
  return size_t(F) * R * 4 + size_t(R) * 8 + size_t(G) * 4 * 8 + 16;
}

}  // namespace gg
