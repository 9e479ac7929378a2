// kmpp_impl.h -- host/device shared declarations of libkmpp (not part of the
// public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "kmpp.h"

namespace kmpp {

struct Ctl;

// Arguments of one seed-loop launch (init or pass).
struct SeedParams {
  const void* xs;        // rows read by the distance pass (FP32, BF16 or FP8)
  const int8_t* xexp;    // FP8 row exponents or null
  const float* X;        // FP32 rows: centres are copied from here
  float* centers;        // [K, d]
  int64_t* idx;          // [K]
  float* D;              // [N]
  double* tsum;          // [ntiles] FP64 tile sums of D
  Ctl* ctl;              // status and arrival counter
  float* recheck;        // [2K] or null
  int64_t N;
  int32_t d;
  int32_t K;
  int32_t pass;          // 1..K: pass m uses centre m-1 and (m < K) draws seed m
  int32_t rows_per_tile;
  int32_t ntiles;
  uint32_t inst;
  uint64_t seed;
  const int32_t* wts;    // weighted seeding: row weights (draws proportional to w * D), or null
  uint32_t tag;          // Philox counter word 3 of the draws (0: the k-means++ stream)
  float* Dw;             // draw at pass start: this pass's D (every row; D holds the previous pass's)
  double* tsum_w;        // draw at pass start: this pass's tile sums (tsum holds the previous pass's)
  double* sumD;          // [K] or null: the FP64 sum of D each draw inverted
  int32_t* status_out;   // or null: the status word, copied by the last pass
  uint64_t lead_wait;    // lead-workgroup draw: budget of one wait in real-time counter ticks (0: give up at once)
};

// One compiled seed-pass kernel.
struct SeedVariant {
  int fmt;
  int dexact;        // > 0: exactly this d with 16-byte (or 8-byte) chunks; < 0: any d <= -dexact
  int cb, g, cpl, u;
  bool full;
  int rl;            // row path: ROW_CACHED, ROW_NONTEMPORAL or ROW_BUFFER
  int cs;            // centre source: CEN_LDS, CEN_SCALAR or CEN_GLOBAL
  int nt;
  int rows_per_iter; // rows one workgroup covers per loop iteration
  const void* fn;
  const void* fn_drawer;  // the same pass drawing the previous seed at its start, or null
  const void* fn_lead;    // the same pass with workgroup 0 drawing the previous seed for all, or null
};

const std::vector<SeedVariant>& seed_variants();
// The one-workgroup seed loop (seed_small.hip): the rows interleaved over
// 1024 threads in an LDS array of kSmallMaxElems FP32 values, at most 16
// rows per thread: ceil(N / 1024) * d * 1024 <= kSmallMaxElems.
constexpr int kSmallMaxElems = 36864;
const void* seed_small_fn(int64_t N, int d, bool weighted);  // null where the input does not fit
int seed_small_threads();
const void* seed_init_fn();
const void* seed_wfirst_fn();
const void* seed_draw_fn(bool weighted);
int seed_draw_threads();

// Maximum number of tiles of one pass; bounds the tile-sum scan of the draw
// and the workspace.
constexpr int64_t kMaxTiles = 8192;  // = draw threads (256) x tile sums per thread (32)

// Workspace of one seeding run: the control block, two FP64 tile-sum
// buffers, two D buffers (the second and the second tile sums only for the
// draw at pass start) and the indices.
constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct SeedLayout {
  size_t tsum, tsum2, D, D2, idx, total;  // tsum2, D2: the second buffers of the draw at pass start
};
constexpr SeedLayout seed_layout(int64_t N, int64_t K) {
  SeedLayout L{};
  size_t off = 256;  // the control block (Ctl)
  const size_t tiles = align256(sizeof(double) * (size_t)(N < kMaxTiles ? N : kMaxTiles));
  L.tsum = off;
  off += tiles;
  L.tsum2 = off;
  off += tiles;
  L.D = off;
  off += align256(sizeof(float) * (size_t)N);
  L.D2 = off;
  off += align256(sizeof(float) * (size_t)N);
  L.idx = off;
  off += align256(sizeof(int64_t) * (size_t)K);
  L.total = off;
  return L;
}

// One k-means++ run (init, K passes, K-1 draws) on the stream; weighted when
// wts is non-null (the first draw proportional to w, then to w * D).
int seed_run(const float* X, int64_t N, int d, int K, uint64_t seed, uint32_t inst, uint32_t tag,
             const int32_t* wts, float* out_centers, float* out_D, int64_t* out_idx, const void* Xq,
             const int8_t* Xq_exp, int dtype, const kmpp_seed_opts* opts, void* ws, size_t ws_bytes,
             hipStream_t stream, int32_t* status_out = nullptr);
size_t seed_workspace(int64_t N, int K);

// Assignment
struct AssignParams;
int launch_assign(const void* X, const int8_t* X_exp, int dtype, const float* C, int64_t N, int d, int K,
                  int32_t* labels, float* mind, void* ws, size_t ws_bytes, hipStream_t stream);
size_t assign_workspace(int64_t N, int d, int K, int dtype);

// Lloyd iterations
size_t lloyd_workspace(int64_t N, int d, int K, int dtype);
int launch_lloyd(const void* X, const int8_t* X_exp, int dtype, int64_t N, int d, int K, float* C, int iters,
                 int32_t* out_labels, double* out_cost, int64_t* out_changed, int32_t* out_counts, void* ws,
                 size_t ws_bytes, hipStream_t stream);

// k-means||
int kpar_capacity(int64_t N, int R, double ell);
size_t kpar_workspace(int64_t N, int d, int K, int R, double ell);
int launch_kpar(const float* X, int64_t N, int d, int K, uint64_t seed, int R, double ell, uint32_t inst,
                float* out_centers, int64_t* out_idx, int64_t* out_cand, int32_t* out_round_end, int32_t* out_weights,
                int32_t* out_labels, void* ws, size_t ws_bytes, hipStream_t stream);

// Quantisers
int launch_quantize(const float* X, int64_t N, int d, int dtype, void* Xq, int8_t* Xq_exp, hipStream_t stream);

// Batched
size_t batched_workspace(const kmpp_instance* inst, int n_inst);
int batched_prepare(const kmpp_instance* inst, int n_inst, uint64_t seed, void* ws, size_t ws_bytes,
                    hipStream_t stream);
int batched_launch(void* ws, hipStream_t stream);
int batched_tune_set(const char* key, double value);

}  // namespace kmpp
