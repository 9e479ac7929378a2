// api.hip -- the C ABI of libkmpp (declared in include/kmpp.h): argument
// checks, workspace carving, kernel choice and launch order.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <utility>

#include <hip/hip_ext.h>

#include "kmpp_dev.h"
#include "kmpp_impl.h"

namespace kmpp {
namespace {

inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

int elem_bytes(int dtype) { return dtype == KMPP_F32 ? 4 : dtype == KMPP_BF16 ? 2 : 1; }
bool valid_dtype(int dtype) { return dtype == KMPP_F32 || dtype == KMPP_BF16 || dtype == KMPP_FP8_E4M3; }

// ---- tuning table: (dtype, d) -> launch schedule
struct SeedTune {
  int threads, rpt, u, ntl;  // u, ntl (row path): 0 / -1 = automatic
  int draw;                  // KMPP_DRAW_PASS, KMPP_DRAW_KERNEL or 0 (automatic)
};
std::mutex g_tune_mu;
std::map<std::pair<int, int>, SeedTune> g_tune;
// budget of one wait for the lead workgroup's index, in ticks of the 100 MHz
// real-time counter: one second unless the tuning table says otherwise
// ("lead wait_ms <v>"; 0 makes every wait give up at once, for testing)
constexpr uint64_t kLeadWaitDefault = 100000000ull;
uint64_t g_lead_wait = kLeadWaitDefault;

bool tuned(int dtype, int d, SeedTune* t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find({dtype, d});
  if (it == g_tune.end()) return false;
  *t = it->second;
  return true;
}

// Most tiles for the draw at pass start (every workgroup reads every tile sum).
constexpr int kDrawAtStartTiles = 2048;
// Up to this many tiles the automatic choice is the draw at pass start (it
// was faster on every measured shape; with ~1000 tiles the draw kernel was).
constexpr int kFewTiles = 256;
constexpr int kLeadTiles = 4096;
// Fewest tiles a tuned schedule leaves a pass (the 512-thread workgroups the
// chip holds at once: 256 CUs x 4).
constexpr int64_t kMinTiles = 1024;

// Rows larger than the 256 MiB last-level cache are streamed with
// non-temporal loads; smaller ones stay cached between passes.
constexpr int64_t kCachedRowBytes = 256ll << 20;

const SeedVariant* pick_seed_variant(int dtype, int d, int nt, int u, int rl, int cs) {
  const auto& vs = seed_variants();
  const int eb = elem_bytes(dtype);
  for (int uu : {u, 8})
    for (const auto& v : vs)
      if (v.fmt == dtype && v.nt == nt && v.dexact == d && (d * eb) % v.cb == 0 && v.u == uu && v.rl == rl &&
          v.cs == cs)
        return &v;
  if (cs != CEN_LDS || rl == ROW_BUFFER) return nullptr;  // memory-space variants: exact widths only
  const SeedVariant* best = nullptr;
  for (const auto& v : vs)
    if (v.fmt == dtype && v.nt == nt && v.dexact < 0 && -v.dexact >= d)
      if (!best || -v.dexact < -best->dexact) best = &v;
  return best;
}

}  // namespace

int seed_pick_config(int dtype, int64_t N, int d, const kmpp_seed_opts* opts, const SeedVariant** var,
                     int* rpt_out, int* ntiles_out, int* draw_out) {
  int nt = 256, rpt = 0, u = 8, tuned_draw = 0;
  int ntl = (int64_t)N * d * elem_bytes(dtype) > kCachedRowBytes ? 1 : 0;
  SeedTune t;
  if (tuned(dtype, d, &t)) {
    nt = t.threads;
    rpt = t.rpt;
    if (t.u > 0) u = t.u;
    if (t.ntl >= 0) ntl = t.ntl;
    tuned_draw = t.draw;
  }
  if (opts && opts->threads) nt = opts->threads;
  const bool caller_rpt = opts && opts->rows_per_tile > 0;
  if (caller_rpt) rpt = opts->rows_per_tile;
  if (opts && opts->loads_per_lane > 0) u = opts->loads_per_lane;
  if (opts && opts->row_loads >= 0) ntl = opts->row_loads;
  int cs = CEN_LDS;
  if (opts && opts->centre_source) cs = opts->centre_source - 1;
  if (nt != 256 && nt != 512) return KMPP_E_UNSUPPORTED;
  if (ntl < ROW_CACHED || ntl > ROW_BUFFER || cs < CEN_LDS || cs > CEN_GLOBAL) return KMPP_E_INVALID;
  const SeedVariant* v = pick_seed_variant(dtype, d, nt, u, ntl, cs);
  if (!v) return KMPP_E_UNSUPPORTED;
  const int64_t it = v->rows_per_iter;
  if (rpt <= 0) {
    // about 64 KiB of rows per tile
    const int64_t row_bytes = (int64_t)d * elem_bytes(dtype);
    rpt = (int)std::max<int64_t>(it, (65536 / std::max<int64_t>(1, row_bytes)) / it * it);
  }
  // a tuned tile (chosen at one size per format and width) or the default
  // one is shrunk where it would leave fewer than kMinTiles tiles, so
  // smaller inputs still spread over the chip (unshrunk 64 KiB tiles give
  // 20,000 x 9 rows 11 workgroups: 21 us per seed, against 6.8 us for the
  // tuned width 8)
  if (!caller_rpt) rpt = (int)std::min<int64_t>(rpt, std::max<int64_t>(it, (N + kMinTiles - 1) / kMinTiles));
  int64_t r = ((int64_t)rpt + it - 1) / it * it;
  const int64_t min_r = (N + kMaxTiles - 1) / kMaxTiles;
  if (r < min_r) r = (min_r + it - 1) / it * it;
  if (r > (int64_t)1 << 30) return KMPP_E_UNSUPPORTED;
  // a buffer resource spans one tile with 32-bit byte offsets
  if (v->rl == ROW_BUFFER && r * d * elem_bytes(dtype) > ((int64_t)1 << 31)) return KMPP_E_UNSUPPORTED;
  *var = v;
  *rpt_out = (int)r;
  *ntiles_out = (int)((N + r - 1) / r);
  // the caller's choice; else the draw at pass start wherever a pass has few
  // tiles (it saves a launch per seed and reads little), else the tuned
  // choice (taken at one size per format and width), else the lead
  // workgroup's draw up to kLeadTiles tiles (faster than the draw kernel
  // there: -7 % per seed on 977 tiles, -1 to -3 % on 2048-4096) and the draw
  // kernel beyond (0.2-2 % faster on 8192 tiles, where the one drawing
  // workgroup reads 64 KiB of tile sums alone)
  int draw = opts && opts->draw ? opts->draw : KMPP_DRAW_AUTO;
  if (draw == KMPP_DRAW_AUTO)
    draw = *ntiles_out <= kFewTiles
               ? KMPP_DRAW_PASS
               : (tuned_draw ? tuned_draw : (*ntiles_out <= kLeadTiles ? KMPP_DRAW_LEAD : KMPP_DRAW_KERNEL));
  *draw_out = draw;
  return KMPP_OK;
}

size_t seed_workspace(int64_t N, int K) { return seed_layout(N, K).total; }

// The one-workgroup loop applies: FP32 rows (and weights) in LDS, no option
// that only the multi-workgroup passes honour.
bool small_applies(int64_t N, int d, int dtype, const int32_t* wts, const kmpp_seed_opts* opts) {
  if (dtype != KMPP_F32 || !seed_small_fn(N, d, wts != nullptr)) return false;
  return !(opts && (opts->threads || opts->rows_per_tile > 0 || opts->loads_per_lane > 0 || opts->row_loads >= 0 ||
                    opts->centre_source || opts->out_recheck || opts->step_events));
}

int seed_run(const float* X, int64_t N, int d, int K, uint64_t seed, uint32_t inst, uint32_t tag,
             const int32_t* wts, float* out_centers, float* out_D, int64_t* out_idx, const void* Xq,
             const int8_t* Xq_exp, int dtype, const kmpp_seed_opts* opts, void* workspace, size_t ws_bytes,
             hipStream_t stream, int32_t* status_out) {
  const SeedLayout L = seed_layout(N, K);
  if (ws_bytes < L.total) return KMPP_E_WORKSPACE;
  const int want = opts ? opts->draw : KMPP_DRAW_AUTO;
  const bool small = small_applies(N, d, dtype, wts, opts);
  if (want == KMPP_DRAW_SINGLE && !small) return KMPP_E_UNSUPPORTED;
  if (small && (want == KMPP_DRAW_SINGLE || want == KMPP_DRAW_AUTO)) {
    char* ws = static_cast<char*>(workspace);
    SeedParams p = {};
    p.xs = X;
    p.X = X;
    p.centers = out_centers;
    p.idx = out_idx ? out_idx : reinterpret_cast<int64_t*>(ws + L.idx);
    p.D = out_D ? out_D : reinterpret_cast<float*>(ws + L.D);
    p.ctl = reinterpret_cast<Ctl*>(ws);
    p.N = N;
    p.d = d;
    p.K = K;
    p.inst = inst;
    p.seed = seed;
    p.tag = tag;
    p.wts = wts;
    p.sumD = opts ? opts->out_sumD : nullptr;
    p.status_out = status_out;
    void* args[] = {&p};
    return hipLaunchKernel(seed_small_fn(N, d, wts != nullptr), dim3(1), dim3((unsigned)seed_small_threads()), args, 0, stream) ==
                   hipSuccess
               ? KMPP_OK
               : KMPP_E_HIP;
  }
  const SeedVariant* v = nullptr;
  int rpt = 0, ntiles = 0, draw = 0;
  const int rc = seed_pick_config(dtype, N, d, opts, &v, &rpt, &ntiles, &draw);
  if (rc != KMPP_OK) return rc;
  char* ws = static_cast<char*>(workspace);

  SeedParams p;
  p.xs = dtype == KMPP_F32 ? static_cast<const void*>(X) : Xq;
  p.xexp = Xq_exp;
  p.X = X;
  p.centers = out_centers;
  p.idx = out_idx ? out_idx : reinterpret_cast<int64_t*>(ws + L.idx);
  p.D = out_D ? out_D : reinterpret_cast<float*>(ws + L.D);
  p.tsum = reinterpret_cast<double*>(ws + L.tsum);
  p.tsum_w = p.tsum;
  p.Dw = p.D;
  p.ctl = reinterpret_cast<Ctl*>(ws);
  p.recheck = opts ? opts->out_recheck : nullptr;
  p.N = N;
  p.d = d;
  p.K = K;
  p.pass = 0;
  p.rows_per_tile = rpt;
  p.ntiles = ntiles;
  p.inst = inst;
  p.seed = seed;
  p.wts = wts;
  p.tag = tag;
  p.sumD = opts ? opts->out_sumD : nullptr;
  p.status_out = status_out;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    p.lead_wait = g_lead_wait;
  }
  // the draw at pass start (unweighted seeding, exact-width passes): every
  // workgroup reads all tile sums, so their number is bounded, and its LDS
  // staging must leave the pass's occupancy alone (160 KiB of LDS per CU,
  // 2048 threads)
  const size_t draw_lds = std::max(sizeof(double) * (size_t)ntiles, sizeof(float) * (size_t)rpt);
  const bool at_start = draw == KMPP_DRAW_PASS && v->fn_drawer && !wts && ntiles <= kDrawAtStartTiles &&
                        draw_lds <= (size_t)160 * 1024 * v->nt / 2048;
  const bool lead = draw == KMPP_DRAW_LEAD && v->fn_lead && !wts;
  const void* pass_fn = at_start ? v->fn_drawer : (lead ? v->fn_lead : v->fn);
  // its buffers: pass m writes D to Dbuf[(K - m) % 2], so pass K ends in the
  // caller's D, and its tile sums to Tbuf[m % 2]
  float* const Dbuf[2] = {p.D, reinterpret_cast<float*>(ws + L.D2)};
  double* const Tbuf[2] = {p.tsum, reinterpret_cast<double*>(ws + L.tsum2)};
  hipEvent_t* ev = opts ? static_cast<hipEvent_t*>(opts->step_events) : nullptr;

  void* args[] = {&p};
  if (hipLaunchKernel(seed_init_fn(), dim3(1), dim3(256), args, 0, stream) != hipSuccess) return KMPP_E_HIP;
  if (wts) {
    // the first centre: a draw proportional to w (D := 1)
    if (hipLaunchKernel(seed_wfirst_fn(), dim3((unsigned)ntiles), dim3(256), args, 0, stream) != hipSuccess ||
        hipLaunchKernel(seed_draw_fn(wts != nullptr), dim3(1), dim3((unsigned)seed_draw_threads()), args, 0, stream) != hipSuccess)
      return KMPP_E_HIP;
  }
  const size_t shmem = std::max(sizeof(float) * (size_t)d, at_start ? draw_lds : (size_t)0);
  const dim3 grid((unsigned)ntiles);
  for (int m = 1; m <= K; ++m) {
    p.pass = m;
    if (at_start) {
      p.Dw = Dbuf[(K - m) % 2];
      p.D = Dbuf[(K - m + 1) % 2];  // pass m-1's (not read by pass 1)
      p.tsum_w = Tbuf[m % 2];
      p.tsum = Tbuf[(m + 1) % 2];
    }
    // with step events, the events are attached to the dispatch itself and
    // track the kernel's own start and stop
    const hipError_t le =
        ev ? hipExtLaunchKernel(pass_fn, grid, dim3((unsigned)v->nt), args, shmem, stream, ev[2 * (m - 1)],
                                ev[2 * (m - 1) + 1], 0)
           : hipLaunchKernel(pass_fn, grid, dim3((unsigned)v->nt), args, shmem, stream);
    if (le != hipSuccess) return KMPP_E_HIP;
    if (m < K && !at_start && !lead &&
        hipLaunchKernel(seed_draw_fn(wts != nullptr), dim3(1), dim3((unsigned)seed_draw_threads()), args, 0, stream) !=
            hipSuccess)
      return KMPP_E_HIP;
  }
  return KMPP_OK;
}

}  // namespace kmpp

using namespace kmpp;

extern "C" {

size_t kmpp_seed_workspace_bytes(int64_t N, int32_t d, int32_t K, int32_t dtype) {
  if (N < 1 || K < 1 || K > N || d < 1 || d > KMPP_MAX_D || !valid_dtype(dtype)) return 0;
  return seed_layout(N, K).total;
}

int kmpp_seed(const float* X, int64_t N, int32_t d, int32_t K, uint64_t seed, float* out_centers, float* out_D,
              int64_t* out_idx, const void* Xq, const int8_t* Xq_exp, int32_t dtype, const kmpp_seed_opts* opts,
              void* workspace, size_t ws_bytes, void* stream_) {
  if (!X || !out_centers || !workspace) return KMPP_E_INVALID;
  if (N < 1 || K < 1 || K > N || N > INT32_MAX || d < 1 || d > KMPP_MAX_D) return KMPP_E_INVALID;
  if (!valid_dtype(dtype)) return KMPP_E_INVALID;
  if (!aligned(X, 16) || !aligned(workspace, 256)) return KMPP_E_INVALID;
  if (dtype != KMPP_F32) {
    if (!Xq || !aligned(Xq, 16)) return KMPP_E_INVALID;
    if (dtype == KMPP_FP8_E4M3 && !Xq_exp) return KMPP_E_INVALID;
  }
  if (opts && (opts->draw < KMPP_DRAW_AUTO || opts->draw > KMPP_DRAW_SINGLE)) return KMPP_E_INVALID;
  return seed_run(X, N, d, K, seed, opts ? opts->instance : 0u, 0u, nullptr, out_centers, out_D, out_idx, Xq, Xq_exp,
                  dtype, opts, workspace, ws_bytes, static_cast<hipStream_t>(stream_));
}

int32_t kmpp_seed_parallel_capacity(int64_t N, int32_t rounds, double ell) {
  if (N < 1 || rounds < 0 || !(ell > 0.0)) return 0;
  return kpar_capacity(N, rounds, ell);
}

size_t kmpp_seed_parallel_workspace_bytes(int64_t N, int32_t d, int32_t K, int32_t rounds, double ell) {
  if (N < 1 || K < 1 || d < 1 || d > KMPP_MAX_D || rounds < 0 || rounds > 64 || !(ell > 0.0)) return 0;
  return kpar_workspace(N, d, K, rounds, ell);
}

int kmpp_seed_parallel(const float* X, int64_t N, int32_t d, int32_t K, uint64_t seed, int32_t rounds, double ell,
                       uint32_t instance, float* out_centers, int64_t* out_idx, int64_t* out_cand,
                       int32_t* out_round_end, int32_t* out_weights, int32_t* out_labels, void* workspace,
                       size_t ws_bytes, void* stream) {
  if (!X || !out_centers || !workspace) return KMPP_E_INVALID;
  if (N < 1 || K < 1 || N > INT32_MAX || d < 1 || d > KMPP_MAX_D || rounds < 0 || rounds > 64 || !(ell > 0.0) ||
      ell > 1e12)
    return KMPP_E_INVALID;
  if (!aligned(X, 16) || !aligned(workspace, 256)) return KMPP_E_INVALID;
  if (ws_bytes < kpar_workspace(N, d, K, rounds, ell)) return KMPP_E_WORKSPACE;
  return launch_kpar(X, N, d, K, seed, rounds, ell, instance, out_centers, out_idx, out_cand, out_round_end,
                     out_weights, out_labels, workspace, ws_bytes, static_cast<hipStream_t>(stream));
}

size_t kmpp_lloyd_workspace_bytes(int64_t N, int32_t d, int32_t K, int32_t dtype) {
  if (N < 1 || K < 1 || d < 1 || d > KMPP_MAX_D || !valid_dtype(dtype)) return 0;
  return lloyd_workspace(N, d, K, dtype);
}

int kmpp_lloyd(const void* X, const int8_t* X_exp, int32_t dtype, int64_t N, int32_t d, int32_t K, float* C,
               int32_t iters, int32_t* out_labels, double* out_cost, int64_t* out_changed, int32_t* out_counts,
               void* workspace, size_t ws_bytes, void* stream) {
  if (!X || !C || !out_labels || !workspace) return KMPP_E_INVALID;
  if (N < 1 || K < 1 || N > INT32_MAX || d < 1 || d > KMPP_MAX_D || iters < 0 || !valid_dtype(dtype))
    return KMPP_E_INVALID;
  if (dtype == KMPP_FP8_E4M3 && !X_exp) return KMPP_E_INVALID;
  if (!aligned(X, 16) || !aligned(C, 16) || !aligned(workspace, 256)) return KMPP_E_INVALID;
  if (ws_bytes < lloyd_workspace(N, d, K, dtype)) return KMPP_E_WORKSPACE;
  return launch_lloyd(X, X_exp, dtype, N, d, K, C, iters, out_labels, out_cost, out_changed, out_counts, workspace,
                      ws_bytes, static_cast<hipStream_t>(stream));
}

int kmpp_quantize(const float* X, int64_t N, int32_t d, int32_t dtype, void* Xq, int8_t* Xq_exp, void* stream) {
  if (!X || !Xq || N < 1 || d < 1 || d > KMPP_MAX_D) return KMPP_E_INVALID;
  if (dtype != KMPP_BF16 && dtype != KMPP_FP8_E4M3) return KMPP_E_INVALID;
  if (dtype == KMPP_FP8_E4M3 && !Xq_exp) return KMPP_E_INVALID;
  if (!aligned(X, 16) || !aligned(Xq, 16)) return KMPP_E_INVALID;
  return launch_quantize(X, N, d, dtype, Xq, Xq_exp, static_cast<hipStream_t>(stream));
}

size_t kmpp_assign_workspace_bytes(int64_t N, int32_t d, int32_t K, int32_t dtype) {
  if (N < 1 || K < 1 || d < 1 || d > KMPP_MAX_D || !valid_dtype(dtype)) return 0;
  return assign_workspace(N, d, K, dtype);
}

int kmpp_assign(const void* X, const int8_t* X_exp, int32_t dtype, const float* C, int64_t N, int32_t d, int32_t K,
                int32_t* out_labels, float* out_mind, void* workspace, size_t ws_bytes, void* stream) {
  if (!X || !C || !out_labels || !workspace) return KMPP_E_INVALID;
  if (N < 1 || K < 1 || N > INT32_MAX || d < 1 || d > KMPP_MAX_D || !valid_dtype(dtype)) return KMPP_E_INVALID;
  if (dtype == KMPP_FP8_E4M3 && !X_exp) return KMPP_E_INVALID;
  if (!aligned(X, 16) || !aligned(C, 16) || !aligned(workspace, 256)) return KMPP_E_INVALID;
  if (ws_bytes < assign_workspace(N, d, K, dtype)) return KMPP_E_WORKSPACE;
  return launch_assign(X, X_exp, dtype, C, N, d, K, out_labels, out_mind, workspace, ws_bytes,
                       static_cast<hipStream_t>(stream));
}

size_t kmpp_batched_workspace_bytes(const kmpp_instance* inst, int32_t n_inst) {
  if (!inst || n_inst < 1) return 0;
  return batched_workspace(inst, n_inst);
}

int kmpp_seed_batched_prepare(const kmpp_instance* inst, int32_t n_inst, uint64_t seed, void* workspace,
                              size_t ws_bytes, void* stream) {
  if (!inst || n_inst < 1 || !workspace || !aligned(workspace, 256)) return KMPP_E_INVALID;
  return batched_prepare(inst, n_inst, seed, workspace, ws_bytes, static_cast<hipStream_t>(stream));
}

int kmpp_seed_batched_launch(void* workspace, void* stream) {
  if (!workspace || !aligned(workspace, 256)) return KMPP_E_INVALID;
  return batched_launch(workspace, static_cast<hipStream_t>(stream));
}

int kmpp_seed_batched(const kmpp_instance* inst, int32_t n_inst, uint64_t seed, void* workspace, size_t ws_bytes,
                      void* stream) {
  const int rc = kmpp_seed_batched_prepare(inst, n_inst, seed, workspace, ws_bytes, stream);
  if (rc != KMPP_OK) return rc;
  return kmpp_seed_batched_launch(workspace, stream);
}

int kmpp_status(const void* workspace, void* stream, int32_t* out) {
  if (!workspace || !out) return KMPP_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(s) != hipSuccess) return KMPP_E_HIP;
  if (hipMemcpy(out, workspace, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) return KMPP_E_HIP;
  return KMPP_OK;
}

int kmpp_status_poll(const void* workspace, int32_t* out) {
  if (!workspace || !out) return KMPP_E_INVALID;
  if (hipMemcpy(out, workspace, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) return KMPP_E_HIP;
  return KMPP_OK;
}

struct kmpp_graph_s {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

int kmpp_graph_begin(void* stream) {
  return hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal) == hipSuccess
             ? KMPP_OK
             : KMPP_E_HIP;
}

int kmpp_graph_end(void* stream, kmpp_graph* out) {
  if (!out) return KMPP_E_INVALID;
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(static_cast<hipStream_t>(stream), &g) != hipSuccess || !g) return KMPP_E_HIP;
  hipGraphExec_t e = nullptr;
  if (hipGraphInstantiate(&e, g, nullptr, nullptr, 0) != hipSuccess) {
    hipGraphDestroy(g);
    return KMPP_E_HIP;
  }
  kmpp_graph h = static_cast<kmpp_graph>(malloc(sizeof(kmpp_graph_s)));
  if (!h) {
    hipGraphExecDestroy(e);
    hipGraphDestroy(g);
    return KMPP_E_INVALID;
  }
  h->graph = g;
  h->exec = e;
  *out = h;
  return KMPP_OK;
}

int kmpp_graph_launch(kmpp_graph g, void* stream) {
  if (!g) return KMPP_E_INVALID;
  return hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? KMPP_OK : KMPP_E_HIP;
}

int kmpp_graph_destroy(kmpp_graph g) {
  if (!g) return KMPP_E_INVALID;
  hipGraphExecDestroy(g->exec);
  hipGraphDestroy(g->graph);
  free(g);
  return KMPP_OK;
}

int kmpp_tune_load(const char* path) {
  if (!path) return KMPP_E_INVALID;
  FILE* f = fopen(path, "r");
  if (!f) return KMPP_E_INVALID;
  char line[256];
  int n = 0;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  while (fgets(line, sizeof(line), f)) {
    char kind[32], key[32];
    int dt, d, nt, rpt, u = 0, ntl = -1, draw = 0;
    double val;
    const int got = sscanf(line, "%31s %d %d %d %d %d %d %d", kind, &dt, &d, &nt, &rpt, &u, &ntl, &draw);
    if (got >= 5 && strcmp(kind, "seed") == 0 && valid_dtype(dt) && (nt == 256 || nt == 512) && rpt > 0 &&
        (u == 0 || u == 8 || u == 16) && ntl >= -1 && ntl <= 1 && draw >= 0 && draw <= KMPP_DRAW_LEAD) {
      g_tune[{dt, d}] = SeedTune{nt, rpt, u, ntl, draw};
      ++n;
    } else if (sscanf(line, "%31s %31s %lf", kind, key, &val) == 3 && strcmp(kind, "batched") == 0 &&
               batched_tune_set(key, val) == KMPP_OK) {
      ++n;
    } else if (sscanf(line, "%31s %31s %lf", kind, key, &val) == 3 && strcmp(kind, "lead") == 0 &&
               strcmp(key, "wait_ms") == 0) {
      g_lead_wait = val < 0.0 ? kLeadWaitDefault : (uint64_t)(val * 1e5);
      ++n;
    }
  }
  fclose(f);
  return n;
}

const char* kmpp_strerror(int code) {
  switch (code) {
    case KMPP_OK: return "ok";
    case KMPP_W_DEGENERATE: return "sum of distances was zero at a draw (fewer distinct points than seeds)";
    case KMPP_E_INVALID: return "invalid argument";
    case KMPP_E_WORKSPACE: return "workspace too small";
    case KMPP_E_HIP: return "HIP runtime error";
    case KMPP_E_NONFINITE: return "non-finite sum of distances (NaN or Inf in the points)";
    case KMPP_E_UNSUPPORTED: return "unsupported shape or format";
    case KMPP_E_TIMEOUT: return "a device-side wait expired";
    case KMPP_E_TOO_LARGE: return "input larger than the fixed scratch of the allocation-free entry point";
    default: return "unknown status";
  }
}

int kmpp_version(void) { return 100; }

}  // extern "C"
