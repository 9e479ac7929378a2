/*
 * kmpp.h -- C ABI of libkmpp: k-means++ seeding (D^2 sampling), the
 * nearest-seed assignment, and the steps around them (Lloyd iterations,
 * k-means|| seeding, a batched form) on AMD Instinct MI355X (gfx950).
 *
 * The method is the one of "Parallelization of Kmeans++ using CUDA"
 * (Heydarpour Shahrezaei and Tavoli, arXiv 1908.02136), Section II:
 *   Algorithm 1 / Algorithm 2: the first seed is a uniformly random point;
 *   every point keeps the squared distance D to its nearest chosen seed
 *   (initially +infinity); each further seed is point l with probability
 *   D(l) / sum_w D(w); the output is the seed set H and the partition O of
 *   the points among the seeds.
 *   Section II (reduction paragraph): the sum of D is taken in double
 *   precision.
 * Where the paper is silent this library fixes:
 *   - random stream: Philox4x32-10 with key (lo32(seed), hi32(seed)) and
 *     counter (step, instance, 0, 0); u = ((r0>>5)*2^26 + (r1>>6)) * 2^-53;
 *   - first seed: min(floor(u_0 * N), N-1);
 *   - draw m: t = u_m * sum(D) (one FP64 multiply); the seed is the first
 *     index i whose inclusive FP64 prefix of D exceeds t; if rounding leaves
 *     none, the last index with D > 0;
 *   - sum(D) == 0 (fewer than K distinct points): uniform index and the
 *     warning KMPP_W_DEGENERATE; non-finite sum(D): KMPP_E_NONFINITE;
 *   - assignment ties go to the smallest seed index.
 *
 * Conventions for every entry point:
 *   - all array pointers are DEVICE pointers unless stated otherwise; rows
 *     are contiguous and row-major; X's base must be 16-byte aligned;
 *   - `stream` is a hipStream_t (NULL = the null stream) on which the work
 *     is enqueued;
 *   - the caller owns every buffer, including the workspace, whose size the
 *     matching *_workspace_bytes function gives; the library allocates no
 *     device memory in any entry point (kmpp_seed_noalloc uses a fixed
 *     device array of the library instead of a workspace);
 *   - work is enqueued without synchronising, except kmpp_status,
 *     kmpp_seed_batched_prepare and kmpp_seed_parallel (stated below);
 *   - arguments are validated before anything is enqueued: a negative
 *     return means nothing was launched; KMPP_E_HIP means a launch failed;
 *   - conditions found on the device (non-finite or zero sum of D, an
 *     expired wait in the batched kernel) are written to a status word in
 *     the workspace; read it with kmpp_status after the stream is idle;
 *   - calls that share a workspace must be ordered on one stream.
 */
#ifndef KMPP_H_
#define KMPP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* storage format of the point rows */
enum {
  KMPP_F32 = 0,      /* IEEE binary32 */
  KMPP_BF16 = 1,     /* bfloat16, round to nearest even from FP32 */
  KMPP_FP8_E4M3 = 2  /* OCP E4M3FN with one power-of-two scale 2^e per row, e int8 */
};

/* status codes: 0 ok, > 0 warning (results valid), < 0 error */
enum {
  KMPP_OK = 0,
  KMPP_W_DEGENERATE = 1,    /* sum(D) was 0 at some draw: uniform draw, seeds may repeat */
  KMPP_E_INVALID = -1,      /* bad sizes, null or misaligned pointer, bad dtype */
  KMPP_E_WORKSPACE = -2,    /* workspace smaller than *_workspace_bytes */
  KMPP_E_HIP = -3,          /* a HIP runtime call failed */
  KMPP_E_NONFINITE = -4,    /* sum(D) not finite (NaN or Inf in X) */
  KMPP_E_UNSUPPORTED = -5,  /* shape or format not supported */
  KMPP_E_TIMEOUT = -6,      /* a bounded device-side wait expired */
  KMPP_E_TOO_LARGE = -7     /* input beyond the fixed scratch of kmpp_seed_noalloc */
};

#define KMPP_MAX_D 4096

/*
 * Memory spaces of the seed pass (Section II keeps the points in global or
 * texture memory and the centroids in global or constant memory; Figs. 2c
 * and 3c compare them).  All choices give bit-identical results; they differ
 * only in speed.  Non-default choices exist for FP32 rows with d in
 * {2, 32, 64, 128} at 256 threads and 8 loads per lane (KMPP_E_UNSUPPORTED
 * otherwise).
 *
 * Row paths (kmpp_seed_opts.row_loads):
 *   KMPP_ROWS_CACHED       plain global loads, kept in the caches
 *   KMPP_ROWS_NONTEMPORAL  non-temporal global loads (streamed once per pass)
 *   KMPP_ROWS_BUFFER       loads through a bounds-checked buffer descriptor per
 *                          workgroup tile (the descriptor-addressed read-only
 *                          path, the analogue of a texture fetch); needs a tile
 *                          of at most 2^31 bytes
 * Centre sources (kmpp_seed_opts.centre_source):
 *   KMPP_CENTRE_LDS        copied once per workgroup into LDS (the default)
 *   KMPP_CENTRE_SCALAR     scalar loads into scalar registers through the
 *                          scalar data cache (the constant-cache analogue)
 *   KMPP_CENTRE_GLOBAL     vector loads by every lane from global memory
 */
enum { KMPP_ROWS_CACHED = 0, KMPP_ROWS_NONTEMPORAL = 1, KMPP_ROWS_BUFFER = 2 };
enum { KMPP_CENTRE_LDS = 1, KMPP_CENTRE_SCALAR = 2, KMPP_CENTRE_GLOBAL = 3 };

/*
 * Where each draw runs (kmpp_seed_opts.draw).  PASS, KERNEL and LEAD follow
 * the same steps in the same order, so for one launch shape they pick the
 * same seeds.
 *   KMPP_DRAW_AUTO    SINGLE where it applies, else PASS where a pass has
 *                     at most 256 tiles, else the tuning table's choice for
 *                     (format, d), else LEAD up to 4096 tiles, else KERNEL
 *   KMPP_DRAW_PASS    every workgroup of pass m+1 draws seed m at its start
 *                     from pass m's D and tile sums (one launch per seed;
 *                     passes then write D and tile sums to alternating
 *                     buffers, every row's D each pass).  Used where it
 *                     applies (unweighted seeding, FP32 rows of any width
 *                     or BF16 / FP8 rows of exact widths, at most 2048
 *                     tiles, the tile sums or one tile's D within the LDS
 *                     share that keeps the pass's occupancy), else KERNEL.
 *   KMPP_DRAW_KERNEL  a one-workgroup draw kernel after each pass (two
 *                     launches per seed; D updated in place where it changed)
 *   KMPP_DRAW_LEAD    workgroup 0 of pass m+1 draws seed m at its start and
 *                     publishes the index; the pass's other workgroups wait
 *                     for it (bounded: KMPP_E_TIMEOUT after one second, see
 *                     kmpp_tune_load; narrow FP32 rows with their first rows
 *                     already in flight).  One launch per seed, D and tile
 *                     sums in place.  The same rows as PASS, unweighted
 *                     seeding; else KERNEL.
 *   KMPP_DRAW_SINGLE  the whole loop (every pass and draw) in one
 *                     1024-thread workgroup with the rows in LDS and D in
 *                     registers: one launch per seeding.  Only for FP32
 *                     rows, unweighted seeding, ceil(N / 1024) * d <= 36
 *                     (so N <= 16384 and N * d <= 36864) and no other
 *                     option set (threads, rows_per_tile,
 *                     loads_per_lane, row_loads, centre_source, out_recheck,
 *                     step_events), else KMPP_E_UNSUPPORTED; KMPP_DRAW_AUTO
 *                     takes it wherever it applies.  Its FP64 partial sums
 *                     run over each thread's rows rather than over tiles, so
 *                     a draw within rounding of a row boundary may differ
 *                     from the other placements'.
 */
enum { KMPP_DRAW_AUTO = 0, KMPP_DRAW_PASS = 1, KMPP_DRAW_KERNEL = 2, KMPP_DRAW_LEAD = 3, KMPP_DRAW_SINGLE = 4 };

/* Optional knobs of kmpp_seed (pass NULL for defaults). */
typedef struct kmpp_seed_opts {
  uint32_t instance;    /* Philox instance id: counter word 1 (default 0) */
  int32_t threads;      /* threads per workgroup of the seed pass: 0 (tuned), 256 or 512 */
  int32_t rows_per_tile;/* rows per workgroup tile: 0 (tuned) or a positive count */
  int16_t loads_per_lane; /* 16-byte row loads in flight per lane: 0 (tuned), 8 or 16 */
  int16_t row_loads;    /* how the passes read the rows: -1 tuned (non-temporal when the rows
                           exceed 256 MiB), KMPP_ROWS_CACHED, KMPP_ROWS_NONTEMPORAL or
                           KMPP_ROWS_BUFFER */
  float* out_recheck;   /* device [K*2] or NULL.  Precision forms: for each draw m >= 1,
                           [2m] = D of the drawn row from the quantised rows before it is
                           committed, [2m+1] = its FP32 nearest distance recomputed from the
                           original FP32 row against the previous seeds. */
  void* step_events;    /* host array of 2K hipEvent_t or NULL: [2m-2] and [2m-1] track the
                           start and the stop of pass m's kernel, its drawer included
                           (profiling only) */
  int32_t centre_source;/* where the passes take the current centre from: 0 (default: LDS),
                           KMPP_CENTRE_LDS, KMPP_CENTRE_SCALAR or KMPP_CENTRE_GLOBAL */
  int32_t draw;         /* KMPP_DRAW_AUTO (0, default), KMPP_DRAW_PASS, KMPP_DRAW_KERNEL,
                           KMPP_DRAW_LEAD or KMPP_DRAW_SINGLE */
  double* out_sumD;     /* device FP64 [K] or NULL: [m] (m >= 1) = the sum of D that draw m
                           inverted (the denominator of P(n_l) in Algorithm 1, summed in
                           FP64 in the fixed tile order); [0] = 0 */
} kmpp_seed_opts;

/*
 * k-means++ seeding (paper, Section II, Algorithms 1 and 2).
 *
 * X            FP32 [N, d]: the points; seeds (centres) are always copied
 *              from these original rows
 * N, d, K      1 <= K <= N <= 2^31 - 1, 1 <= d <= KMPP_MAX_D
 * seed         Philox key
 * out_centers  FP32 [K, d]: the chosen rows, in draw order (required)
 * out_D        FP32 [N] or NULL: the final squared distance of every point to
 *              its nearest seed (the D array lives in the workspace if NULL)
 * out_idx      int64 [K] or NULL: the chosen row indices
 * Xq, Xq_exp   precision forms only (dtype != KMPP_F32): the quantised rows
 *              the distance passes read (BF16 or FP8 [N, d], from
 *              kmpp_quantize) and, for FP8, the int8 [N] row exponents; the
 *              drawn seed's own D is then set to 0, its FP32 distance to
 *              itself; NULL for KMPP_F32
 * opts         NULL or knobs above
 * Returns KMPP_OK or an error from argument checking / launching.
 * Work per call: K passes over the rows, one per seed; pass m < K also draws
 * seed m.
 */
size_t kmpp_seed_workspace_bytes(int64_t N, int32_t d, int32_t K, int32_t dtype);
int kmpp_seed(const float* X, int64_t N, int32_t d, int32_t K, uint64_t seed, float* out_centers,
              float* out_D, int64_t* out_idx, const void* Xq, const int8_t* Xq_exp, int32_t dtype,
              const kmpp_seed_opts* opts, void* workspace, size_t ws_bytes, void* stream);

/*
 * kmpp_seed without a workspace, for callers that cannot allocate device
 * memory (code under graph capture, tight serving loops, harnesses that
 * forbid allocation).  Exported by libkmpp_noalloc.so (linked to
 * libkmpp.so), so that only its callers load its fixed device array.
 * Same arguments, results and launches as kmpp_seed (bit-identical seeds,
 * centres and D), except:
 *   - the workspace is a fixed device array inside the library (about
 *     16 MiB per device, held by every device the library runs on until the
 *     process ends), so N <= KMPP_NOALLOC_MAX_N, else KMPP_E_TOO_LARGE and
 *     nothing is launched; the entry point allocates nothing;
 *   - out_status: device int32 [1] or NULL, receives the status word
 *     (KMPP_OK, KMPP_W_DEGENERATE or KMPP_E_NONFINITE) from the last pass;
 *     kmpp_status does not apply;
 *   - `stream` must belong to the current device (the array used is the
 *     current device's);
 *   - every call on one device shares that device's array: calls that may
 *     overlap on one device (other streams, other threads) race and give
 *     undefined results; order them on one stream.
 */
#define KMPP_NOALLOC_MAX_N 1048576
int kmpp_seed_noalloc(const float* X, int64_t N, int32_t d, int32_t K, uint64_t seed, float* out_centers,
                      float* out_D, int64_t* out_idx, const void* Xq, const int8_t* Xq_exp, int32_t dtype,
                      const kmpp_seed_opts* opts, int32_t* out_status, void* stream);

/*
 * Nearest-seed assignment: the partition O of the paper's Algorithm 1.
 *
 * X            [N, d] rows in `dtype` (FP32, BF16 or FP8 with X_exp)
 * C            FP32 [K, d] seeds
 * out_labels   int32 [N]: index of the nearest seed; ties -> smallest index;
 *              -1 for a row with no comparable distance (NaN in the row)
 * out_mind     FP32 [N] or NULL: squared distance to that seed, direct form
 * Scores ||c||^2 - 2<x,c> come from matrix-core products with FP32
 * accumulation; rows whose best and second-best scores are closer than the
 * product's error bound are re-evaluated in the direct FP32 form.
 * Distances use the dequantised rows for BF16/FP8.
 */
size_t kmpp_assign_workspace_bytes(int64_t N, int32_t d, int32_t K, int32_t dtype);
int kmpp_assign(const void* X, const int8_t* X_exp, int32_t dtype, const float* C, int64_t N, int32_t d,
                int32_t K, int32_t* out_labels, float* out_mind, void* workspace, size_t ws_bytes,
                void* stream);

/*
 * k-means|| initialisation (Bahmani, Moseley, Vattani, Kumar, Vassilvitskii,
 * "Scalable K-Means++", PVLDB 2012, Algorithm 2), the different
 * initialisation the paper's introduction attributes to Bahmani et al.
 * A uniform first point; `rounds` rounds in which every point joins the
 * candidate list independently with probability min(1, ell * D / phi)
 * (D: squared distance to the nearest candidate, phi = sum D in FP64);
 * candidate weights = points whose nearest candidate it is (ties to the
 * smaller candidate index); then weighted k-means++ over the candidates
 * (first centre proportional to w, then to w * D) gives the K centres.
 * Philox4x32-10 keyed by `seed`, counters (0, instance, 0, 0) for the
 * first point, (i, instance, r, 1) for point i in round r = 1..rounds and
 * (m, instance, 0, 2) for the m-th recluster draw.
 *
 * X             FP32 [N, d], 16-byte aligned, d <= KMPP_MAX_D, N <= 2^31 - 1
 * rounds        0..64; ell > 0 (typically 2K)
 * out_centers   FP32 [K, d]: the chosen points, in draw order (required)
 * out_idx       int64 [K] or NULL: their point indices
 * out_cand      int64 [cap] or NULL: the candidates' point indices, in the
 *               order they joined (within a round in point order);
 *               cap = kmpp_seed_parallel_capacity(N, rounds, ell)
 *               = min(N, 1 + rounds * (3 ceil(ell) + 64))
 * out_round_end int32 [rounds + 1] or NULL: list length after the first
 *               point and after each round
 * out_weights   int32 [cap] or NULL: candidate weights (the first
 *               round_end[rounds] entries are valid)
 * out_labels    int32 [N] or NULL: every point's nearest candidate
 * Device status (kmpp_status): KMPP_W_DEGENERATE when a recluster draw found
 * every weighted distance zero (fewer than K distinct candidates),
 * KMPP_E_NONFINITE for NaN/Inf, KMPP_E_WORKSPACE when more than cap points
 * joined (the list is cut at cap; vanishingly unlikely: a round's expected
 * number of joiners is at most ell).
 * Synchronises `stream` once per round (the host reads the list length to
 * size the next round's assignment), so it cannot be captured in a graph.
 */
int32_t kmpp_seed_parallel_capacity(int64_t N, int32_t rounds, double ell);
size_t kmpp_seed_parallel_workspace_bytes(int64_t N, int32_t d, int32_t K, int32_t rounds, double ell);
int kmpp_seed_parallel(const float* X, int64_t N, int32_t d, int32_t K, uint64_t seed, int32_t rounds, double ell,
                       uint32_t instance, float* out_centers, int64_t* out_idx, int64_t* out_cand,
                       int32_t* out_round_end, int32_t* out_weights, int32_t* out_labels, void* workspace,
                       size_t ws_bytes, void* stream);

/*
 * Lloyd iterations after seeding.  Section II: once the initial centroids
 * are chosen, the clustering proceeds as standard k-means, whose result is
 * the partition O of Algorithm 1.  One iteration assigns every row to its
 * nearest centre (the kmpp_assign rule) and then moves every centre to the
 * mean of its rows; a centre with no rows keeps its position.
 *
 * X, X_exp, dtype  rows as for kmpp_assign (means of the dequantised rows)
 * C                FP32 [K, d], 16-byte aligned, in/out: the starting
 *                  centres (e.g. kmpp_seed's out_centers), replaced by the
 *                  centres after `iters` updates
 * iters            >= 0 iterations, all enqueued (no host synchronisation)
 * out_labels       int32 [N]: the last iteration's assignment (against the
 *                  centres before its update; call kmpp_assign on the final
 *                  C for labels that match it)
 * out_cost         FP64 [iters] or NULL: sum over rows of the squared
 *                  distance to the assigned centre, per iteration
 * out_changed      int64 [iters] or NULL: rows whose label differs from the
 *                  previous iteration (N in the first)
 * out_counts       int32 [K] or NULL: cluster sizes of the last assignment
 * Means are FP64 divisions of 64-bit fixed-point cluster sums (scale 2^F,
 * F = 62 - e - ceil(log2 N), max|x| < 2^e), rounded to FP32: every run
 * gives the same bits.  Device status (kmpp_status on this workspace):
 * KMPP_E_NONFINITE if X holds NaN or Inf.
 */
size_t kmpp_lloyd_workspace_bytes(int64_t N, int32_t d, int32_t K, int32_t dtype);
int kmpp_lloyd(const void* X, const int8_t* X_exp, int32_t dtype, int64_t N, int32_t d, int32_t K, float* C,
               int32_t iters, int32_t* out_labels, double* out_cost, int64_t* out_changed, int32_t* out_counts,
               void* workspace, size_t ws_bytes, void* stream);

/*
 * Storage formats for the precision forms.
 * KMPP_BF16:     Xq uint16 [N, d] = bf16(X), round to nearest even; Xq_exp unused (NULL)
 * KMPP_FP8_E4M3: e_i = smallest integer e with max_j |X_ij| <= 448 * 2^e (0 for an
 *                all-zero row), clamped to [-117, 127]; Xq_exp int8 [N] = e_i;
 *                Xq uint8 [N, d] = E4M3FN(X_ij * 2^-e_i), round to nearest even.
 * Dequantised values (q * 2^e) are exact in FP32.
 */
int kmpp_quantize(const float* X, int64_t N, int32_t d, int32_t dtype, void* Xq, int8_t* Xq_exp,
                  void* stream);

/* One independent seeding instance of the batched form.  The last three
 * fields choose the rows the passes stream, as kmpp_seed's dtype, Xq and
 * Xq_exp do (zero / NULL: the FP32 rows X); the centres are always the
 * original FP32 rows of X, and with BF16 / FP8 rows each drawn row's D is
 * set to 0. */
typedef struct kmpp_instance {
  const float* X;       /* FP32 [N, d], 16-byte aligned */
  int64_t N;
  int32_t d;
  int32_t K;
  float* out_centers;   /* FP32 [K, d] */
  float* out_D;         /* FP32 [N] or NULL */
  int64_t* out_idx;     /* int64 [K] or NULL */
  int32_t dtype;        /* KMPP_F32, KMPP_BF16 or KMPP_FP8_E4M3 */
  const void* Xq;       /* BF16 / FP8 rows [N, d] (kmpp_quantize), 16-byte aligned, or NULL for KMPP_F32 */
  const int8_t* Xq_exp; /* FP8 row exponents [N], or NULL */
} kmpp_instance;

/*
 * Batched form: n_inst independent seedings (instance b uses Philox
 * instance id b) run by ONE persistent kernel.  Each instance is handled by
 * a gang of workgroups (one workgroup for small instances) that meets at a
 * device-side barrier per seed; gangs are scheduled longest-first by a
 * host planner onto the co-resident workgroups.
 *
 * inst         HOST array [n_inst]; every instance of one batch has the same
 *              dtype (one launch streams one row format), else
 *              KMPP_E_UNSUPPORTED (and a workspace size of 0)
 * kmpp_seed_batched_prepare: plans the schedule and uploads the descriptor
 *              table into the workspace (a synchronous host-to-device copy);
 * kmpp_seed_batched_launch:  enqueues only kernel launches and so may be
 *              captured into a graph and replayed;
 * kmpp_seed_batched:         prepare + launch.
 * Status: KMPP_W_DEGENERATE or KMPP_E_NONFINITE as for kmpp_seed (for the
 * whole batch: some instance met the condition), KMPP_E_TIMEOUT if a gang
 * barrier wait expired (results undefined; the budget scales with the plan's
 * estimated length, see kmpp_tune_load).
 */
size_t kmpp_batched_workspace_bytes(const kmpp_instance* inst, int32_t n_inst);
int kmpp_seed_batched_prepare(const kmpp_instance* inst, int32_t n_inst, uint64_t seed, void* workspace,
                              size_t ws_bytes, void* stream);
int kmpp_seed_batched_launch(void* workspace, void* stream);
int kmpp_seed_batched(const kmpp_instance* inst, int32_t n_inst, uint64_t seed, void* workspace,
                      size_t ws_bytes, void* stream);

/* Status word written by the device (KMPP_OK, KMPP_W_DEGENERATE,
 * KMPP_E_NONFINITE, KMPP_E_TIMEOUT, KMPP_E_WORKSPACE).  Synchronises
 * `stream`, then copies the word of `workspace` (as passed to kmpp_seed,
 * kmpp_seed_batched, kmpp_lloyd or kmpp_seed_parallel) into *out.  Returns
 * KMPP_OK or KMPP_E_HIP. */
int kmpp_status(const void* workspace, void* stream, int32_t* out);
/* The same word without synchronising any stream, for a caller that has
 * already waited for the work that wrote it (the copy itself is a plain
 * blocking device-to-host copy).  Returns KMPP_OK, KMPP_E_INVALID or
 * KMPP_E_HIP. */
int kmpp_status_poll(const void* workspace, int32_t* out);

/* Graph capture helpers: capture the work a sequence of calls enqueues on
 * `stream` into an executable HIP graph and replay it.  The captured calls
 * must not be _prepare calls. */
typedef struct kmpp_graph_s* kmpp_graph;
int kmpp_graph_begin(void* stream);
int kmpp_graph_end(void* stream, kmpp_graph* out);
int kmpp_graph_launch(kmpp_graph g, void* stream);
int kmpp_graph_destroy(kmpp_graph g);

/* Tuning table: text lines
 * "seed <dtype> <d> <threads> <rows_per_tile> [<loads_per_lane> <row path> [<draw>]]"
 * override the built-in choices for the seed pass (draw: KMPP_DRAW_PASS,
 * KMPP_DRAW_KERNEL or KMPP_DRAW_LEAD); lines
 * "batched <key> <value>" (keys wg_per_cu, chip_gbs, sync1_us, syncw_us,
 * alpha) set the batched planner's cost model; "batched wait_ms <v>" sets
 * the budget of one gang wait (v < 0: automatic, eight times the plan's
 * estimated length and at least one second; 0: every wait gives up at once,
 * which forces KMPP_E_TIMEOUT for testing); "lead wait_ms <v>" sets the
 * budget of a pass's wait for the lead workgroup's index (KMPP_DRAW_LEAD;
 * v < 0: one second, the default; 0: every wait gives up at once, which
 * forces KMPP_E_TIMEOUT for testing).  Returns the number of entries read or
 * KMPP_E_INVALID. */
int kmpp_tune_load(const char* path);

/*
 * Read-bandwidth probe (a measurement helper, not part of the method): reads
 * `bytes` of device memory at `buf` once (grid-stride over `blocks`
 * workgroups of 256 threads, 8 16-byte loads per lane in flight, cached or
 * non-temporal loads) and writes the FP32 sum of the floats each workgroup
 * read to out_partial[blocks] (device).  Timing it gives the attainable read
 * bandwidth that the seed pass's rate is compared with.  buf 16-byte
 * aligned, bytes a positive multiple of 16, 1 <= blocks <= 65536,
 * nontemporal 0 or 1, else KMPP_E_INVALID.  Asynchronous on `stream`.
 */
int kmpp_read_probe(const void* buf, size_t bytes, int32_t blocks, int32_t nontemporal, float* out_partial,
                    void* stream);

const char* kmpp_strerror(int code);
int kmpp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* KMPP_H_ */
