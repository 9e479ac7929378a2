/*
 * kmpp_oracle.c -- plain FP64 CPU oracle for k-means++ seeding and the
 * nearest-seed assignment that follows it.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or constant table
 * with the HIP library; both sides implement the method from the paper
 * ("Parallelization of Kmeans++ using CUDA", arXiv 1908.02136) and the
 * counter-based generator from its published definition.
 *
 * What it computes (paper, Section II, Algorithm 1 "Serial K-means++" and
 * Algorithm 2 "Parallel K-means++"):
 *   - the first seed is a uniformly random point;
 *   - every point keeps the squared distance to its nearest chosen seed,
 *     initialised to +infinity (O(l) = inf in Algorithm 1);
 *   - each further seed is point l with probability d_sn(l) / sum_w d_sn(w)
 *     (the P(n_l) line of Algorithm 1);
 *   - the sum over all points is taken in double precision (Section II,
 *     the thrust::reduce paragraph).
 * Readings where the paper is silent (all listed in the design notes):
 *   - the random stream is Philox4x32-10 (Salmon et al., SC'11) with
 *     key = (lo32(seed), hi32(seed)) and counter = (step, instance, 0, 0);
 *   - u = ((r0 >> 5) * 2^26 + (r1 >> 6)) * 2^-53, a 53-bit uniform in [0,1);
 *   - first seed i0 = min(floor(u0 * N), N - 1);
 *   - the draw is the inverse CDF over points in index order:
 *     t = u_m * S_{N-1}, i_m = min { i : S_i > t } with S the inclusive
 *     prefix sum of D; if rounding leaves no such i, the last i with D_i > 0;
 *   - sum D == 0 (fewer than K distinct points): uniform draw, warning code;
 *   - non-finite sum D: error code;
 *   - the nearest distance is kept incrementally, D = min(D, delta), which
 *     equals the paper's recompute-over-all-seeds minimum exactly;
 *   - precision forms: distances use the dequantised rows, centres are the
 *     original FP32 rows, and the chosen seed's own D is set to its FP32
 *     distance to itself, zero.
 * Everything is FP64; the prefix is summed sequentially in index order in
 * fixed 65536-row chunks so the result does not depend on thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define KMO_OK 0
#define KMO_W_DEGENERATE 1
#define KMO_E_INVALID (-1)
#define KMO_E_NONFINITE (-4)
#define KMO_CHUNK 65536

/* ---- Philox4x32-10, from Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3" (SC'11), Section 5: four 32-bit words, two
 * 32x32->64 multiplications per round, Weyl-sequence key schedule. ---- */
static void kmo_philox_round(uint32_t x[4], const uint32_t k[2]) {
  const uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)x[0];
  const uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)x[2];
  const uint32_t y0 = (uint32_t)(pb >> 32) ^ x[1] ^ k[0];
  const uint32_t y1 = (uint32_t)pb;
  const uint32_t y2 = (uint32_t)(pa >> 32) ^ x[3] ^ k[1];
  const uint32_t y3 = (uint32_t)pa;
  x[0] = y0;
  x[1] = y1;
  x[2] = y2;
  x[3] = y3;
}

void kmo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k[0] += 0x9E3779B9u;
      k[1] += 0xBB67AE85u;
    }
    kmo_philox_round(x, k);
  }
  memcpy(out, x, sizeof(x));
}

/* 53-bit uniform in [0, 1) for seeding step `step` of instance `inst`. */
double kmo_uniform(uint64_t seed, uint32_t step, uint32_t inst) {
  const uint32_t ctr[4] = {step, inst, 0u, 0u};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t r[4];
  kmo_philox4x32_10(ctr, key, r);
  const uint64_t hi = (uint64_t)(r[0] >> 5);
  const uint64_t lo = (uint64_t)(r[1] >> 6);
  return (double)(hi * 67108864ull + lo) / 9007199254740992.0; /* / 2^53 */
}

static int kmo_threads(int32_t nthreads) {
#ifdef _OPENMP
  return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

/* delta = sum_j (a_j - c_j)^2 in FP64, summed in j order. */
static double kmo_sqdist(const float* a, const double* c, int32_t d) {
  double s = 0.0;
  for (int32_t j = 0; j < d; ++j) {
    const double t = (double)a[j] - c[j];
    s += t * t;
  }
  return s;
}

/* Inclusive prefix S of D (FP64), chunked sequential sum; returns S[N-1]. */
static double kmo_prefix(const double* D, double* S, double* chunk, int64_t N, int nt) {
  const int64_t nch = (N + KMO_CHUNK - 1) / KMO_CHUNK;
#pragma omp parallel for schedule(static) num_threads(nt)
  for (int64_t q = 0; q < nch; ++q) {
    const int64_t a = q * KMO_CHUNK, b = (a + KMO_CHUNK < N) ? a + KMO_CHUNK : N;
    double s = 0.0;
    for (int64_t i = a; i < b; ++i) s += D[i];
    chunk[q] = s;
  }
  double run = 0.0;
  for (int64_t q = 0; q < nch; ++q) {
    const double v = chunk[q];
    chunk[q] = run; /* exclusive */
    run += v;
  }
#pragma omp parallel for schedule(static) num_threads(nt)
  for (int64_t q = 0; q < nch; ++q) {
    const int64_t a = q * KMO_CHUNK, b = (a + KMO_CHUNK < N) ? a + KMO_CHUNK : N;
    double s = chunk[q];
    for (int64_t i = a; i < b; ++i) {
      s += D[i];
      S[i] = s;
    }
  }
  return S[N - 1];
}

/* first i with S[i] > t (S non-decreasing); N if none. */
int64_t kmo_upper_bound(const double* S, int64_t N, double t) {
  int64_t lo = 0, hi = N;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (S[mid] > t)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

static int64_t kmo_uniform_index(double u, int64_t N) {
  int64_t i = (int64_t)floor(u * (double)N);
  return i > N - 1 ? N - 1 : i;
}

/*
 * One draw of Algorithm 1 (the P(n_l) line with the readings above) on the
 * current D: S = inclusive FP64 prefix of D in index order (fixed chunks),
 * T = S_{N-1}, t = u * T (one IEEE multiply), i = min { i : S_i > t }; if
 * no such i exists (t >= S_{N-1}), the last i with D_i > 0.  T == 0: the
 * uniform index and KMO_W_DEGENERATE; T not finite: KMO_E_NONFINITE (no
 * index).  *T_out, *t_out receive T and t.
 */
static int kmo_draw_on(const double* D, double* S, double* chunk, int64_t N, double u, int nt, int64_t* out_i,
                       double* T_out, double* t_out) {
  const double T = kmo_prefix(D, S, chunk, N, nt);
  volatile double tv = u * T; /* one IEEE multiply */
  const double t = tv;
  *T_out = T;
  *t_out = t;
  if (!isfinite(T)) return KMO_E_NONFINITE;
  if (T == 0.0) {
    *out_i = kmo_uniform_index(u, N);
    return KMO_W_DEGENERATE;
  }
  int64_t i = kmo_upper_bound(S, N, t);
  if (i >= N) { /* t >= S_{N-1}: the last positive D */
    i = N - 1;
    while (i > 0 && !(D[i] > 0.0)) --i;
  }
  *out_i = i;
  return KMO_OK;
}

/*
 * The draw alone, with u given: for checking the inverse-CDF rule, its
 * boundaries and its fallbacks directly.  rec4 (nullable): T, t, S_{i-1},
 * S_i (S_{i-1} = 0 for i = 0; NaN where there is no index).  Returns
 * KMO_OK, KMO_W_DEGENERATE, KMO_E_NONFINITE or KMO_E_INVALID.
 */
int kmo_draw(const double* D, int64_t N, double u, int64_t* out_i, double* rec4, int32_t nthreads) {
  if (!D || !out_i || N < 1) return KMO_E_INVALID;
  const int nt = kmo_threads(nthreads);
  double* S = (double*)malloc(sizeof(double) * (size_t)N);
  double* chunk = (double*)malloc(sizeof(double) * (size_t)((N + KMO_CHUNK - 1) / KMO_CHUNK));
  if (!S || !chunk) {
    free(S);
    free(chunk);
    return KMO_E_INVALID;
  }
  double T, t;
  int64_t i = -1;
  const int st = kmo_draw_on(D, S, chunk, N, u, nt, &i, &T, &t);
  *out_i = i;
  if (rec4) {
    rec4[0] = T;
    rec4[1] = t;
    rec4[2] = (i > 0 && i < N) ? S[i - 1] : (i == 0 ? 0.0 : NAN);
    rec4[3] = (i >= 0 && i < N) ? S[i] : NAN;
  }
  free(S);
  free(chunk);
  return st;
}

/*
 * k-means++ seeding, Algorithm 1 with the readings above, passes
 * m_begin..m_end (1 <= m_begin <= m_end <= K) of a run: pass m moves every
 * D to its distance to seed m-1 if that is smaller (pass 1 replaces the
 * initial +infinity), and for m < K draws seed m.  D must hold the state
 * after pass m_begin - 1 (anything for m_begin = 1) and out_idx[0..m_begin-1]
 * the earlier seeds (the first seed is drawn here when m_begin = 1).  A run
 * split into consecutive ranges computes exactly what one range computes.
 *
 * Xd     [N*d] values distances are computed from (FP32 data or dequantised rows)
 * Xc     [N*d] values the centres take (FP32 data); may equal Xd
 * zero_seed_rows  1 for the precision forms: D of the chosen row := 0
 * replay [K] or NULL: if given, the centre used after step m is replay[m]
 *        (the GPU's index), while out_idx[m] is still the oracle's own
 *        draw from the same D; this checks each draw independently.
 * out_idx [K]   the oracle's draws
 * D       [N]   nearest squared distance (FP64), in and out
 * rec     [K*8] or NULL, per step m >= 1:
 *        T, t, S_{i-1}, S_i (oracle's own i), S_{g-1}, S_g, D_g (g = replay[m],
 *        or the oracle's own index without replay), u
 * Returns 0, KMO_W_DEGENERATE (some draw in the range was degenerate), or a
 * negative error.
 */
int kmo_seed_range(const float* Xd, const float* Xc, int64_t N, int32_t d, int32_t K, uint64_t seed,
                   uint32_t inst, int32_t zero_seed_rows, const int64_t* replay, int32_t m_begin, int32_t m_end,
                   int64_t* out_idx, double* D, double* rec, int32_t nthreads) {
  if (!Xd || !Xc || !out_idx || !D || N < 1 || d < 1 || K < 1 || K > N) return KMO_E_INVALID;
  if (m_begin < 1 || m_end < m_begin || m_end > K) return KMO_E_INVALID;
  const int nt = kmo_threads(nthreads);
  const int64_t nch = (N + KMO_CHUNK - 1) / KMO_CHUNK;
  double* S = (double*)malloc(sizeof(double) * (size_t)N);
  double* chunk = (double*)malloc(sizeof(double) * (size_t)nch);
  double* c = (double*)malloc(sizeof(double) * (size_t)d);
  if (!S || !chunk || !c) {
    free(S);
    free(chunk);
    free(c);
    return KMO_E_INVALID;
  }
  int status = KMO_OK;

  if (m_begin == 1) out_idx[0] = kmo_uniform_index(kmo_uniform(seed, 0u, inst), N);
  int64_t prev = replay ? replay[m_begin - 1] : out_idx[m_begin - 1];
  if (prev < 0 || prev >= N) status = KMO_E_INVALID;

  for (int32_t m = m_begin; m <= m_end && status >= 0; ++m) {
    /* centre c_{m-1}: the original row of the previous seed */
    for (int32_t j = 0; j < d; ++j) c[j] = (double)Xc[prev * (int64_t)d + j];
    /* D_i = min(D_i, ||x_i - c||^2); the first pass replaces +inf */
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t i = 0; i < N; ++i) {
      const double delta = kmo_sqdist(Xd + i * (int64_t)d, c, d);
      D[i] = (m == 1 || delta < D[i]) ? delta : D[i];
    }
    if (zero_seed_rows) D[prev] = 0.0;
    if (m == K) break;

    const double u = kmo_uniform(seed, (uint32_t)m, inst);
    double T, t;
    int64_t i = -1;
    const int st = kmo_draw_on(D, S, chunk, N, u, nt, &i, &T, &t);
    if (st < 0) {
      status = st;
      break;
    }
    if (st == KMO_W_DEGENERATE) status = KMO_W_DEGENERATE;
    out_idx[m] = i;
    const int64_t g = replay ? replay[m] : i;
    if (rec) {
      double* r = rec + (size_t)m * 8;
      r[0] = T;
      r[1] = t;
      r[2] = i > 0 ? S[i - 1] : 0.0;
      r[3] = S[i];
      r[4] = (g > 0 && g < N) ? S[g - 1] : 0.0;
      r[5] = (g >= 0 && g < N) ? S[g] : NAN;
      r[6] = (g >= 0 && g < N) ? D[g] : NAN;
      r[7] = u;
    }
    if (g < 0 || g >= N) {
      status = KMO_E_INVALID;
      break;
    }
    prev = g;
  }
  free(S);
  free(chunk);
  free(c);
  return status;
}

/* The whole run (passes 1..K); out_D receives the final D. */
int kmo_seed(const float* Xd, const float* Xc, int64_t N, int32_t d, int32_t K, uint64_t seed,
             uint32_t inst, int32_t zero_seed_rows, const int64_t* replay, int64_t* out_idx,
             double* out_D, double* rec, int32_t nthreads) {
  return kmo_seed_range(Xd, Xc, N, d, K, seed, inst, zero_seed_rows, replay, 1, K, out_idx, out_D, rec, nthreads);
}

/* Nearest-seed assignment (output O of Algorithm 1): label = smallest j
 * attaining min_j ||x_i - c_j||^2, all in FP64.  mind/second nullable. */
int kmo_assign(const float* X, int64_t N, int32_t d, const float* C, int32_t K, int32_t* labels,
               double* mind, double* second, int32_t nthreads) {
  if (!X || !C || !labels || N < 0 || d < 1 || K < 1) return KMO_E_INVALID;
  const int nt = kmo_threads(nthreads);
#pragma omp parallel num_threads(nt)
  {
    double* c = (double*)malloc(sizeof(double) * (size_t)d);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
      double best = INFINITY, sec = INFINITY;
      int32_t bj = 0;
      for (int32_t j = 0; j < K; ++j) {
        for (int32_t q = 0; q < d; ++q) c[q] = (double)C[(int64_t)j * d + q];
        const double v = kmo_sqdist(X + i * (int64_t)d, c, d);
        if (v < best) {
          sec = best;
          best = v;
          bj = j;
        } else if (v < sec) {
          sec = v;
        }
      }
      labels[i] = bj;
      if (mind) mind[i] = best;
      if (second) second[i] = sec;
    }
    free(c);
  }
  return KMO_OK;
}

/* For sampled checks at full size: FP64 min distance and label of the rows
 * listed in `rows` against K centres. */
int kmo_assign_rows(const float* X, int32_t d, const int64_t* rows, int64_t nrows, const float* C,
                    int32_t K, int32_t* labels, double* mind, double* second) {
  if (!X || !C || !rows || !labels || !mind || d < 1 || K < 1) return KMO_E_INVALID;
  double* c = (double*)malloc(sizeof(double) * (size_t)d);
  for (int64_t r = 0; r < nrows; ++r) {
    double best = INFINITY, sec = INFINITY;
    int32_t bj = 0;
    for (int32_t j = 0; j < K; ++j) {
      for (int32_t q = 0; q < d; ++q) c[q] = (double)C[(int64_t)j * d + q];
      const double v = kmo_sqdist(X + rows[r] * (int64_t)d, c, d);
      if (v < best) {
        sec = best;
        best = v;
        bj = j;
      } else if (v < sec) {
        sec = v;
      }
    }
    labels[r] = bj;
    mind[r] = best;
    if (second) second[r] = sec;
  }
  free(c);
  return KMO_OK;
}

/* FP64 squared distance of listed rows to one listed centre each. */
int kmo_pair_dist(const float* X, int32_t d, const int64_t* rows, int64_t nrows, const float* C,
                  const int32_t* cols, double* out) {
  if (!X || !C || !rows || !cols || !out || d < 1) return KMO_E_INVALID;
  double* c = (double*)malloc(sizeof(double) * (size_t)d);
  for (int64_t r = 0; r < nrows; ++r) {
    for (int32_t q = 0; q < d; ++q) c[q] = (double)C[(int64_t)cols[r] * d + q];
    out[r] = kmo_sqdist(X + rows[r] * (int64_t)d, c, d);
  }
  free(c);
  return KMO_OK;
}

/* ---- storage formats for the precision forms ----
 * BF16: the upper half of an IEEE binary32, rounded to nearest, ties to an
 * even last mantissa bit.  Written from that definition: the two bf16
 * neighbours of x are compared in FP64. */
static float kmo_bits_to_float(uint32_t b) {
  float f;
  memcpy(&f, &b, 4);
  return f;
}
static uint32_t kmo_float_to_bits(float f) {
  uint32_t b;
  memcpy(&b, &f, 4);
  return b;
}

uint16_t kmo_bf16_encode(float x) {
  const uint32_t b = kmo_float_to_bits(x);
  if (isnan(x)) return (uint16_t)((b >> 16) | 0x0040u);
  const uint32_t lo = b & 0xFFFF0000u;        /* truncation toward zero */
  if ((b & 0xFFFFu) == 0) return (uint16_t)(lo >> 16);
  const uint32_t hi = lo + 0x00010000u;       /* next magnitude up */
  const double dx = fabs((double)x);
  const double dlo = fabs((double)kmo_bits_to_float(lo));
  double dhi = fabs((double)kmo_bits_to_float(hi));
  if (isinf(kmo_bits_to_float(hi))) dhi = 3.402823669209385e38; /* 2^128, the overflow point */
  const double elo = dx - dlo, ehi = dhi - dx;
  if (elo < ehi) return (uint16_t)(lo >> 16);
  if (ehi < elo) return (uint16_t)(hi >> 16);
  return (uint16_t)(((lo >> 16) & 1u) ? (hi >> 16) : (lo >> 16));
}

float kmo_bf16_decode(uint16_t h) { return kmo_bits_to_float((uint32_t)h << 16); }

void kmo_bf16_encode_n(const float* x, int64_t n, uint16_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = kmo_bf16_encode(x[i]);
}
void kmo_bf16_decode_n(const uint16_t* h, int64_t n, float* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = kmo_bf16_decode(h[i]);
}

/* FP8 E4M3 "FN" (OCP 8-bit floating point specification): sign, 4-bit
 * exponent with bias 7, 3-bit mantissa; exponent field 0 encodes subnormals
 * m * 2^-9; S.1111.111 is NaN; there are no infinities; the largest finite
 * magnitude is 1.75 * 2^8 = 448. */
double kmo_fp8_decode(uint8_t q) {
  const int s = q >> 7, e = (q >> 3) & 15, m = q & 7;
  double v;
  if (e == 15 && m == 7)
    return NAN;
  else if (e == 0)
    v = ldexp((double)m, -9);
  else
    v = ldexp(1.0 + m / 8.0, e - 7);
  return s ? -v : v;
}

/* nearest finite E4M3FN value, ties to even mantissa, saturating at 448:
 * a direct search over the 127 non-negative finite codes. */
uint8_t kmo_fp8_encode(double v) {
  if (isnan(v)) return 0x7F;
  const uint8_t sign = (v < 0 || (v == 0 && signbit(v))) ? 0x80 : 0x00;
  const double a = fabs(v);
  int best = 0;
  double berr = INFINITY;
  for (int c = 0; c < 127; ++c) {
    const double err = fabs(kmo_fp8_decode((uint8_t)c) - a);
    if (err < berr || (err == berr && (c & 1) == 0 && (best & 1) == 1)) {
      berr = err;
      best = c;
    }
  }
  return (uint8_t)(sign | best);
}

/* The same nearest-code rule by bisection over the ascending table of the
 * 127 non-negative finite codes (code c has value fp8_decode(c), increasing
 * in c): the two neighbours of |v| are compared, ties go to the even code.
 * Used for large inputs; equal to kmo_fp8_encode everywhere (tested). */
static double kmo_fp8_table[127];
static int kmo_fp8_table_ready = 0;

uint8_t kmo_fp8_encode_bisect(double v) {
  if (!kmo_fp8_table_ready) {
    for (int c = 0; c < 127; ++c) kmo_fp8_table[c] = kmo_fp8_decode((uint8_t)c);
    kmo_fp8_table_ready = 1;
  }
  if (isnan(v)) return 0x7F;
  const uint8_t sign = (v < 0 || (v == 0 && signbit(v))) ? 0x80 : 0x00;
  const double a = fabs(v);
  if (a >= kmo_fp8_table[126]) return (uint8_t)(sign | 126);
  int lo = 0, hi = 126; /* table[lo] <= a < table[hi] */
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (kmo_fp8_table[mid] <= a)
      lo = mid;
    else
      hi = mid;
  }
  const double elo = a - kmo_fp8_table[lo], ehi = kmo_fp8_table[hi] - a;
  int c = elo < ehi ? lo : (ehi < elo ? hi : ((lo & 1) == 0 ? lo : hi));
  return (uint8_t)(sign | c);
}

/* Per-row power-of-two scale: e_i = smallest integer e with
 * amax_i <= 448 * 2^e (e_i = 0 for an all-zero row), clamped to
 * [-117, 127]; q = E4M3(x / 2^e_i).
 * The scale is a power of two, so x / 2^e is exact and q * 2^e is exact in
 * FP32. */
int32_t kmo_fp8_row_exponent(const float* row, int32_t d) {
  double amax = 0.0;
  for (int32_t j = 0; j < d; ++j) {
    const double a = fabs((double)row[j]);
    if (a > amax) amax = a;
  }
  if (amax == 0.0 || !isfinite(amax)) return 0;
  int e = -160;
  while (amax > ldexp(448.0, e)) ++e;
  /* keep 2^e and the smallest dequantised step (2^(e-9)) normal in FP32 */
  if (e < -117) e = -117;
  if (e > 127) e = 127;
  return e;
}

void kmo_fp8_quantize_rows(const float* X, int64_t N, int32_t d, uint8_t* q, int8_t* ex) {
  for (int64_t i = 0; i < N; ++i) {
    const int32_t e = kmo_fp8_row_exponent(X + i * (int64_t)d, d);
    ex[i] = (int8_t)e;
    for (int32_t j = 0; j < d; ++j) q[i * (int64_t)d + j] = kmo_fp8_encode(ldexp((double)X[i * (int64_t)d + j], -e));
  }
}

/* Same as kmo_fp8_quantize_rows with the bisection encoder, rows in
 * parallel; for the full-size workloads. */
void kmo_fp8_quantize_rows_fast(const float* X, int64_t N, int32_t d, uint8_t* q, int8_t* ex, int32_t nthreads) {
  const int nt = kmo_threads(nthreads);
  kmo_fp8_encode_bisect(0.0); /* fill the table before the parallel region */
#pragma omp parallel for schedule(static) num_threads(nt)
  for (int64_t i = 0; i < N; ++i) {
    const int32_t e = kmo_fp8_row_exponent(X + i * (int64_t)d, d);
    ex[i] = (int8_t)e;
    for (int32_t j = 0; j < d; ++j)
      q[i * (int64_t)d + j] = kmo_fp8_encode_bisect(ldexp((double)X[i * (int64_t)d + j], -e));
  }
}

void kmo_fp8_dequantize_rows(const uint8_t* q, const int8_t* ex, int64_t N, int32_t d, float* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i)
    for (int32_t j = 0; j < d; ++j)
      out[i * (int64_t)d + j] = (float)ldexp(kmo_fp8_decode(q[i * (int64_t)d + j]), ex[i]);
}

/* ---- Lloyd iterations after seeding.  Section II says that once the
 * initial centroids are chosen the clustering proceeds as in standard
 * k-means; the output O of Algorithm 1 is the partition.  One iteration:
 *   1. every point takes its nearest centre (kmo_assign's rule, ties to the
 *      smallest index), and the cost is sum_i min_j ||x_i - c_j||^2;
 *   2. every centre moves to the mean of its points.
 * Readings: a centre with no points keeps its position; the mean is the
 * FP64 sum in point-index order divided by the count, rounded to FP32 (the
 * centres are FP32 arrays); the number of points whose label changed is
 * counted against the previous iteration (all N in the first). */
int kmo_lloyd_update(const float* X, int64_t N, int32_t d, const int32_t* labels, int32_t K, const float* C_prev,
                     float* C_out, int64_t* counts) {
  if (!X || !labels || !C_prev || !C_out || N < 0 || d < 1 || K < 1) return KMO_E_INVALID;
  double* sum = (double*)calloc((size_t)K * (size_t)d, sizeof(double));
  int64_t* n = (int64_t*)calloc((size_t)K, sizeof(int64_t));
  if (!sum || !n) {
    free(sum);
    free(n);
    return KMO_E_INVALID;
  }
  for (int64_t i = 0; i < N; ++i) {
    const int32_t j = labels[i];
    if (j < 0 || j >= K) {
      free(sum);
      free(n);
      return KMO_E_INVALID;
    }
    n[j] += 1;
    for (int32_t q = 0; q < d; ++q) sum[(int64_t)j * d + q] += (double)X[i * (int64_t)d + q];
  }
  for (int32_t j = 0; j < K; ++j) {
    for (int32_t q = 0; q < d; ++q) {
      const int64_t e = (int64_t)j * d + q;
      C_out[e] = n[j] > 0 ? (float)(sum[e] / (double)n[j]) : C_prev[e];
    }
    if (counts) counts[j] = n[j];
  }
  free(sum);
  free(n);
  return KMO_OK;
}

/* `iters` iterations from the centres in C (updated in place).  labels: the
 * last iteration's assignment (against the centres before its update);
 * cost[t], changed[t]: of iteration t's assignment (nullable). */
int kmo_lloyd(const float* X, int64_t N, int32_t d, int32_t K, float* C, int32_t iters, int32_t* labels,
              double* cost, int64_t* changed, int32_t nthreads) {
  if (!X || !C || !labels || N < 1 || d < 1 || K < 1 || iters < 0) return KMO_E_INVALID;
  double* mind = (double*)malloc(sizeof(double) * (size_t)N);
  int32_t* prev = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  float* Cn = (float*)malloc(sizeof(float) * (size_t)K * (size_t)d);
  if (!mind || !prev || !Cn) {
    free(mind);
    free(prev);
    free(Cn);
    return KMO_E_INVALID;
  }
  for (int64_t i = 0; i < N; ++i) prev[i] = -1;
  for (int32_t t = 0; t < iters; ++t) {
    kmo_assign(X, N, d, C, K, labels, mind, NULL, nthreads);
    double s = 0.0;
    int64_t ch = 0;
    for (int64_t i = 0; i < N; ++i) {
      s += mind[i];
      ch += labels[i] != prev[i];
      prev[i] = labels[i];
    }
    if (cost) cost[t] = s;
    if (changed) changed[t] = ch;
    kmo_lloyd_update(X, N, d, labels, K, C, Cn, NULL);
    memcpy(C, Cn, sizeof(float) * (size_t)K * (size_t)d);
  }
  free(mind);
  free(prev);
  free(Cn);
  return KMO_OK;
}

/* ---- k-means|| (Bahmani, Moseley, Vattani, Kumar, Vassilvitskii, "Scalable
 * K-Means++", PVLDB 5(7), 2012: Algorithm 2), the different initialisation
 * the paper's introduction attributes to Bahmani et al.  Its steps, in
 * order:
 *   1. C = one point drawn uniformly at random;
 *   2. `rounds` times: every point x joins C' independently with
 *      probability min(1, ell * d^2(x, C) / phi(C)), phi(C) = sum_x d^2(x, C);
 *      then C = C u C';
 *   3. w_c = the number of points whose nearest candidate is c;
 *   4. the weighted candidates are reclustered into K centres by weighted
 *      k-means++: the first with probability proportional to w, each next
 *      with probability proportional to w * d^2(c, chosen centres).
 * Readings: the number of rounds is a parameter (the O(log psi) of the
 * algorithm); candidates are kept in the order they join, within a round in
 * point order; nearest-candidate ties go to the smaller candidate index;
 * phi is the FP64 sum of D in point order; the random numbers are Philox
 * words turned into u in [0,1) as in kmo_uniform with counters
 *   first point               (0, inst, 0, 0)   (the k-means++ first seed)
 *   point i in round r >= 1   (i, inst, r, 1)
 *   recluster draw m >= 0     (m, inst, 0, 2);
 * point i joins iff u < p (p computed in FP64 as ell * D_i / phi, capped at
 * 1); a recluster draw inverts the weighted CDF over candidates in index
 * order exactly like the k-means++ draw (first index whose inclusive prefix
 * exceeds t = u * total; rounding fallback to the last positive entry;
 * uniform candidate with a warning when the total is zero).
 */
static double kmo_u_ctr(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
  const uint32_t ctr[4] = {c0, c1, c2, c3};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t r[4];
  kmo_philox4x32_10(ctr, key, r);
  return (double)((uint64_t)(r[0] >> 5) * 67108864ull + (uint64_t)(r[1] >> 6)) / 9007199254740992.0;
}

double kmo_uniform4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
  return kmo_u_ctr(seed, c0, c1, c2, c3);
}

/*
 * One draw of the weighted recluster (step 4 of k-means||): S = inclusive
 * FP64 prefix of the shares in order (sequential), T = S_{n-1},
 * t = u * T (one IEEE multiply), the first j with S_j > t; if none (t >= T),
 * the last j whose share raised S.  T == 0: the uniform index and
 * KMO_W_DEGENERATE; T not finite: KMO_E_NONFINITE (no index).
 */
static int kmo_wdraw_on(const double* share, double* S, int64_t n, double u, int64_t* out_j, double* T_out,
                        double* t_out) {
  double acc = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    acc += share[j];
    S[j] = acc;
  }
  const double T = acc;
  volatile double tv = u * T;
  const double t = tv;
  *T_out = T;
  *t_out = t;
  if (!isfinite(T)) return KMO_E_NONFINITE;
  if (T == 0.0) {
    *out_j = kmo_uniform_index(u, n);
    return KMO_W_DEGENERATE;
  }
  int64_t g = kmo_upper_bound(S, n, t);
  if (g >= n) {
    g = n - 1;
    while (g > 0 && S[g] == S[g - 1]) --g;
  }
  *out_j = g;
  return KMO_OK;
}

/* The recluster draw alone, with u given (rec4 as for kmo_draw). */
int kmo_wdraw(const double* share, int64_t n, double u, int64_t* out_j, double* rec4) {
  if (!share || !out_j || n < 1) return KMO_E_INVALID;
  double* S = (double*)malloc(sizeof(double) * (size_t)n);
  if (!S) return KMO_E_INVALID;
  double T, t;
  int64_t g = -1;
  const int st = kmo_wdraw_on(share, S, n, u, &g, &T, &t);
  *out_j = g;
  if (rec4) {
    rec4[0] = T;
    rec4[1] = t;
    rec4[2] = (g > 0 && g < n) ? S[g - 1] : (g == 0 ? 0.0 : NAN);
    rec4[3] = (g >= 0 && g < n) ? S[g] : NAN;
  }
  free(S);
  return st;
}

/*
 * X [N*d] FP32 points; K centres; cap = capacity of the candidate list.
 * Outputs: cand [cap] candidate point indices, *ncand, round_end [rounds+1]
 * (candidates after the first point and after each round), weights [cap],
 * labels [N] (nullable: nearest candidate of every point), out_idx [K]
 * (point indices of the centres), rec [K*8] (per recluster draw: total, t,
 * the prefix interval of the oracle's own index, the prefix interval of the
 * replayed index, its weighted distance, u; row 0 for the first draw too),
 * phi [rounds] (phi before each round) and Dr [rounds*N] (D before each
 * round; nullable).
 * Replay (all nullable): rp_cand/rp_end make every round start from the
 * given candidates instead of the oracle's own; rp_w replaces the weights
 * of the recluster; rp_idx makes every recluster draw start from the given
 * earlier centres.  Returns KMO_OK, KMO_W_DEGENERATE, or a negative error
 * (KMO_E_INVALID also when more than cap candidates would be needed).
 */
int kmo_kmpar(const float* X, int64_t N, int32_t d, int32_t K, uint64_t seed, uint32_t inst, int32_t rounds,
              double ell, int64_t cap, int64_t* cand, int64_t* ncand, int64_t* round_end, int64_t* weights,
              int32_t* labels, int64_t* out_idx, double* rec, double* phi, double* Dr, const int64_t* rp_cand,
              const int64_t* rp_end, const int64_t* rp_w, const int64_t* rp_idx, int32_t nthreads) {
  if (!X || !cand || !ncand || !round_end || !weights || !out_idx || N < 1 || d < 1 || K < 1 || rounds < 0 ||
      cap < 1 || !(ell > 0.0))
    return KMO_E_INVALID;
  const int nt = kmo_threads(nthreads);
  int status = KMO_OK;
  double* D = (double*)malloc(sizeof(double) * (size_t)N);
  int32_t* lab = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  double* c = (double*)malloc(sizeof(double) * (size_t)d);
  if (!D || !lab || !c) {
    free(D);
    free(lab);
    free(c);
    return KMO_E_INVALID;
  }
  /* 1. the first point */
  int64_t m = 0;
  cand[m++] = kmo_uniform_index(kmo_u_ctr(seed, 0u, inst, 0u, 0u), N);
  const int64_t* C = rp_cand ? rp_cand : cand;
  for (int64_t i = 0; i < N; ++i) {
    D[i] = INFINITY;
    lab[i] = -1;
  }
  round_end[0] = 1;
  int64_t done = 0; /* candidates already folded into D */
  for (int32_t r = 0; r <= rounds && status >= 0; ++r) {
    /* fold the candidates that joined last into D and the labels */
    const int64_t upto = r == 0 ? 1 : (rp_end ? rp_end[r] : round_end[r]);
    for (int64_t j = done; j < upto; ++j) {
      for (int32_t q = 0; q < d; ++q) c[q] = (double)X[C[j] * (int64_t)d + q];
#pragma omp parallel for schedule(static) num_threads(nt)
      for (int64_t i = 0; i < N; ++i) {
        const double v = kmo_sqdist(X + i * (int64_t)d, c, d);
        if (v < D[i]) {
          D[i] = v;
          lab[i] = (int32_t)j;
        }
      }
    }
    done = upto;
    if (r == rounds) break;
    /* 2. one round of independent draws */
    double s = 0.0;
    for (int64_t i = 0; i < N; ++i) s += D[i];
    if (phi) phi[r] = s;
    if (Dr) memcpy(Dr + (int64_t)r * N, D, sizeof(double) * (size_t)N);
    if (!isfinite(s)) {
      status = KMO_E_NONFINITE;
      break;
    }
    const int64_t before = m;
    for (int64_t i = 0; i < N && status >= 0; ++i) {
      double p = s > 0.0 ? ell * D[i] / s : 0.0;
      if (p > 1.0) p = 1.0;
      if (kmo_u_ctr(seed, (uint32_t)i, inst, (uint32_t)(r + 1), 1u) < p) {
        if (m >= cap) {
          status = KMO_E_INVALID;
          break;
        }
        cand[m++] = i;
      }
    }
    (void)before;
    round_end[r + 1] = m;
  }
  *ncand = m;
  if (status < 0) {
    free(D);
    free(lab);
    free(c);
    return status;
  }
  /* 3. weights: points per nearest candidate (of the candidates in use) */
  const int64_t mc = rp_end ? rp_end[rounds] : m;
  for (int64_t j = 0; j < mc; ++j) weights[j] = 0;
  for (int64_t i = 0; i < N; ++i) weights[lab[i]] += 1;
  if (labels)
    for (int64_t i = 0; i < N; ++i) labels[i] = lab[i];
  const int64_t* W = rp_w ? rp_w : weights;
  /* 4. weighted k-means++ over the candidates */
  double* Dc = (double*)malloc(sizeof(double) * (size_t)mc);
  double* S = (double*)malloc(sizeof(double) * (size_t)mc);
  double* Sh = (double*)malloc(sizeof(double) * (size_t)mc);
  for (int64_t j = 0; j < mc; ++j) Dc[j] = INFINITY;
  for (int32_t k = 0; k < K; ++k) {
    /* weights of this draw: w (first) or w * Dc */
    for (int64_t j = 0; j < mc; ++j) Sh[j] = k == 0 ? (double)W[j] : (double)W[j] * Dc[j];
    const double u = kmo_u_ctr(seed, (uint32_t)k, inst, 0u, 2u);
    int64_t g = -1;
    double T, t;
    double* rr = rec ? rec + (int64_t)k * 8 : NULL;
    const int st = kmo_wdraw_on(Sh, S, mc, u, &g, &T, &t);
    if (st < 0) {
      status = st;
      break;
    }
    if (st == KMO_W_DEGENERATE && status == KMO_OK) status = KMO_W_DEGENERATE;
    out_idx[k] = C[g];
    const int64_t gr = rp_idx ? -1 : g; /* replayed candidate position, found below */
    int64_t gp = gr;
    if (rp_idx) {
      for (int64_t j = 0; j < mc; ++j)
        if (C[j] == rp_idx[k]) {
          gp = j;
          break;
        }
      if (gp < 0) gp = g;
    }
    if (rr) {
      rr[0] = T;
      rr[1] = t;
      rr[2] = g > 0 ? S[g - 1] : 0.0;
      rr[3] = S[g];
      rr[4] = gp > 0 ? S[gp - 1] : 0.0;
      rr[5] = S[gp];
      rr[6] = k == 0 ? (double)W[gp] : (double)W[gp] * Dc[gp];
      rr[7] = u;
    }
    /* the chosen centre (replayed if given) updates the candidates' D */
    const int64_t cj = gp;
    for (int32_t q = 0; q < d; ++q) c[q] = (double)X[C[cj] * (int64_t)d + q];
    for (int64_t j = 0; j < mc; ++j) {
      const double v = kmo_sqdist(X + C[j] * (int64_t)d, c, d);
      if (v < Dc[j]) Dc[j] = v;
    }
  }
  free(Dc);
  free(S);
  free(Sh);
  free(D);
  free(lab);
  free(c);
  return status;
}
