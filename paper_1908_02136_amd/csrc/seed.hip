// seed.hip -- the k-means++ seed loop (paper, Section II, Algorithms 1-2).
//
// One launch per seed pass.  Pass m (1..K) streams the point rows once,
// updates every point's nearest squared distance D = min(D, ||x - c_{m-1}||^2)
// and reduces D per workgroup tile into an FP64 tile sum.  For m < K the
// last workgroup of the pass to arrive (an epoch-free arrival counter that
// only grows during a run) draws seed m:
//   t = u_m * sum(D) (FP64),  tile j = first tile whose inclusive FP64 prefix
//   of tile sums exceeds t,  seed = first row of tile j whose inclusive FP64
//   prefix exceeds t,
// and copies that row (the original FP32 row) into out_centers[m], which
// the next pass broadcasts from LDS.  Nothing returns to the host between
// passes, and no workgroup ever waits on another, so the launch needs no
// co-residency.
//
// Row streaming: a row of d elements is split into 16-byte chunks; a group
// of G lanes covers one row (G*CPL chunks), so one wave-wide load reads 64/G
// whole consecutive rows (1 KiB contiguous).  Each lane keeps the centre
// slice of its chunks in registers and the row distance is reduced across
// the G lanes with xor shuffles.  U loads per lane are issued before any is
// consumed.  D is read and written once per row per pass with one coalesced
// access per 64 rows.
#include "kmpp_dev.h"
#include "kmpp_impl.h"

namespace kmpp {

// Tile-sum slots hold this NaN pattern (signalling, never produced by
// arithmetic) tagged with the pass number until the tile's sum arrives.
__device__ __forceinline__ uint64_t slot_sentinel(int pass) { return 0x7FF4000000000000ull | (uint32_t)pass; }

// ---------------------------------------------------------------- S1
// First seed: i0 = min(floor(u_0 N), N-1); resets the run's counters and
// arms the tile-sum slots for pass 1.
__global__ __launch_bounds__(256) void seed_init_kernel(SeedParams p) {
  __shared__ int64_t s_i0;
  if (threadIdx.x == 0) {
    p.ctl->status = KMPP_OK;
    p.ctl->arrive = 0u;
    const double u0 = draw_uniform(p.seed, 0u, p.inst);
    const int64_t i0 = uniform_index(u0, p.N);
    p.idx[0] = i0;
    s_i0 = i0;
  }
  uint64_t* slots = reinterpret_cast<uint64_t*>(p.tsum);
  for (int i = threadIdx.x; i < p.ntiles; i += blockDim.x) slots[i] = slot_sentinel(1);
  __syncthreads();
  const float* src = p.X + s_i0 * (int64_t)p.d;
  for (int j = threadIdx.x; j < p.d; j += blockDim.x) p.centers[j] = src[j];
}

// ---------------------------------------------------------------- S2 core
// Streams rows [r0, r1) with the wave layout described above and hands
// every row's new nearest distance to `sink(row, dnew)`.  The arithmetic of
// a row's distance depends only on the template parameters, so any caller
// with the same instance recomputes bit-identical values.
template <int FMT, int CB, int G, int CPL, int U, bool FULL, int NT>
struct Streamer {
  static constexpr int EB = ElemBytes<FMT>::value;
  static constexpr int VEC = CB / EB;
  static constexpr int RPL = 64 / G;  // rows per wave-wide load
  static constexpr int R = U * RPL;   // rows per wave iteration
  static constexpr int NW = NT / 64;
  static constexpr int NJ = (U + G - 1) / G;  // D rows per lane per iteration
  using RawT = typename Raw<CB>::T;

  float cen[CPL][VEC];
  int sub, rg, wave;

  __device__ __forceinline__ void init(const float* cs, int d) {
    const int lane = threadIdx.x & 63;
    wave = threadIdx.x >> 6;
    sub = lane % G;
    rg = lane / G;
    const int nchunk = d / VEC;
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
      const int c = sub + G * k;
#pragma unroll
      for (int e = 0; e < VEC; ++e) cen[k][e] = (FULL || c < nchunk) ? cs[c * VEC + e] : 0.0f;
    }
  }

  // One iteration: this wave's R rows starting at `base` (rows >= r1 skipped).
  template <class Sink>
  __device__ __forceinline__ void iter(const SeedParams& p, int64_t base, int64_t r1, bool first, int64_t prev,
                                       Sink&& sink) const {
    const int d = p.d;
    const int nchunk = d / VEC;
    const char* xb = static_cast<const char*>(p.xs);
    const int64_t rb = (int64_t)d * EB;
    float dold[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int uu = sub + G * j;
      const int64_t row = base + (int64_t)uu * RPL + rg;
      dold[j] = (!first && uu < U && row < r1) ? p.D[row] : INFINITY;
    }
    RawT raw[U][CPL];
    float sc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int64_t row = base + u * RPL + rg;
      row = row < r1 ? row : r1 - 1;  // in bounds; the value is discarded
      const char* rp = xb + row * rb;
#pragma unroll
      for (int k = 0; k < CPL; ++k) {
        const int c = sub + G * k;
        if (FULL || c < nchunk)
          raw[u][k] = *reinterpret_cast<const RawT*>(rp + (int64_t)c * CB);
        else
          raw[u][k] = RawT{};
      }
      if constexpr (FMT == FMT_FP8) sc[u] = exp2i((int)p.xexp[row]);
    }
    float delta[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      float a = 0.0f;
#pragma unroll
      for (int k = 0; k < CPL; ++k) {
        float v[VEC];
        decode<FMT, CB>(raw[u][k], v);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const float df = (FMT == FMT_FP8) ? fmaf(v[e], sc[u], -cen[k][e]) : v[e] - cen[k][e];
          a = fmaf(df, df, a);
        }
      }
#pragma unroll
      for (int o = G / 2; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
      delta[u] = a;
    }
    // lane (rg, sub) owns rows base + uu*RPL + rg for uu = sub, sub+G, ...
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int uu = sub + G * j;
      float dv = delta[0];
#pragma unroll
      for (int w = 1; w < U; ++w) dv = (w == uu) ? delta[w] : dv;
      const int64_t row = base + (int64_t)uu * RPL + rg;
      if (uu < U && row < r1) {
        float dn = first ? dv : fminf(dold[j], dv);
        if constexpr (FMT != FMT_F32) dn = (row == prev) ? 0.0f : dn;
        sink(row, dn);
      }
    }
  }
};

// ---------------------------------------------------------------- S3-S5
// Draw seed p.pass.  Runs in the last workgroup of the pass to arrive.
//  1. read the FP64 tile sums (waiting out any slot still armed), scan them
//     in a fixed order, t = u * total, pick the first tile whose inclusive
//     prefix exceeds t;
//  2. recompute that tile's new D with the pass's own arithmetic (whether a
//     row's D in memory is already this pass's or still the previous one,
//     min(D, delta) is this pass's value), one workgroup iteration at a time,
//     scanning each chunk in FP64 until the prefix exceeds t;
//  3. publish the index, copy the original FP32 row to out_centers, arm the
//     slots for the next pass.
template <int FMT, int CB, int G, int CPL, int U, bool FULL, int NT>
__device__ __forceinline__ void draw_and_commit(const SeedParams& p, const Streamer<FMT, CB, G, CPL, U, FULL, NT>& st,
                                                bool first, int64_t prev) {
  using S = Streamer<FMT, CB, G, CPL, U, FULL, NT>;
  constexpr int NW = NT / 64;
  constexpr int CH = NW * S::R;  // rows per chunk: one iteration of every wave
  __shared__ double sh[NW + 1];
  __shared__ int64_t shi[NW];
  __shared__ double s_lo;
  __shared__ float shf[NW];
  __shared__ float chunk[CH];
  __shared__ int64_t s_seed;
  const int tid = threadIdx.x;
  const int G_t = p.ntiles;
  const uint64_t armed = slot_sentinel(p.pass);
  uint64_t* slots = reinterpret_cast<uint64_t*>(p.tsum);

  const int per = (G_t + NT - 1) / NT;
  const int b0 = min(G_t, tid * per), b1 = min(G_t, b0 + per);
  double part = 0.0;
  bool late = false;
  for (int i = b0; i < b1; ++i) {
    uint64_t b = __hip_atomic_load(&slots[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int spin = 0; b == armed && spin < (1 << 22); ++spin) {
      __builtin_amdgcn_s_sleep(2);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      b = __hip_atomic_load(&slots[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    late |= b == armed;
    part += __longlong_as_double((long long)b);
  }
  if (late) raise_status(p.ctl, KMPP_E_TIMEOUT);
  double T;
  const double ex = block_exclusive_scan<NT>(part, sh, &T);
  const double u = draw_uniform(p.seed, (uint32_t)p.pass, p.inst);

  int64_t seed_row;
  if (!isfinite(T)) {
    if (tid == 0) raise_status(p.ctl, KMPP_E_NONFINITE);
    seed_row = 0;
  } else if (T == 0.0) {
    if (tid == 0) raise_status(p.ctl, KMPP_W_DEGENERATE);
    seed_row = uniform_index(u, p.N);
  } else {
    const double t = __dmul_rn(u, T);
    int64_t cand = INT64_MAX;
    double run = ex;
    int64_t lastpos = -1;
    for (int i = b0; i < b1; ++i) {
      const double v = __longlong_as_double((long long)slots[i]);
      if (v > 0.0) lastpos = i;
      const double nr = run + v;
      if (cand == INT64_MAX && nr > t) cand = i;
      if (cand == INT64_MAX) run = nr;
    }
    const int64_t tj = block_min<NT>(cand, shi);
    if (cand == tj && cand != INT64_MAX) s_lo = run;
    const int64_t tl = block_max<NT>(lastpos, shi);
    int64_t tile = tj != INT64_MAX ? tj : tl;
    if (tile < 0 || tile >= G_t) tile = G_t - 1;
    __syncthreads();
    const bool inside = tj != INT64_MAX;  // else: rounding put t past the total
    double run2 = inside ? s_lo : 0.0;
    const int64_t r0 = tile * (int64_t)p.rows_per_tile;
    const int64_t r1 = min(p.N, r0 + (int64_t)p.rows_per_tile);
    int64_t found = INT64_MAX, lastrow = -1;
    for (int64_t c0 = r0; c0 < r1 && found == INT64_MAX; c0 += CH) {
      const int64_t c1 = min(r1, c0 + (int64_t)CH);
      st.iter(p, c0 + (int64_t)st.wave * S::R, c1, first, prev,
              [&](int64_t row, float dn) { chunk[row - c0] = dn; });
      __syncthreads();
      const int n = (int)(c1 - c0);
      const int per2 = (n + NT - 1) / NT;
      const int q0 = min(n, tid * per2), q1 = min(n, q0 + per2);
      double part2 = 0.0;
      int64_t lp = -1;
      for (int q = q0; q < q1; ++q) {
        part2 += (double)chunk[q];
        if (chunk[q] > 0.0f) lp = c0 + q;
      }
      double tot2;
      const double ex2 = block_exclusive_scan<NT>(part2, sh, &tot2);
      int64_t c2 = INT64_MAX;
      if (inside) {
        double r = run2 + ex2;
        for (int q = q0; q < q1; ++q) {
          r += (double)chunk[q];
          if (r > t) {
            c2 = c0 + q;
            break;
          }
        }
      }
      found = block_min<NT>(c2, shi);
      const int64_t lpc = block_max<NT>(lp, shi);
      lastrow = lpc >= 0 ? lpc : lastrow;
      run2 += tot2;
    }
    seed_row = found != INT64_MAX ? found : (lastrow >= 0 ? lastrow : r1 - 1);
  }
  if (tid == 0) s_seed = seed_row;
  __syncthreads();
  seed_row = s_seed;

  // precision forms: the drawn row's D from the quantised rows (recomputed
  // with the pass's arithmetic) and its FP32 nearest distance from the
  // original row against the earlier seeds
  if (p.recheck != nullptr) {
    const int64_t r0s = seed_row / p.rows_per_tile * (int64_t)p.rows_per_tile;
    const int64_t r1s = min(p.N, r0s + (int64_t)p.rows_per_tile);
    const int64_t c0 = r0s + (seed_row - r0s) / CH * CH;
    const int64_t c1 = min(r1s, c0 + (int64_t)CH);
    __syncthreads();
    st.iter(p, c0 + (int64_t)st.wave * S::R, c1, first, prev,
            [&](int64_t row, float dn) { chunk[row - c0] = dn; });
    const float* xr = p.X + seed_row * (int64_t)p.d;
    float best = INFINITY;
    for (int j = tid; j < p.pass; j += NT) {
      const float* c = p.centers + (int64_t)j * p.d;
      float a = 0.0f;
      for (int k = 0; k < p.d; ++k) {
        const float df = xr[k] - c[k];
        a = fmaf(df, df, a);
      }
      best = fminf(best, a);
    }
    best = block_minf<NT>(best, shf);  // (synchronises the chunk writes too)
    if (tid == 0) {
      p.recheck[2 * (int64_t)p.pass] = chunk[seed_row - c0];
      p.recheck[2 * (int64_t)p.pass + 1] = best;
    }
  }
  if (tid == 0) p.idx[p.pass] = seed_row;
  const float* src = p.X + seed_row * (int64_t)p.d;
  float* dst = p.centers + (int64_t)p.pass * p.d;
  for (int j = tid; j < p.d; j += NT) dst[j] = src[j];
  const uint64_t next = slot_sentinel(p.pass + 1);
  for (int i = tid; i < G_t; i += NT) slots[i] = next;
}

// ---------------------------------------------------------------- S2 (+S3-S5)
template <int FMT, int CB, int G, int CPL, int U, bool FULL, int NT>
__global__ __launch_bounds__(NT) void seed_pass_kernel(SeedParams p) {
  using S = Streamer<FMT, CB, G, CPL, U, FULL, NT>;
  constexpr int NW = NT / 64;
  extern __shared__ float cs[];  // centre row, d floats
  __shared__ double red[NW];
  __shared__ int s_last;

  const int tid = threadIdx.x;
  const int d = p.d;
  const bool first = p.pass == 1;
  const int64_t t0 = (int64_t)blockIdx.x * p.rows_per_tile;
  const int64_t t1 = min(p.N, t0 + (int64_t)p.rows_per_tile);

  const float* cg = p.centers + (int64_t)(p.pass - 1) * d;
  for (int j = tid; j < d; j += NT) cs[j] = cg[j];
  const int64_t prev = (FMT != FMT_F32) ? p.idx[p.pass - 1] : -1;
  __syncthreads();
  S st;
  st.init(cs, d);

  double acc = 0.0;
  float* D = p.D;
  for (int64_t base = t0 + (int64_t)st.wave * S::R; base < t1; base += (int64_t)NW * S::R)
    st.iter(p, base, t1, first, prev, [&](int64_t row, float dn) {
      D[row] = dn;
      acc += (double)dn;
    });

  acc = wave_sum(acc);
  if ((tid & 63) == 0) red[st.wave] = acc;
  __syncthreads();
  if (p.pass == p.K) return;  // final pass: D is the output, no draw
  if (tid == 0) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[w];
    uint64_t* slots = reinterpret_cast<uint64_t*>(p.tsum);
    __hip_atomic_store(&slots[blockIdx.x], (uint64_t)__double_as_longlong(s), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t old = __hip_atomic_fetch_add(&p.ctl->arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_last = old == (uint32_t)p.pass * (uint32_t)p.ntiles - 1u;
  }
  __syncthreads();
  if (!s_last) return;
  draw_and_commit<FMT, CB, G, CPL, U, FULL, NT>(p, st, first, prev);
}

// ---------------------------------------------------------------- registry
template <int FMT, int CB, int G, int CPL, int U, bool FULL, int NT>
static SeedVariant make_variant(int dexact) {
  SeedVariant v;
  v.fmt = FMT;
  v.dexact = dexact;
  v.cb = CB;
  v.g = G;
  v.cpl = CPL;
  v.u = U;
  v.full = FULL;
  v.nt = NT;
  v.rows_per_iter = (NT / 64) * U * (64 / G);
  v.fn = reinterpret_cast<const void*>(&seed_pass_kernel<FMT, CB, G, CPL, U, FULL, NT>);
  return v;
}

#define KMPP_VARIANTS_NT(NT)                                                                  \
  /* FP32, 16-byte chunks: d = 4*G*CPL */                                                    \
  make_variant<FMT_F32, 8, 1, 1, 8, true, NT>(2), make_variant<FMT_F32, 16, 1, 1, 8, true, NT>(4), \
      make_variant<FMT_F32, 16, 2, 1, 8, true, NT>(8), make_variant<FMT_F32, 16, 4, 1, 8, true, NT>(16), \
      make_variant<FMT_F32, 16, 8, 1, 8, true, NT>(32), make_variant<FMT_F32, 16, 16, 1, 8, true, NT>(64), \
      make_variant<FMT_F32, 16, 32, 1, 8, true, NT>(128), make_variant<FMT_F32, 16, 64, 1, 8, true, NT>(256), \
      make_variant<FMT_F32, 16, 64, 2, 4, true, NT>(512),                                    \
      /* BF16, 16-byte chunks: d = 8*G*CPL */                                                \
      make_variant<FMT_BF16, 16, 1, 1, 8, true, NT>(8), make_variant<FMT_BF16, 16, 2, 1, 8, true, NT>(16), \
      make_variant<FMT_BF16, 16, 4, 1, 8, true, NT>(32), make_variant<FMT_BF16, 16, 8, 1, 8, true, NT>(64), \
      make_variant<FMT_BF16, 16, 16, 1, 8, true, NT>(128), make_variant<FMT_BF16, 16, 32, 1, 8, true, NT>(256), \
      /* FP8, 16-byte chunks: d = 16*G*CPL */                                                \
      make_variant<FMT_FP8, 16, 1, 1, 8, true, NT>(16), make_variant<FMT_FP8, 16, 2, 1, 8, true, NT>(32), \
      make_variant<FMT_FP8, 16, 4, 1, 8, true, NT>(64), make_variant<FMT_FP8, 16, 8, 1, 8, true, NT>(128), \
      make_variant<FMT_FP8, 16, 16, 1, 8, true, NT>(256),                                    \
      /* any d: one element per chunk, G = min(64, pow2 >= d) lanes per row */               \
      make_variant<FMT_F32, 4, 1, 1, 8, false, NT>(-1), make_variant<FMT_F32, 4, 2, 1, 8, false, NT>(-2), \
      make_variant<FMT_F32, 4, 4, 1, 8, false, NT>(-4), make_variant<FMT_F32, 4, 8, 1, 8, false, NT>(-8), \
      make_variant<FMT_F32, 4, 16, 1, 8, false, NT>(-16), make_variant<FMT_F32, 4, 32, 1, 8, false, NT>(-32), \
      make_variant<FMT_F32, 4, 64, 1, 8, false, NT>(-64), make_variant<FMT_F32, 4, 64, 4, 8, false, NT>(-256), \
      make_variant<FMT_F32, 4, 64, 16, 2, false, NT>(-1024), make_variant<FMT_F32, 4, 64, 64, 1, false, NT>(-4096), \
      make_variant<FMT_BF16, 2, 1, 1, 8, false, NT>(-1), make_variant<FMT_BF16, 2, 2, 1, 8, false, NT>(-2), \
      make_variant<FMT_BF16, 2, 4, 1, 8, false, NT>(-4), make_variant<FMT_BF16, 2, 8, 1, 8, false, NT>(-8), \
      make_variant<FMT_BF16, 2, 16, 1, 8, false, NT>(-16), make_variant<FMT_BF16, 2, 32, 1, 8, false, NT>(-32), \
      make_variant<FMT_BF16, 2, 64, 1, 8, false, NT>(-64), make_variant<FMT_BF16, 2, 64, 4, 8, false, NT>(-256), \
      make_variant<FMT_BF16, 2, 64, 16, 2, false, NT>(-1024), make_variant<FMT_BF16, 2, 64, 64, 1, false, NT>(-4096), \
      make_variant<FMT_FP8, 1, 1, 1, 8, false, NT>(-1), make_variant<FMT_FP8, 1, 2, 1, 8, false, NT>(-2), \
      make_variant<FMT_FP8, 1, 4, 1, 8, false, NT>(-4), make_variant<FMT_FP8, 1, 8, 1, 8, false, NT>(-8), \
      make_variant<FMT_FP8, 1, 16, 1, 8, false, NT>(-16), make_variant<FMT_FP8, 1, 32, 1, 8, false, NT>(-32), \
      make_variant<FMT_FP8, 1, 64, 1, 8, false, NT>(-64), make_variant<FMT_FP8, 1, 64, 4, 8, false, NT>(-256), \
      make_variant<FMT_FP8, 1, 64, 16, 2, false, NT>(-1024), make_variant<FMT_FP8, 1, 64, 64, 1, false, NT>(-4096)

const std::vector<SeedVariant>& seed_variants() {
  static const std::vector<SeedVariant> v = {KMPP_VARIANTS_NT(256), KMPP_VARIANTS_NT(512)};
  return v;
}

const void* seed_init_fn() { return reinterpret_cast<const void*>(&seed_init_kernel); }

}  // namespace kmpp
