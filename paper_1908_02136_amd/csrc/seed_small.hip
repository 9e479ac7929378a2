// seed_small.hip -- the whole k-means++ seed loop (paper, Section II,
// Algorithm 1) in ONE workgroup, for inputs whose rows fit its LDS.
//
// A small input spends almost all of its time between passes: each seed of
// the multi-workgroup loop costs a kernel boundary and the draw's dependent
// round trips through memory.  Here one 1024-thread workgroup copies the
// FP32 rows into LDS once, keeps each thread's D values in registers (thread
// t owns the contiguous rows [t R, t R + R), R = ceil(N / 1024)) and runs
// all K passes and K - 1 draws with workgroup barriers only.  In LDS, value
// k of the thread's row r sits at (r d + k) 1024 + t, so a wave's loads of
// one (r, k) are consecutive words, and a pass issues the R loads of each k
// together.
//   pass m:  D_i = min(D_i, ||x_i - c_{m-1}||^2) for the thread's rows (the
//            distance summed over k in order in FP32), and the thread's FP64
//            sum of its D values in row order;
//   draw m:  a fixed-order FP64 exclusive scan of the thread sums gives each
//            thread its prefix and the total T; t = u_m T; the first row
//            whose inclusive prefix exceeds t is the seed (if rounding leaves
//            none, the last row with D > 0); T = 0 draws uniformly
//            (KMPP_W_DEGENERATE), a non-finite T raises KMPP_E_NONFINITE.
// Weighted seeding (the k-means|| recluster) draws in proportion to w D
// (FP64 products), the first seed in proportion to w.  The draws follow the
// same definition as the other placements, but the FP64 partial sums are
// taken over each thread's rows instead of over tiles, so a draw that falls
// within rounding of a row boundary may pick the neighbouring row.
#include "kmpp_dev.h"
#include "kmpp_impl.h"

namespace kmpp {

constexpr int kSmallNT = 1024;
constexpr int kSmallNW = kSmallNT / 64;

// Exclusive scan of one double per thread over the workgroup, fixed order
// (within waves by lane, then waves in order); returns (exclusive, total).
__device__ __forceinline__ double2 small_scan(double v, double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  double ex = __shfl_up(x, 1, 64);
  if (lane == 0) ex = 0.0;
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  double off = 0.0, tot = 0.0;
#pragma unroll
  for (int w = 0; w < kSmallNW; ++w) {
    if (w == wave) off = tot;
    tot += sh[w];
  }
  __syncthreads();
  return make_double2(off + ex, tot);
}

// min (MIN) or max over the workgroup (the draw's rare fallbacks).
template <bool MIN>
__device__ __forceinline__ int small_ext(int b, int* sb) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int v = __shfl_xor(b, o, 64);
    b = MIN ? min(b, v) : max(b, v);
  }
  if ((threadIdx.x & 63) == 0) sb[threadIdx.x >> 6] = b;
  __syncthreads();
  b = sb[0];
#pragma unroll
  for (int w = 1; w < kSmallNW; ++w) b = MIN ? min(b, sb[w]) : max(b, sb[w]);
  __syncthreads();
  return b;
}

template <int RMAX, bool WEIGHTED>
__global__ __launch_bounds__(kSmallNT) void seed_small_kernel(SeedParams p) {
  __shared__ float xs[kSmallMaxElems];
  __shared__ double sh[kSmallNW];
  __shared__ int sb[kSmallNW];
  __shared__ int s_found[2];  // by draw parity: the smallest candidate row
  const int tid = threadIdx.x;
  const int64_t N = p.N;
  const int d = p.d, K = p.K;
  const int R = (int)((N + kSmallNT - 1) / kSmallNT);  // <= RMAX (host check)
  const int64_t r0 = min(N, (int64_t)tid * R);
  const int nr = (int)min((int64_t)R, N - r0);
  constexpr int NONE = INT_MAX;
  // weighted seeding: the weights after the rows, interleaved the same way
  const int* wl = reinterpret_cast<const int*>(xs) + R * d * kSmallNT;

  // row i = t R + r, value k -> xs[(r d + k) 1024 + t]
  for (int64_t e = tid; e < N * d; e += kSmallNT) {
    const int64_t i = e / d;
    const int k = (int)(e - i * d);
    const int t = (int)(i / R), r = (int)(i - (int64_t)t * R);
    xs[(r * d + k) * kSmallNT + t] = p.X[e];
  }
  if constexpr (WEIGHTED) {
    for (int64_t i = tid; i < N; i += kSmallNT) {
      const int t = (int)(i / R), r = (int)(i - (int64_t)t * R);
      reinterpret_cast<int*>(xs)[R * d * kSmallNT + r * kSmallNT + t] = p.wts[i];
    }
  }
  if (tid == 0) {
    p.ctl->status = KMPP_OK;
    if (p.sumD) p.sumD[0] = 0.0;
    s_found[0] = NONE;
    s_found[1] = NONE;
  }
  __syncthreads();

  float D[RMAX];
#pragma unroll
  for (int r = 0; r < RMAX; ++r) D[r] = 1.0f;  // the weighted first draw: shares w * 1
  // a row's share of the draw: D, or w D in FP64
  auto share = [&](int r) -> double {
    if constexpr (WEIGHTED)
      return (double)D[r] * (double)wl[r * kSmallNT + tid];
    else
      return (double)D[r];
  };
  // draw m from the current D (every thread returns the same row)
  auto draw = [&](int m) -> int64_t {
    double part = 0.0;
    int lastpos = -1;
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      if (r < nr) {
        const double v = share(r);
        part += v;
        if (v > 0.0) lastpos = (int)r0 + r;
      }
    }
    const double2 sc = small_scan(part, sh);
    const double T = sc.y;
    // the next draw's candidate slot (its last readers, in the previous
    // draw, are past this draw's scan barriers)
    if (tid == 0) s_found[(m + 1) & 1] = NONE;
    const double u = draw_uniform(p.seed, (uint32_t)m, p.inst, p.tag);
    if (tid == 0 && p.sumD) p.sumD[m] = T;
    if (!isfinite(T)) {
      if (tid == 0) raise_status(p.ctl, KMPP_E_NONFINITE);
      return 0;
    }
    if (T == 0.0) {
      if (tid == 0) raise_status(p.ctl, KMPP_W_DEGENERATE);
      return uniform_index(u, N);
    }
    // the seed is the smallest candidate row over the workgroup (a thread's
    // candidate: its first row whose inclusive prefix exceeds t).  Every
    // thread past the owner of t has one (its first row), so the owner's
    // candidate (the one thread with exclusive prefix <= t that finds one)
    // is posted alone to an LDS minimum; only where rounding leaves the
    // owner without one is the full minimum taken, and where no thread has
    // one, the last row with a positive share.
    const double t = __dmul_rn(u, T);
    int found = NONE;
    double run = sc.x;
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      if (r < nr) {
        run += share(r);
        if (found == NONE && run > t) found = (int)r0 + r;
      }
    }
    if (found != NONE && sc.x <= t) atomicMin(&s_found[m & 1], found);
    __syncthreads();
    int f = s_found[m & 1];
    if (f == NONE) f = small_ext<true>(found, sb);
    if (f != NONE) return f;
    const int l = small_ext<false>(lastpos, sb);
    return l >= 0 ? l : N - 1;
  };

  // the first seed: uniform, or (weighted) drawn in proportion to w
  int64_t cidx;
  if constexpr (WEIGHTED) {
    cidx = draw(0);
  } else {
    cidx = uniform_index(draw_uniform(p.seed, 0u, p.inst, p.tag), N);
  }
  if (tid == 0) p.idx[0] = cidx;
  for (int m = 1; m <= K; ++m) {
    // pass m: centre m - 1 (row cidx = tc R + rc)
    const int tc = (int)(cidx / R), rc = (int)(cidx - (int64_t)tc * R);
    const float* c = xs + rc * d * kSmallNT + tc;  // value k at c[k * kSmallNT]
    for (int j = tid; j < d; j += kSmallNT) p.centers[(int64_t)(m - 1) * d + j] = c[j * kSmallNT];
    float a[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) a[r] = 0.0f;
    for (int k = 0; k < d; ++k) {
      const float ck = c[k * kSmallNT];
#pragma unroll
      for (int r = 0; r < RMAX; ++r) {
        // slots r >= R (past the layout) re-read slot R - 1 and are dropped,
        // as are the rows past the thread's own
        const int rr = min(r, R - 1);
        const float df = xs[(rr * d + k) * kSmallNT + tid] - ck;
        a[r] = fmaf(df, df, a[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < RMAX; ++r)
      if (r < nr) D[r] = m == 1 ? a[r] : fminf(D[r], a[r]);
    if (m == K) break;
    cidx = draw(m);
    if (tid == 0) p.idx[m] = cidx;
  }
#pragma unroll
  for (int r = 0; r < RMAX; ++r)
    if (r < nr) p.D[r0 + r] = D[r];
  if (p.status_out) {
    __syncthreads();
    if (tid == 0) *p.status_out = __hip_atomic_load(&p.ctl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// The kernel for N rows of width d (weighted: plus a weight per row), or
// null where the interleaved rows (R (d + weighted) 1024 values) would not
// fit the LDS array or R exceeds 16 (24 rows per thread spilled D to
// scratch).
const void* seed_small_fn(int64_t N, int d, bool weighted) {
  const int64_t R = (N + kSmallNT - 1) / kSmallNT;
  if (R * (d + (weighted ? 1 : 0)) * kSmallNT > kSmallMaxElems) return nullptr;
#define KMPP_SMALL(RM)                                                                                \
  if (R <= RM)                                                                                        \
    return weighted ? reinterpret_cast<const void*>(&seed_small_kernel<RM, true>)                     \
                    : reinterpret_cast<const void*>(&seed_small_kernel<RM, false>);
  KMPP_SMALL(4)
  KMPP_SMALL(8)
  KMPP_SMALL(12)
  KMPP_SMALL(16)
#undef KMPP_SMALL
  return nullptr;
}
int seed_small_threads() { return kSmallNT; }

}  // namespace kmpp
