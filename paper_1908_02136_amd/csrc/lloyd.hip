// lloyd.hip -- Lloyd iterations after seeding.  Section II of the paper
// says that once the initial centroids are chosen the clustering proceeds as
// in standard k-means; the partition O of Algorithm 1 is its output.  One
// iteration is the nearest-seed assignment (assign.hip) followed by moving
// every centre to the mean of its points; a centre with no points keeps its
// position.
//
// Cluster sums are accumulated in 64-bit fixed point: every value x becomes
// the integer nearest to x * 2^F, with F = 62 - e - ceil(log2 N) and
// max|x| < 2^e, so no cluster sum can overflow.  Integer addition is
// associative, so the sums do not depend on the order of the atomic adds and
// every run gives the same bits.  The rounding of one value is at most
// 2^(-F-1) = 2^(e + ceil(log2 N) - 63): for N = 2^24 and max|x| = 100 that is
// 2^-32, far below half a unit in the last place of an FP32 mean unless the
// mean is about 2^13 times smaller than max|x|; integer-valued points are
// summed exactly.
//
// Accumulation without global atomics: the clusters are split into R ranges
// whose sums fit in one workgroup's LDS, and W workgroups per range each
// take every W-th group of rows.  A workgroup adds the rows whose label lies
// in its range into LDS (integer LDS atomics), then writes its partial sums
// to global memory; the finalize kernel adds the W partials of every sum in
// a fixed order and divides.  Workgroups of all ranges are interleaved in
// the grid, so the ranges read the same labels at about the same time and
// the repeated label reads hit the caches; each row is read once.
#include "kmpp_dev.h"
#include "kmpp_impl.h"

namespace kmpp {

// First 256 bytes of a Lloyd workspace; the status word comes first as in
// every workspace.
struct LloydCtl {
  int32_t status;
  uint32_t amax_bits;  // max |x| over the rows (FP32 bits; non-negative, so ordered as integers)
  uint32_t pad[62];
};
static_assert(sizeof(LloydCtl) == 256, "control block is 256 bytes");

struct LloydParams {
  const void* X;
  const int8_t* xexp;
  int64_t N;
  int32_t d, K;
  int32_t G, lgG;             // lanes per row (power of two <= 64) and its log2
  int32_t R, Kr, W;           // cluster ranges, clusters per range, workgroups per range
  const int32_t* labels;      // this iteration's assignment
  const int32_t* prev;        // the previous iteration's, or null (first iteration)
  const float* mind;          // distance of every row to its centre
  float* C;                   // [K, d], updated in place
  long long* pacc;            // [W, K * d] partial fixed-point sums
  int32_t* pcnt;              // [W, K] partial cluster sizes
  double* pcost;              // [W] partial costs (range 0)
  uint32_t* pchg;             // [W] partial changed-label counts (range 0)
  float* pamax;               // [max-pass workgroups] partial max |x|
  unsigned long long* changed;  // rows whose label changed, or null
  double* cost;               // sum of mind, or null
  int32_t* counts_out;        // cluster sizes out, or null
  LloydCtl* lc;
  int32_t Wc;                 // partial costs / changed counts to add in the finalize
  // sorted path (see lloyd_hist_kernel)
  int32_t Wh;                 // histogram workgroups; workgroup w takes rows [w * B, (w + 1) * B)
  int64_t B;
  int32_t CH;                 // sorted positions per run-sum workgroup
  int32_t* hist;              // [K, Wh] rows of cluster j in block w, then their first position
  int32_t* order;             // [N] row indices grouped by cluster
  int32_t* coff;              // [K + 1] first sorted position of cluster j; coff[K] = rows with a label
};

template <int FMT>
__device__ __forceinline__ float lx(const LloydParams& p, int64_t row, int k) {
  if constexpr (FMT == FMT_F32) {
    return static_cast<const float*>(p.X)[row * p.d + k];
  } else if constexpr (FMT == FMT_BF16) {
    return __uint_as_float((uint32_t) static_cast<const uint16_t*>(p.X)[row * p.d + k] << 16);
  } else {
    const uint8_t q = static_cast<const uint8_t*>(p.X)[row * p.d + k];
    return __builtin_amdgcn_cvt_f32_fp8((int)q, 0) * exp2i((int)p.xexp[row]);
  }
}

// The fixed-point exponent F from max|x| and N (see the top of the file).
__device__ __forceinline__ int lloyd_F(const LloydParams& p) {
  const float amax = __uint_as_float(p.lc->amax_bits);
  int e = 0;
  if (amax > 0.0f && amax <= 3.4028235e38f) (void)frexpf(amax, &e);  // amax < 2^e
  const int lgN = p.N > 1 ? 64 - __clzll((unsigned long long)(p.N - 1)) : 0;
  return 62 - e - lgN;
}

__global__ void lloyd_reset_kernel(LloydCtl* lc) { lc->status = KMPP_OK; }

// max |x| over all rows; a NaN or infinite value sets KMPP_E_NONFINITE.
// FP32 / BF16: the rows as one flat array in 16-byte chunks; FP8: row by
// row (each row has its own scale).
// One partial maximum per workgroup (no contended atomics); a one-workgroup
// kernel reduces them.
__device__ __forceinline__ void absmax_publish(const LloydParams& p, float m, bool bad) {
  __shared__ float sh[4];
  m = block_minf<256>(-m, sh);
  if (threadIdx.x == 0) p.pamax[blockIdx.x] = -m;
  if (bad) raise_status(reinterpret_cast<Ctl*>(p.lc), KMPP_E_NONFINITE);
}

__global__ __launch_bounds__(256) void lloyd_absmax_final_kernel(LloydParams p, int n) {
  __shared__ float sh[4];
  float m = 0.0f;
  for (int i = threadIdx.x; i < n; i += 256) m = fmaxf(m, p.pamax[i]);
  m = block_minf<256>(-m, sh);
  if (threadIdx.x == 0) p.lc->amax_bits = __float_as_uint(-m);
}

template <int FMT>
__global__ __launch_bounds__(256) void lloyd_absmax_kernel(LloydParams p) {
  float m = 0.0f;
  bool bad = false;
  if constexpr (FMT == FMT_FP8) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sub = lane & (p.G - 1), rg = lane >> p.lgG;
    const int rpw = 64 >> p.lgG;
    for (int64_t row = ((int64_t)blockIdx.x * 4 + wave) * rpw + rg; row < p.N;
         row += (int64_t)gridDim.x * 4 * rpw)
      for (int k = sub; k < p.d; k += p.G) {
        const float a = fabsf(lx<FMT>(p, row, k));
        bad |= !(a <= 3.4028235e38f);
        m = fmaxf(m, a);
      }
  } else {
    constexpr int VEC = 16 / ElemBytes<FMT>::value;
    const int64_t n = p.N * (int64_t)p.d;
    const int64_t nchunk = n / VEC;
    const gptr<const char> xb = as_global(static_cast<const char*>(p.X));
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t c0 = (int64_t)blockIdx.x * 256 + threadIdx.x; c0 < nchunk; c0 += 4 * stride) {
      uint4 raw[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t c = c0 + u * stride;
        raw[u] = c < nchunk ? load_raw<16>(xb + c * 16) : make_uint4(0u, 0u, 0u, 0u);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        float v[VEC];
        decode<FMT, 16>(raw[u], v);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const float a = fabsf(v[e]);
          bad |= !(a <= 3.4028235e38f);
          m = fmaxf(m, a);
        }
      }
    }
    // the elements after the last whole chunk
    for (int64_t e = nchunk * VEC + (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += stride) {
      const float a = fabsf(lx<FMT>(p, e / p.d, (int)(e % p.d)));
      bad |= !(a <= 3.4028235e38f);
      m = fmaxf(m, a);
    }
  }
  absmax_publish(p, m, bad);
}


// Partial cluster sums of one iteration.  Workgroup (w, r) = blockIdx.x
// (w * R + r) takes blocks of kLB * 64 consecutive rows, member w's waves
// striding over the blocks.  Per block a wave loads the labels (kLB
// coalesced loads in flight), keeps the rows whose label lies in range r
// (ballots, compacted through LDS), and adds them into LDS with G lanes per
// row and U rows per lane group in flight.  Sixteen waves share one copy of
// the sums, so the copies' LDS still leaves room for 32 waves per CU.  The
// range-0 workgroups also sum the cost and count the changed labels over
// their blocks, so every row is counted once.
constexpr int kLB = 4;       // 64-row label chunks per block
constexpr int kLNT = 1024;   // threads per accumulation workgroup
constexpr int kLNW = kLNT / 64;

template <int FMT, int EPL>
__global__ __launch_bounds__(kLNT) void lloyd_accum_kernel(LloydParams p) {
  constexpr int U = EPL >= 16 ? 1 : 16 / EPL;  // rows per lane group in flight
  extern __shared__ long long sh_acc[];        // [Kr * d] sums, then [Kr] int sizes
  __shared__ double red[kLNW];
  __shared__ unsigned int red_ch[kLNW];
  __shared__ int s_pk[kLNW][kLB * 64];  // compacted rows: (label - j0) << 8 | row in block
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int G = p.G;
  const int sub = lane & (G - 1), rg = lane >> p.lgG;
  const int rpw = 64 >> p.lgG;
  const int r = blockIdx.x % p.R, w = blockIdx.x / p.R;
  const int j0 = r * p.Kr, j1 = min(p.K, j0 + p.Kr);
  const int nj = j1 - j0;
  const int64_t kd = (int64_t)nj * p.d;
  int* cnt = reinterpret_cast<int*>(sh_acc + (int64_t)p.Kr * p.d);
  for (int64_t e = tid; e < kd; e += kLNT) sh_acc[e] = 0;
  for (int j = tid; j < nj; j += kLNT) cnt[j] = 0;
  __syncthreads();
  const int F = lloyd_F(p);
  const bool tally = r == 0;
  double cost = 0.0;
  unsigned int changed = 0;
  const int64_t nblocks = (p.N + kLB * 64 - 1) / (kLB * 64);
  for (int64_t c = (int64_t)w * kLNW + wave; c < nblocks; c += (int64_t)p.W * kLNW) {
    const int64_t base = c * (kLB * 64);
    int lab[kLB];
#pragma unroll
    for (int i = 0; i < kLB; ++i) {
      const int64_t row = base + i * 64 + lane;
      lab[i] = row < p.N ? p.labels[row] : -1;
    }
    int nm = 0;
#pragma unroll
    for (int i = 0; i < kLB; ++i) {
      const int64_t row = base + i * 64 + lane;
      // label -1 (a row with NaN; status set by the max pass) is in no range
      if (tally && (unsigned)lab[i] < (unsigned)p.K) {
        cost += (double)p.mind[row];
        changed += p.prev ? (p.prev[row] != lab[i]) : 1u;
      }
      const bool in = lab[i] >= j0 && lab[i] < j1;
      const unsigned long long m = __ballot(in);
      if (in) s_pk[wave][nm + __popcll(m & ((1ull << lane) - 1ull))] = ((lab[i] - j0) << 8) | (i * 64 + lane);
      nm += __popcll(m);
    }
    if (nm == 0) continue;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    for (int q0 = 0; q0 < nm; q0 += rpw * U) {
      float v[U][EPL];
      int jr[U];
      // unconditional loads (row and element clamped into range, values
      // masked afterwards): all of them in flight together
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int slot = q0 + u * rpw + rg;
        const bool ok = slot < nm;
        const int pk = ok ? s_pk[wave][slot] : -1;
        const int64_t rr = min(p.N - 1, base + (pk & 255));
        jr[u] = ok ? (pk >> 8) : -1;
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          const int k = sub + G * e;
          const float x = lx<FMT>(p, rr, k < p.d ? k : p.d - 1);
          v[u][e] = (ok && k < p.d) ? x : 0.0f;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (jr[u] < 0) continue;
        long long* a = sh_acc + (int64_t)jr[u] * p.d;
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          const int k = sub + G * e;
          if (k < p.d)
            atomicAdd(reinterpret_cast<unsigned long long*>(a + k),
                      (unsigned long long)__float2ll_rn(ldexpf(v[u][e], F)));
        }
        if (sub == 0) atomicAdd(cnt + jr[u], 1);
      }
    }
    // s_pk is rewritten by the next block
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
  __syncthreads();
  long long* pa = p.pacc + ((int64_t)w * p.K + j0) * p.d;
  for (int64_t e = tid; e < kd; e += kLNT) pa[e] = sh_acc[e];
  int32_t* pc = p.pcnt + (int64_t)w * p.K + j0;
  for (int j = tid; j < nj; j += kLNT) pc[j] = cnt[j];
  if (tally) {
    cost = wave_sum(cost);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) changed += __shfl_xor(changed, o, 64);
    if (lane == 0) {
      red[wave] = cost;
      red_ch[wave] = changed;
    }
    __syncthreads();
    if (tid == 0) {
      double sc = 0.0;
      unsigned int cc = 0;
      for (int i = 0; i < kLNW; ++i) {
        sc += red[i];
        cc += red_ch[i];
      }
      p.pcost[w] = sc;
      p.pchg[w] = cc;
    }
  }
}

// New centres from the W partials of every sum, added in member order
// (empty clusters keep theirs); sizes; the cost as the sum of the range-0
// partials in member order.
__global__ __launch_bounds__(256) void lloyd_finalize_kernel(LloydParams p) {
  __shared__ double red[4];
  __shared__ unsigned long long redc[4];
  const int F = lloyd_F(p);
  const int64_t kd = (int64_t)p.K * p.d;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < kd) {
    const int64_t j = e / p.d;
    long long s = 0;
    int n = 0;
#pragma unroll 8
    for (int w = 0; w < p.W; ++w) {
      s += p.pacc[(int64_t)w * kd + e];
      n += p.pcnt[(int64_t)w * p.K + j];
    }
    if (n > 0) p.C[e] = (float)(ldexp((double)s, -F) / (double)n);
    if (p.counts_out && e % p.d == 0) p.counts_out[j] = n;
  }
  if (blockIdx.x == 0) {
    const int per = (p.Wc + 255) / 256;
    const int b0 = threadIdx.x * per;
    double s = 0.0;
    unsigned long long c = 0;
    for (int i = b0; i < min(p.Wc, b0 + per); ++i) {
      s += p.pcost[i];
      c += p.pchg[i];
    }
    s = wave_sum(s);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) {
      red[threadIdx.x >> 6] = s;
      redc[threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      if (p.cost) *p.cost = ((red[0] + red[1]) + red[2]) + red[3];
      if (p.changed) *p.changed = ((redc[0] + redc[1]) + redc[2]) + redc[3];
    }
  }
}

// ---------------------------------------------------------------- sorted path
// With many cluster ranges (large K * d) the LDS path re-reads the labels
// once per range and adds every element with an LDS atomic.  The sorted
// path groups the rows by label instead (a counting sort: per-block label
// histograms, per-cluster positions, a scatter of row indices), then each
// run-sum workgroup adds contiguous runs of one cluster's rows in registers
// and each run's fixed-point sums into the cluster's sums with one 64-bit
// integer atomic per element.  Integer additions do not depend on their
// order, so the centres are the same bits as on the LDS path; the cost and
// the changed-label count are added per block in a fixed order.
constexpr int kSNT = 256;  // threads of the sorted-path kernels

// Block w: label histogram (LDS) of rows [w * B, (w + 1) * B), written to
// hist[j * Wh + w], and the block's cost and changed count.
__global__ __launch_bounds__(kSNT) void lloyd_hist_kernel(LloydParams p) {
  extern __shared__ int sh_h[];  // [K]
  __shared__ double red[kSNT / 64];
  __shared__ unsigned int red_c[kSNT / 64];
  const int tid = threadIdx.x, w = blockIdx.x;
  for (int j = tid; j < p.K; j += kSNT) sh_h[j] = 0;
  __syncthreads();
  const int64_t r0 = (int64_t)w * p.B, r1 = min(p.N, r0 + p.B);
  double cost = 0.0;
  unsigned int ch = 0;
  for (int64_t r = r0 + tid; r < r1; r += kSNT) {
    const int lab = p.labels[r];
    if ((unsigned)lab < (unsigned)p.K) {  // -1: a row with NaN, in no cluster
      atomicAdd(&sh_h[lab], 1);
      cost += (double)p.mind[r];
      ch += p.prev ? (p.prev[r] != lab) : 1u;
    }
  }
  cost = wave_sum(cost);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) ch += __shfl_xor(ch, o, 64);
  if ((tid & 63) == 0) {
    red[tid >> 6] = cost;
    red_c[tid >> 6] = ch;
  }
  __syncthreads();
  if (tid == 0) {
    p.pcost[w] = ((red[0] + red[1]) + red[2]) + red[3];
    p.pchg[w] = red_c[0] + red_c[1] + red_c[2] + red_c[3];
  }
  for (int j = tid; j < p.K; j += kSNT) p.hist[(int64_t)j * p.Wh + w] = sh_h[j];
}

// One wave per cluster: exclusive prefix of its block counts (in place) and
// its size.
__global__ __launch_bounds__(kSNT) void lloyd_cscan_kernel(LloydParams p) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * (kSNT / 64) + (threadIdx.x >> 6);
  if (j >= p.K) return;  // whole waves; no barriers below
  int32_t* h = p.hist + (int64_t)j * p.Wh;
  int run = 0;
  for (int w0 = 0; w0 < p.Wh; w0 += 64) {
    const int w = w0 + lane;
    const int v = w < p.Wh ? h[w] : 0;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (w < p.Wh) h[w] = run + x - v;
    run += __shfl(x, 63, 64);
  }
  if (lane == 0) p.pcnt[j] = run;
}

// One workgroup: coff = exclusive prefix of the cluster sizes.
__global__ __launch_bounds__(1024) void lloyd_oscan_kernel(LloydParams p) {
  __shared__ int sh[1024];
  const int per = (p.K + 1023) / 1024;
  const int b0 = min(p.K, (int)threadIdx.x * per), b1 = min(p.K, b0 + per);
  int s = 0;
  for (int i = b0; i < b1; ++i) s += p.pcnt[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int i = 0; i < 1024; ++i) {
      const int v = sh[i];
      sh[i] = run;
      run += v;
    }
    p.coff[p.K] = run;
  }
  __syncthreads();
  int off = sh[threadIdx.x];
  for (int i = b0; i < b1; ++i) {
    p.coff[i] = off;
    off += p.pcnt[i];
  }
}

// Block w: row r with label j goes to order[coff[j] + hist[j][w] + its rank
// among the block's rows of cluster j] (the rank order is arbitrary; the sums
// do not depend on it).
__global__ __launch_bounds__(kSNT) void lloyd_scatter_kernel(LloydParams p) {
  extern __shared__ int cur[];  // [K]
  const int tid = threadIdx.x, w = blockIdx.x;
  for (int j = tid; j < p.K; j += kSNT) cur[j] = p.coff[j] + p.hist[(int64_t)j * p.Wh + w];
  __syncthreads();
  const int64_t r0 = (int64_t)w * p.B, r1 = min(p.N, r0 + p.B);
  for (int64_t r = r0 + tid; r < r1; r += kSNT) {
    const int lab = p.labels[r];
    if ((unsigned)lab < (unsigned)p.K) p.order[atomicAdd(&cur[lab], 1)] = (int32_t)r;
  }
}

__global__ __launch_bounds__(kSNT) void lloyd_zero_kernel(long long* a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kSNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kSNT) a[i] = 0;
}

// Workgroup c: sorted positions [c * CH, (c + 1) * CH) cut into runs of one
// cluster; the four waves take every fourth row of a run with lanes over
// the elements (DPL per lane, d <= 64 * DPL) and kRU rows in flight (the
// next rows' indices load with the current rows), the run's sums meet in
// LDS and go to sums[j] (pacc) with integer atomics.
constexpr int kRU = 8;
template <int FMT, int DPL>
__global__ __launch_bounds__(kSNT) void lloyd_runsum_kernel(LloydParams p) {
  __shared__ long long part[kSNT / 64 - 1][64 * DPL];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int M = p.coff[p.K];
  const int64_t s0 = (int64_t)blockIdx.x * p.CH;
  if (s0 >= M) return;  // uniform over the workgroup
  const int64_t s1 = min((int64_t)M, s0 + p.CH);
  // the last cluster starting at or before s0 (it holds s0: s0 < coff[K])
  int lo = 0, hi = p.K - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (p.coff[mid] <= s0)
      lo = mid;
    else
      hi = mid - 1;
  }
  int j = lo;
  const int F = lloyd_F(p);
  int64_t s = s0;
  while (s < s1) {
    const int64_t e = min(s1, (int64_t)p.coff[j + 1]);
    long long acc[DPL];
#pragma unroll
    for (int i = 0; i < DPL; ++i) acc[i] = 0;
    constexpr int64_t kStep = (int64_t)(kSNT / 64) * kRU;
    // every load is unconditional (indices clamped into range, values
    // masked afterwards), so a wave's loads are all in flight together
    int64_t nrow[kRU];
#pragma unroll
    for (int u = 0; u < kRU; ++u) {
      const int64_t q = s + wave + (int64_t)u * (kSNT / 64);
      nrow[u] = p.order[q < e ? q : e - 1];
    }
    for (int64_t q0 = s + wave; q0 < e; q0 += kStep) {
      int64_t row[kRU];
#pragma unroll
      for (int u = 0; u < kRU; ++u) {
        row[u] = nrow[u];
        const int64_t q = q0 + kStep + (int64_t)u * (kSNT / 64);
        nrow[u] = p.order[q < e ? q : e - 1];
      }
      float v[kRU][DPL];
#pragma unroll
      for (int u = 0; u < kRU; ++u)
#pragma unroll
        for (int i = 0; i < DPL; ++i) {
          const int k = lane + 64 * i;
          const float x = lx<FMT>(p, row[u], k < p.d ? k : p.d - 1);
          v[u][i] = (q0 + (int64_t)u * (kSNT / 64) < e && k < p.d) ? x : 0.0f;
        }
#pragma unroll
      for (int u = 0; u < kRU; ++u)
#pragma unroll
        for (int i = 0; i < DPL; ++i) acc[i] += __float2ll_rn(ldexpf(v[u][i], F));
    }
    if (wave > 0)
#pragma unroll
      for (int i = 0; i < DPL; ++i) part[wave - 1][lane + 64 * i] = acc[i];
    __syncthreads();
    if (wave == 0)
#pragma unroll
      for (int i = 0; i < DPL; ++i) {
        const int k = lane + 64 * i;
        const long long t = acc[i] + part[0][lane + 64 * i] + part[1][lane + 64 * i] + part[2][lane + 64 * i];
        if (k < p.d && t != 0)
          atomicAdd(reinterpret_cast<unsigned long long*>(p.pacc + (int64_t)j * p.d + k), (unsigned long long)t);
      }
    __syncthreads();  // part is rewritten by the next run
    s = e;
    ++j;
    while (j < p.K && (int64_t)p.coff[j + 1] <= s) ++j;  // empty clusters
  }
}

// ---------------------------------------------------------------- host
namespace {
inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int64_t kLdsBudget = 65536 - 17408;  // dynamic LDS of one workgroup (static LDS aside)
constexpr int64_t kMaxAmaxWG = 2048;          // max-pass workgroups at most
constexpr int64_t kTargetWG = 512;           // two workgroups per CU (LDS-bound)

struct LloydPlan {
  int G, lgG, R, Kr, W;
  int epl;      // elements per lane per row: a power of two with G * epl >= d
  bool sorted;  // the sorted path (many cluster ranges)
  int Wh, CH, dpl;
  int64_t B;
};

// The sorted path from this many cluster ranges on (K <= 15360 for its LDS
// histograms within 64 KiB, d <= 512 for its registers).
constexpr int kSortedRanges = 4;
constexpr int kSortedMaxK = 15360;
constexpr int kSortedMaxD = 512;

LloydPlan lloyd_plan(int64_t N, int d, int K) {
  LloydPlan P;
  int lg = 0;
  while ((1 << lg) < d && lg < 6) ++lg;
  P.G = 1 << lg;
  P.lgG = lg;
  const int64_t per = (int64_t)d * 8 + 4;  // LDS bytes of one cluster
  const int64_t kr_max = std::max<int64_t>(1, kLdsBudget / per);
  P.R = (int)((K + kr_max - 1) / kr_max);
  P.Kr = (K + P.R - 1) / P.R;
  const int64_t steps = (N + kLNW * kLB * 64 - 1) / (kLNW * kLB * 64);  // one block per wave
  P.W = (int)std::max<int64_t>(1, std::min<int64_t>(steps, kTargetWG / P.R));
  P.epl = 1;
  while (P.epl * P.G < d) P.epl <<= 1;
  P.sorted = P.R >= kSortedRanges && K <= kSortedMaxK && d <= kSortedMaxD;
  P.Wh = (int)std::max<int64_t>(1, std::min<int64_t>(2048, (N + 4095) / 4096));
  P.B = (N + P.Wh - 1) / P.Wh;
  P.CH = 2048;
  P.dpl = 1;
  while (P.dpl * 64 < d) P.dpl <<= 1;
  if (P.sorted) P.W = 1;  // one set of sums, added to with integer atomics
  return P;
}

template <int FMT, int EPL>
hipError_t launch_accum_e(const LloydParams& p, unsigned grid, size_t shmem, hipStream_t s) {
  hipLaunchKernelGGL((lloyd_accum_kernel<FMT, EPL>), dim3(grid), dim3(kLNT), shmem, s, p);
  return hipGetLastError();
}

template <int FMT>
hipError_t launch_accum(const LloydParams& p, int epl, unsigned grid, size_t shmem, hipStream_t s) {
  switch (epl) {
    case 1: return launch_accum_e<FMT, 1>(p, grid, shmem, s);
    case 2: return launch_accum_e<FMT, 2>(p, grid, shmem, s);
    case 4: return launch_accum_e<FMT, 4>(p, grid, shmem, s);
    case 8: return launch_accum_e<FMT, 8>(p, grid, shmem, s);
    case 16: return launch_accum_e<FMT, 16>(p, grid, shmem, s);
    case 32: return launch_accum_e<FMT, 32>(p, grid, shmem, s);
    case 64: return launch_accum_e<FMT, 64>(p, grid, shmem, s);
    default: return hipErrorInvalidValue;
  }
}

template <int FMT, int DPL>
hipError_t launch_runsum_e(const LloydParams& p, unsigned grid, hipStream_t s) {
  hipLaunchKernelGGL((lloyd_runsum_kernel<FMT, DPL>), dim3(grid), dim3(kSNT), 0, s, p);
  return hipGetLastError();
}

template <int FMT>
hipError_t launch_runsum(const LloydParams& p, int dpl, unsigned grid, hipStream_t s) {
  switch (dpl) {
    case 1: return launch_runsum_e<FMT, 1>(p, grid, s);
    case 2: return launch_runsum_e<FMT, 2>(p, grid, s);
    case 4: return launch_runsum_e<FMT, 4>(p, grid, s);
    case 8: return launch_runsum_e<FMT, 8>(p, grid, s);
    default: return hipErrorInvalidValue;
  }
}

// One iteration's sums on the sorted path: histograms, positions, scatter,
// zeroed sums, run sums.
hipError_t launch_sorted(const LloydParams& p, const LloydPlan& P, int dtype, hipStream_t s) {
  const size_t hsh = sizeof(int) * (size_t)p.K;
  const int64_t kd = (int64_t)p.K * p.d;
  hipLaunchKernelGGL(lloyd_hist_kernel, dim3((unsigned)P.Wh), dim3(kSNT), hsh, s, p);
  hipLaunchKernelGGL(lloyd_cscan_kernel, dim3((unsigned)((p.K + kSNT / 64 - 1) / (kSNT / 64))), dim3(kSNT), 0, s, p);
  hipLaunchKernelGGL(lloyd_oscan_kernel, dim3(1), dim3(1024), 0, s, p);
  hipLaunchKernelGGL(lloyd_scatter_kernel, dim3((unsigned)P.Wh), dim3(kSNT), hsh, s, p);
  hipLaunchKernelGGL(lloyd_zero_kernel, dim3((unsigned)std::min<int64_t>(1024, (kd + kSNT - 1) / kSNT)), dim3(kSNT), 0,
                     s, p.pacc, kd);
  if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  const unsigned grid = (unsigned)((p.N + P.CH - 1) / P.CH);
  if (dtype == KMPP_F32) return launch_runsum<FMT_F32>(p, P.dpl, grid, s);
  if (dtype == KMPP_BF16) return launch_runsum<FMT_BF16>(p, P.dpl, grid, s);
  return launch_runsum<FMT_FP8>(p, P.dpl, grid, s);
}

struct LloydLayout {
  size_t assign, mind, labels, pacc, pcnt, pcost, pchg, pamax, changed, hist, order, coff, total;
};

LloydLayout lloyd_layout(int64_t N, int d, int K, int dtype) {
  const LloydPlan P = lloyd_plan(N, d, K);
  LloydLayout L;
  size_t off = sizeof(LloydCtl);
  L.assign = off;
  off += a256(assign_workspace(N, d, K, dtype));
  L.mind = off;
  off += a256(sizeof(float) * (size_t)N);
  L.labels = off;
  off += a256(sizeof(int32_t) * (size_t)N);
  L.pacc = off;
  off += a256(sizeof(long long) * (size_t)P.W * (size_t)K * (size_t)d);
  L.pcnt = off;
  off += a256(sizeof(int32_t) * (size_t)P.W * (size_t)K);
  const size_t nparts = (size_t)std::max(P.W, P.sorted ? P.Wh : 1);
  L.pcost = off;
  off += a256(sizeof(double) * nparts);
  L.pchg = off;
  off += a256(sizeof(uint32_t) * nparts);
  L.pamax = off;
  off += a256(sizeof(float) * kMaxAmaxWG);
  L.changed = off;
  off += 256;
  L.hist = L.order = L.coff = off;
  if (P.sorted) {
    L.hist = off;
    off += a256(sizeof(int32_t) * (size_t)K * (size_t)P.Wh);
    L.order = off;
    off += a256(sizeof(int32_t) * (size_t)N);
    L.coff = off;
    off += a256(sizeof(int32_t) * ((size_t)K + 1));
  }
  L.total = off;
  return L;
}
}  // namespace

size_t lloyd_workspace(int64_t N, int d, int K, int dtype) { return lloyd_layout(N, d, K, dtype).total; }

int launch_lloyd(const void* X, const int8_t* X_exp, int dtype, int64_t N, int d, int K, float* C, int iters,
                 int32_t* out_labels, double* out_cost, int64_t* out_changed, int32_t* out_counts, void* ws,
                 size_t ws_bytes, hipStream_t stream) {
  const LloydLayout L = lloyd_layout(N, d, K, dtype);
  if (ws_bytes < L.total) return KMPP_E_WORKSPACE;
  const LloydPlan P = lloyd_plan(N, d, K);
  char* w = static_cast<char*>(ws);
  LloydParams p;
  p.X = X;
  p.xexp = X_exp;
  p.N = N;
  p.d = d;
  p.K = K;
  p.G = P.G;
  p.lgG = P.lgG;
  p.R = P.R;
  p.Kr = P.Kr;
  p.W = P.W;
  p.mind = reinterpret_cast<float*>(w + L.mind);
  p.C = C;
  p.pacc = reinterpret_cast<long long*>(w + L.pacc);
  p.pcnt = reinterpret_cast<int32_t*>(w + L.pcnt);
  p.pcost = reinterpret_cast<double*>(w + L.pcost);
  p.pchg = reinterpret_cast<uint32_t*>(w + L.pchg);
  p.pamax = reinterpret_cast<float*>(w + L.pamax);
  p.lc = reinterpret_cast<LloydCtl*>(w);
  p.labels = nullptr;
  p.prev = nullptr;
  p.changed = nullptr;
  p.cost = nullptr;
  p.counts_out = nullptr;
  p.Wc = P.W;
  p.Wh = P.Wh;
  p.B = P.B;
  p.CH = P.CH;
  p.hist = reinterpret_cast<int32_t*>(w + L.hist);
  p.order = reinterpret_cast<int32_t*>(w + L.order);
  p.coff = reinterpret_cast<int32_t*>(w + L.coff);
  if (P.sorted) p.Wc = P.Wh;

  const size_t shmem = (size_t)P.Kr * ((size_t)d * 8 + 4);
  const int64_t kd = (int64_t)K * d;
  const unsigned fin_grid = (unsigned)((kd + 255) / 256);
  const unsigned grid = (unsigned)(P.R * P.W);

  hipLaunchKernelGGL(lloyd_reset_kernel, dim3(1), dim3(1), 0, stream, p.lc);
  const int64_t rows_per_step = 4 * (64 >> P.lgG);
  const unsigned amax_grid =
      (unsigned)std::max<int64_t>(1, std::min<int64_t>(dtype == KMPP_FP8_E4M3 ? (N + rows_per_step - 1) / rows_per_step
                                                                              : (N * d / 4 + 1023) / 1024,
                                                       kMaxAmaxWG));
  if (dtype == KMPP_F32)
    hipLaunchKernelGGL(lloyd_absmax_kernel<FMT_F32>, dim3(amax_grid), dim3(256), 0, stream, p);
  else if (dtype == KMPP_BF16)
    hipLaunchKernelGGL(lloyd_absmax_kernel<FMT_BF16>, dim3(amax_grid), dim3(256), 0, stream, p);
  else
    hipLaunchKernelGGL(lloyd_absmax_kernel<FMT_FP8>, dim3(amax_grid), dim3(256), 0, stream, p);
  hipLaunchKernelGGL(lloyd_absmax_final_kernel, dim3(1), dim3(256), 0, stream, p, (int)amax_grid);
  if (hipGetLastError() != hipSuccess) return KMPP_E_HIP;

  int32_t* ws_labels = reinterpret_cast<int32_t*>(w + L.labels);
  for (int t = 0; t < iters; ++t) {
    // the last iteration writes out_labels
    int32_t* dst = ((iters - 1 - t) % 2 == 0) ? out_labels : ws_labels;
    int32_t* other = dst == out_labels ? ws_labels : out_labels;
    const int rc = launch_assign(X, X_exp, dtype, C, N, d, K, dst, const_cast<float*>(p.mind), w + L.assign,
                                 L.mind - L.assign, stream);
    if (rc != KMPP_OK) return rc;
    p.labels = dst;
    p.prev = t > 0 ? other : nullptr;
    p.changed = out_changed ? reinterpret_cast<unsigned long long*>(out_changed + t)
                            : reinterpret_cast<unsigned long long*>(w + L.changed);
    p.cost = out_cost ? out_cost + t : nullptr;
    p.counts_out = t == iters - 1 ? out_counts : nullptr;
    hipError_t e;
    if (P.sorted) {
      e = launch_sorted(p, P, dtype, stream);
    } else if (dtype == KMPP_F32) {
      e = launch_accum<FMT_F32>(p, P.epl, grid, shmem, stream);
    } else if (dtype == KMPP_BF16) {
      e = launch_accum<FMT_BF16>(p, P.epl, grid, shmem, stream);
    } else {
      e = launch_accum<FMT_FP8>(p, P.epl, grid, shmem, stream);
    }
    if (e != hipSuccess) return KMPP_E_HIP;
    hipLaunchKernelGGL(lloyd_finalize_kernel, dim3(fin_grid), dim3(256), 0, stream, p);
    if (hipGetLastError() != hipSuccess) return KMPP_E_HIP;
  }
  return KMPP_OK;
}

}  // namespace kmpp
