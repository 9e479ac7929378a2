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
// summed exactly.  Each workgroup first adds its rows into a private copy of
// the sums in LDS when K * d is small enough, then adds that copy to the
// global sums once.
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
  const int32_t* labels;      // this iteration's assignment
  const int32_t* prev;        // the previous iteration's, or null (first iteration)
  const float* mind;          // distance of every row to its centre
  float* C;                   // [K, d], updated in place
  long long* acc;             // [K * d] fixed-point sums
  int32_t* cnt;               // [K] cluster sizes
  double* part;               // [gridDim] per-workgroup cost sums
  int32_t nparts;
  unsigned long long* changed;  // rows whose label changed, or null
  double* cost;               // sum of mind, or null
  int32_t* counts_out;        // cluster sizes out, or null
  LloydCtl* lc;
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

__global__ void lloyd_reset_kernel(LloydCtl* lc) {
  lc->status = KMPP_OK;
  lc->amax_bits = 0u;
}

// max |x| over all rows; a NaN or infinite value sets KMPP_E_NONFINITE.
template <int FMT>
__global__ __launch_bounds__(256) void lloyd_absmax_kernel(LloydParams p) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sub = lane & (p.G - 1), rg = lane >> p.lgG;
  const int rpw = 64 >> p.lgG;
  float m = 0.0f;
  bool bad = false;
  for (int64_t row = ((int64_t)blockIdx.x * 4 + wave) * rpw + rg; row < p.N; row += (int64_t)gridDim.x * 4 * rpw)
    for (int k = sub; k < p.d; k += p.G) {
      const float a = fabsf(lx<FMT>(p, row, k));
      bad |= !(a <= 3.4028235e38f);
      m = fmaxf(m, a);
    }
  m = wave_minf(-m);
  if (lane == 0) atomicMax(&p.lc->amax_bits, __float_as_uint(-m));
  if (bad) raise_status(reinterpret_cast<Ctl*>(p.lc), KMPP_E_NONFINITE);
}

__global__ __launch_bounds__(256) void lloyd_clear_kernel(LloydParams p) {
  const int64_t n = (int64_t)p.K * p.d;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) p.acc[e] = 0;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < p.K; j += (int64_t)gridDim.x * 256) p.cnt[j] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0 && p.changed) *p.changed = 0ull;
}

// Cluster sums, sizes, the cost and the changed-label count of one
// iteration.  G lanes per row, 64/G rows per wave, workgroups stride over
// the rows in a fixed order (so the FP64 cost partials are reproducible).
template <int FMT, bool LDS>
__global__ __launch_bounds__(256) void lloyd_accum_kernel(LloydParams p) {
  extern __shared__ long long sh_acc[];  // LDS: [K * d] sums, then [K] int sizes
  __shared__ double red[4];
  __shared__ unsigned int red_ch[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int sub = lane & (p.G - 1), rg = lane >> p.lgG;
  const int rpw = 64 >> p.lgG;
  const int64_t kd = (int64_t)p.K * p.d;
  long long* acc = LDS ? sh_acc : p.acc;
  int* cnt = LDS ? reinterpret_cast<int*>(sh_acc + kd) : p.cnt;
  if constexpr (LDS) {
    for (int64_t e = tid; e < kd; e += 256) sh_acc[e] = 0;
    for (int j = tid; j < p.K; j += 256) cnt[j] = 0;
    __syncthreads();
  }
  const int F = lloyd_F(p);
  double cost = 0.0;
  unsigned int changed = 0;
  for (int64_t row = ((int64_t)blockIdx.x * 4 + wave) * rpw + rg; row < p.N; row += (int64_t)gridDim.x * 4 * rpw) {
    const int lab = p.labels[row];
    if ((unsigned)lab >= (unsigned)p.K) continue;  // label -1: a row with NaN (status set by the max pass)
    long long* a = acc + (int64_t)lab * p.d;
    for (int k = sub; k < p.d; k += p.G) {
      const long long v = __float2ll_rn(ldexpf(lx<FMT>(p, row, k), F));
      atomicAdd(reinterpret_cast<unsigned long long*>(a + k), (unsigned long long)v);
    }
    if (sub == 0) {
      atomicAdd(cnt + lab, 1);
      cost += (double)p.mind[row];
      changed += p.prev ? (p.prev[row] != lab) : 1u;
    }
  }
  if constexpr (LDS) {
    __syncthreads();
    for (int64_t e = tid; e < kd; e += 256) {
      const long long v = sh_acc[e];
      if (v) atomicAdd(reinterpret_cast<unsigned long long*>(p.acc + e), (unsigned long long)v);
    }
    for (int j = tid; j < p.K; j += 256)
      if (cnt[j]) atomicAdd(p.cnt + j, cnt[j]);
  }
  cost = wave_sum(cost);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) changed += __shfl_xor(changed, o, 64);
  if (lane == 0) {
    red[wave] = cost;
    red_ch[wave] = changed;
  }
  __syncthreads();
  if (tid == 0) {
    p.part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
    const unsigned int c = red_ch[0] + red_ch[1] + red_ch[2] + red_ch[3];
    if (p.changed && c) atomicAdd(p.changed, (unsigned long long)c);
  }
}

// New centres (empty clusters keep theirs), sizes, and the cost as the sum
// of the workgroup partials in a fixed order.
__global__ __launch_bounds__(256) void lloyd_finalize_kernel(LloydParams p) {
  __shared__ double red[4];
  const int F = lloyd_F(p);
  const int64_t kd = (int64_t)p.K * p.d;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < kd) {
    const int n = p.cnt[e / p.d];
    if (n > 0) p.C[e] = (float)(ldexp((double)p.acc[e], -F) / (double)n);
  }
  if (p.counts_out && e < p.K) p.counts_out[e] = p.cnt[e];
  if (blockIdx.x == 0 && p.cost) {
    const int per = (p.nparts + 255) / 256;
    const int b0 = threadIdx.x * per;
    double s = 0.0;
    for (int i = b0; i < min(p.nparts, b0 + per); ++i) s += p.part[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *p.cost = ((red[0] + red[1]) + red[2]) + red[3];
  }
}

// ---------------------------------------------------------------- host
namespace {
inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int kMaxParts = 4096;            // accumulation workgroups at most
constexpr size_t kLdsBudget = 60 << 10;   // private sums in LDS up to this size

struct LloydLayout {
  size_t assign, mind, labels, acc, cnt, part, changed, total;
};

LloydLayout lloyd_layout(int64_t N, int d, int K, int dtype) {
  LloydLayout L;
  size_t off = sizeof(LloydCtl);
  L.assign = off;
  off += a256(assign_workspace(N, d, K, dtype));
  L.mind = off;
  off += a256(sizeof(float) * (size_t)N);
  L.labels = off;
  off += a256(sizeof(int32_t) * (size_t)N);
  L.acc = off;
  off += a256(sizeof(long long) * (size_t)K * (size_t)d);
  L.cnt = off;
  off += a256(sizeof(int32_t) * (size_t)K);
  L.part = off;
  off += a256(sizeof(double) * kMaxParts);
  L.changed = off;
  off += 256;
  L.total = off;
  return L;
}

template <int FMT>
hipError_t launch_accum(const LloydParams& p, bool lds, int grid, size_t shmem, hipStream_t s) {
  if (lds)
    hipLaunchKernelGGL((lloyd_accum_kernel<FMT, true>), dim3(grid), dim3(256), shmem, s, p);
  else
    hipLaunchKernelGGL((lloyd_accum_kernel<FMT, false>), dim3(grid), dim3(256), 0, s, p);
  return hipGetLastError();
}
}  // namespace

size_t lloyd_workspace(int64_t N, int d, int K, int dtype) { return lloyd_layout(N, d, K, dtype).total; }

int launch_lloyd(const void* X, const int8_t* X_exp, int dtype, int64_t N, int d, int K, float* C, int iters,
                 int32_t* out_labels, double* out_cost, int64_t* out_changed, int32_t* out_counts, void* ws,
                 size_t ws_bytes, hipStream_t stream) {
  const LloydLayout L = lloyd_layout(N, d, K, dtype);
  if (ws_bytes < L.total) return KMPP_E_WORKSPACE;
  char* w = static_cast<char*>(ws);
  LloydParams p;
  p.X = X;
  p.xexp = X_exp;
  p.N = N;
  p.d = d;
  p.K = K;
  int lg = 0;
  while ((1 << lg) < d && lg < 6) ++lg;
  p.G = 1 << lg;
  p.lgG = lg;
  p.mind = reinterpret_cast<float*>(w + L.mind);
  p.C = C;
  p.acc = reinterpret_cast<long long*>(w + L.acc);
  p.cnt = reinterpret_cast<int32_t*>(w + L.cnt);
  p.part = reinterpret_cast<double*>(w + L.part);
  p.lc = reinterpret_cast<LloydCtl*>(w);
  p.counts_out = nullptr;

  const size_t lds_bytes = sizeof(long long) * (size_t)K * d + sizeof(int) * (size_t)K;
  const bool lds = lds_bytes <= kLdsBudget;
  const int64_t rows_per_wg = 4 * (64 >> lg);
  const int64_t want = (N + rows_per_wg - 1) / rows_per_wg;
  const int grid = (int)std::min<int64_t>(want, lds ? 512 : kMaxParts);
  p.nparts = grid;
  const int64_t kd = (int64_t)K * d;
  const unsigned fin_grid = (unsigned)((std::max<int64_t>(kd, K) + 255) / 256);

  hipLaunchKernelGGL(lloyd_reset_kernel, dim3(1), dim3(1), 0, stream, p.lc);
  p.labels = nullptr;
  p.prev = nullptr;
  p.changed = nullptr;
  p.cost = nullptr;
  const unsigned amax_grid = (unsigned)std::min<int64_t>(want, 2048);
  if (dtype == KMPP_F32)
    hipLaunchKernelGGL(lloyd_absmax_kernel<FMT_F32>, dim3(amax_grid), dim3(256), 0, stream, p);
  else if (dtype == KMPP_BF16)
    hipLaunchKernelGGL(lloyd_absmax_kernel<FMT_BF16>, dim3(amax_grid), dim3(256), 0, stream, p);
  else
    hipLaunchKernelGGL(lloyd_absmax_kernel<FMT_FP8>, dim3(amax_grid), dim3(256), 0, stream, p);
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
    hipLaunchKernelGGL(lloyd_clear_kernel, dim3((unsigned)std::min<int64_t>((kd + 255) / 256, 1024)), dim3(256), 0,
                       stream, p);
    hipError_t e;
    if (dtype == KMPP_F32)
      e = launch_accum<FMT_F32>(p, lds, grid, lds_bytes, stream);
    else if (dtype == KMPP_BF16)
      e = launch_accum<FMT_BF16>(p, lds, grid, lds_bytes, stream);
    else
      e = launch_accum<FMT_FP8>(p, lds, grid, lds_bytes, stream);
    if (e != hipSuccess) return KMPP_E_HIP;
    hipLaunchKernelGGL(lloyd_finalize_kernel, dim3(fin_grid), dim3(256), 0, stream, p);
    if (hipGetLastError() != hipSuccess) return KMPP_E_HIP;
  }
  return KMPP_OK;
}

}  // namespace kmpp
