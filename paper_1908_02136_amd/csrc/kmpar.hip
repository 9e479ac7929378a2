// kmpar.hip -- k-means|| initialisation (Bahmani, Moseley, Vattani, Kumar,
// Vassilvitskii, "Scalable K-Means++", PVLDB 2012, Algorithm 2), which the
// paper's introduction names as the different initialisation of Bahmani et
// al.  Steps:
//   1. a uniform first point;
//   2. R rounds: every point joins the candidates independently with
//      probability min(1, ell * D / phi), D the squared distance to the
//      nearest candidate, phi = sum D (FP64, fixed order);
//   3. every candidate is weighted by the points whose nearest candidate it
//      is (ties to the smaller candidate index);
//   4. weighted k-means++ over the candidates picks the K centres (first
//      proportional to w, then to w * D).
// Random numbers: Philox4x32-10 keyed by the seed, counters (0, inst, 0, 0)
// for the first point, (i, inst, r, 1) for point i in round r >= 1 and
// (m, inst, 0, 2) for recluster draw m.
//
// Per round: the candidates that joined last are gathered into a
// contiguous block and every point is assigned to them with the matrix-core
// assignment (assign.hip: direct-form distance of the chosen candidate,
// ties to the smaller index); a merge keeps the nearer of the old and new
// candidate (strict comparison, so earlier candidates win exact ties) and
// writes the FP64 tile sums of D; phi is added from the tile sums in a fixed
// order; the joiners are counted per tile, scanned, and written in point
// order.  The host reads each round's list length (one stream
// synchronisation per round) to size the next assignment.  After the last
// round: weights from the labels (LDS histograms), then the weighted
// k-means++ recluster runs on the gathered candidates with the seed-loop
// kernels (seed.hip, weighted mode, Philox stream tag 2).
#include "kmpp_dev.h"
#include "kmpp_impl.h"

namespace kmpp {

struct KparCtl {
  int32_t ncand;     // candidates so far
  int32_t pad[63];
};
static_assert(sizeof(KparCtl) == 256, "256 bytes");

struct KparParams {
  const float* X;
  int64_t N;
  int32_t d, K, R;
  double ell;
  uint64_t seed;
  uint32_t inst;
  int32_t cap;           // candidate capacity
  int32_t round;         // current round r (0 = the first point only)
  int32_t iter;          // rows per thread per tile
  int32_t ntiles;
  Ctl* ctl;              // status
  KparCtl* kc;
  int32_t* round_end;    // [R + 1] candidates after the first point and after each round
  double* phi;           // [R]
  float* D;              // [N]
  int32_t* labels;       // [N] nearest candidate
  double* tsum;          // [ntiles]
  int32_t* tcount;       // [ntiles]
  int32_t* toff;         // [ntiles]
  int64_t* cand;         // [cap] point index of each candidate
  int32_t* w;            // [cap] weights
  float* Cg;             // [cap, d] gathered candidate rows
  int32_t* lab_new;      // [N] nearest of the candidates just gathered
  float* mind_new;       // [N] its distance
  int32_t from;          // first list position of the gathered candidates
  int32_t first;         // 1: the first merge (D starts at +inf)
  int64_t* idx_c;        // [K] recluster picks as list positions
  int64_t* out_idx;      // [K] point indices of the centres, or null
};

constexpr int kPNT = 256;    // threads of the row kernels

__global__ void kmpar_init_kernel(KparParams p) {
  p.ctl->status = KMPP_OK;
  const double u0 = draw_uniform(p.seed, 0u, p.inst);
  p.cand[0] = uniform_index(u0, p.N);
  p.kc->ncand = 1;
  p.round_end[0] = 1;
}

// u in [0,1) from counter (c0, c1, c2, c3), 53 bits as in draw_uniform.
__device__ __forceinline__ double kp_uniform(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
  const uint4 r = philox4x32_10(make_uint4(c0, c1, c2, c3), (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t m = ((uint64_t)(r.x >> 5) << 26) | (uint64_t)(r.y >> 6);
  return (double)m * 0x1p-53;
}

// Cg[j] = X[cand[from + j]] for j < n (contiguous rows for the assignment
// or the recluster).
__global__ __launch_bounds__(256) void kmpar_gather_kernel(KparParams p, int n) {
  const int64_t total = (int64_t)n * p.d;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t j = e / p.d, k = e % p.d;
    p.Cg[e] = p.X[p.cand[p.from + j] * (int64_t)p.d + k];
  }
}

// D, labels := the nearer of the current candidate and the one just
// assigned (strict comparison: earlier candidates win exact ties); the
// FP64 tile sums of D for phi.
__global__ __launch_bounds__(kPNT) void kmpar_merge_kernel(KparParams p) {
  __shared__ double red[kPNT / 64];
  const int tid = threadIdx.x;
  const int64_t t0 = (int64_t)blockIdx.x * kPNT * p.iter;
  double acc = 0.0;
  for (int it = 0; it < p.iter; ++it) {
    const int64_t row = t0 + (int64_t)it * kPNT + tid;
    if (row < p.N) {
      const float dn = p.mind_new[row];
      float dv = p.first ? INFINITY : p.D[row];
      if (p.first || dn < dv) {
        dv = dn;
        const int ln = p.lab_new[row];
        p.D[row] = dn;
        p.labels[row] = ln >= 0 ? p.from + ln : -1;
      }
      acc += (double)dv;
    }
  }
  acc = wave_sum(acc);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kPNT / 64; ++w) s += red[w];
    p.tsum[blockIdx.x] = s;
  }
}

// The recluster's device status joins this run's.
__global__ void kmpar_status_kernel(KparParams p, const Ctl* sub) {
  const int32_t st = sub->status;
  if (st != KMPP_OK) raise_status(p.ctl, st);
}

// out_idx[k] = cand[idx_c[k]]: list positions to point indices.
__global__ void kmpar_map_kernel(KparParams p) {
  for (int k = threadIdx.x; k < p.K; k += blockDim.x) p.out_idx[k] = p.cand[p.idx_c[k]];
}

// phi of this round: the tile sums added in a fixed order (one workgroup).
__global__ __launch_bounds__(256) void kmpar_phi_kernel(KparParams p) {
  __shared__ double sh[8];
  const int per = (p.ntiles + 255) / 256;
  const int b0 = threadIdx.x * per;
  double s = 0.0;
  for (int i = b0; i < min(p.ntiles, b0 + per); ++i) s += p.tsum[i];
  double tot;
  (void)block_exclusive_scan<256>(s, sh, &tot);
  if (threadIdx.x == 0) {
    p.phi[p.round] = tot;
    if (!isfinite(tot)) raise_status(p.ctl, KMPP_E_NONFINITE);
  }
}

// Whether point `row` joins in this round (round index p.round, 0-based:
// counter word 2 is round + 1).
__device__ __forceinline__ bool kp_joins(const KparParams& p, int64_t row, double phi) {
  if (!(phi > 0.0)) return false;
  double pr = p.ell * (double)p.D[row] / phi;
  pr = pr < 1.0 ? pr : 1.0;
  const double u = kp_uniform(p.seed, (uint32_t)row, p.inst, (uint32_t)(p.round + 1), 1u);
  return u < pr;
}

__global__ __launch_bounds__(kPNT) void kmpar_count_kernel(KparParams p) {
  __shared__ int red[kPNT / 64];
  const int tid = threadIdx.x;
  const double phi = p.phi[p.round];
  const int64_t t0 = (int64_t)blockIdx.x * kPNT * p.iter;
  int c = 0;
  for (int it = 0; it < p.iter; ++it) {
    const int64_t row = t0 + (int64_t)it * kPNT + tid;
    if (row < p.N && kp_joins(p, row, phi)) ++c;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((tid & 63) == 0) red[tid >> 6] = c;
  __syncthreads();
  if (tid == 0) {
    int s = 0;
#pragma unroll
    for (int w = 0; w < kPNT / 64; ++w) s += red[w];
    p.tcount[blockIdx.x] = s;
  }
}

// Exclusive scan of the per-tile counts (one workgroup); the new list end.
__global__ __launch_bounds__(256) void kmpar_scan_kernel(KparParams p) {
  __shared__ int sh[256];
  const int per = (p.ntiles + 255) / 256;
  const int b0 = threadIdx.x * per;
  int s = 0;
  for (int i = b0; i < min(p.ntiles, b0 + per); ++i) s += p.tcount[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int i = 0; i < 256; ++i) {
      const int v = sh[i];
      sh[i] = run;
      run += v;
    }
    const int64_t end = (int64_t)p.kc->ncand + run;
    if (end > p.cap) raise_status(p.ctl, KMPP_E_WORKSPACE);
    const int e = (int)min<int64_t>(end, p.cap);
    p.round_end[p.round + 1] = e;
    p.kc->ncand = e;
  }
  __syncthreads();
  int off = p.round_end[p.round] + sh[threadIdx.x];
  for (int i = b0; i < min(p.ntiles, b0 + per); ++i) {
    p.toff[i] = off;
    off += p.tcount[i];
  }
}

// Writes the joiners of every tile in point order from the tile's offset.
__global__ __launch_bounds__(kPNT) void kmpar_write_kernel(KparParams p) {
  __shared__ int sw[kPNT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double phi = p.phi[p.round];
  const int64_t t0 = (int64_t)blockIdx.x * kPNT * p.iter;
  int base = p.toff[blockIdx.x];
  for (int it = 0; it < p.iter; ++it) {
    const int64_t row = t0 + (int64_t)it * kPNT + tid;
    const bool j = row < p.N && kp_joins(p, row, phi);
    const unsigned long long m = __ballot(j);
    const int rk = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) sw[wave] = __popcll(m);
    __syncthreads();
    int before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kPNT / 64; ++w) {
      before += w < wave ? sw[w] : 0;
      total += sw[w];
    }
    const int pos = base + before + rk;
    if (j && pos < p.cap) p.cand[pos] = row;
    base += total;
    __syncthreads();
  }
}

// Weights: points per nearest candidate (LDS histogram when the list fits).
__global__ __launch_bounds__(kPNT) void kmpar_weights_kernel(KparParams p, int lds) {
  extern __shared__ int hist[];
  const int tid = threadIdx.x;
  const int m = p.kc->ncand;
  if (lds) {
    for (int j = tid; j < m; j += kPNT) hist[j] = 0;
    __syncthreads();
  }
  const int64_t t0 = (int64_t)blockIdx.x * kPNT * p.iter;
  for (int it = 0; it < p.iter; ++it) {
    const int64_t row = t0 + (int64_t)it * kPNT + tid;
    if (row < p.N) {
      const int l = p.labels[row];
      if ((unsigned)l < (unsigned)m) atomicAdd(lds ? hist + l : p.w + l, 1);
    }
  }
  if (lds) {
    __syncthreads();
    for (int j = tid; j < m; j += kPNT)
      if (hist[j]) atomicAdd(p.w + j, hist[j]);
  }
}

__global__ void kmpar_wclear_kernel(KparParams p) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < p.cap; j += (int64_t)gridDim.x * 256) p.w[j] = 0;
}

// ---------------------------------------------------------------- host
namespace {
inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

struct KparLayout {
  size_t kc, round_end, phi, D, labels, tsum, tcount, toff, cand, w, Cg, lab_new, mind_new, idx_c, aws, sws, total;
  size_t aws_bytes, sws_bytes;
  int iter, ntiles;
};

KparLayout kpar_layout(int64_t N, int d, int K, int R, int cap) {
  KparLayout L;
  L.iter = (int)std::max<int64_t>(1, (N + (int64_t)kPNT * 4096 - 1) / ((int64_t)kPNT * 4096));
  L.ntiles = (int)((N + (int64_t)kPNT * L.iter - 1) / ((int64_t)kPNT * L.iter));
  size_t off = sizeof(Ctl);
  L.kc = off;
  off += sizeof(KparCtl);
  L.round_end = off;
  off += a256(sizeof(int32_t) * (size_t)(R + 1));
  L.phi = off;
  off += a256(sizeof(double) * (size_t)std::max(R, 1));
  L.D = off;
  off += a256(sizeof(float) * (size_t)N);
  L.labels = off;
  off += a256(sizeof(int32_t) * (size_t)N);
  L.tsum = off;
  off += a256(sizeof(double) * (size_t)L.ntiles);
  L.tcount = off;
  off += a256(sizeof(int32_t) * (size_t)L.ntiles);
  L.toff = off;
  off += a256(sizeof(int32_t) * (size_t)L.ntiles);
  L.cand = off;
  off += a256(sizeof(int64_t) * (size_t)cap);
  L.w = off;
  off += a256(sizeof(int32_t) * (size_t)cap);
  L.Cg = off;
  off += a256(sizeof(float) * (size_t)cap * (size_t)d);
  L.lab_new = off;
  off += a256(sizeof(int32_t) * (size_t)N);
  L.mind_new = off;
  off += a256(sizeof(float) * (size_t)N);
  L.idx_c = off;
  off += a256(sizeof(int64_t) * (size_t)K);
  L.aws_bytes = a256(assign_workspace(N, d, cap, KMPP_F32));
  L.aws = off;
  off += L.aws_bytes;
  L.sws_bytes = a256(seed_workspace(cap, K));
  L.sws = off;
  off += L.sws_bytes;
  L.total = off;
  return L;
}
}  // namespace

int kpar_capacity(int64_t N, int R, double ell) {
  const double per = 3.0 * std::ceil(ell) + 64.0;
  const double c = 1.0 + (double)R * per;
  return (int)std::min<double>((double)N, c);
}

size_t kpar_workspace(int64_t N, int d, int K, int R, double ell) {
  return kpar_layout(N, d, K, R, kpar_capacity(N, R, ell)).total;
}

int launch_kpar(const float* X, int64_t N, int d, int K, uint64_t seed, int R, double ell, uint32_t inst,
                float* out_centers, int64_t* out_idx, int64_t* out_cand, int32_t* out_round_end, int32_t* out_weights,
                int32_t* out_labels, void* ws, size_t ws_bytes, hipStream_t stream) {
  const int cap = kpar_capacity(N, R, ell);
  const KparLayout L = kpar_layout(N, d, K, R, cap);
  if (ws_bytes < L.total) return KMPP_E_WORKSPACE;
  char* w = static_cast<char*>(ws);
  KparParams p;
  p.X = X;
  p.N = N;
  p.d = d;
  p.K = K;
  p.R = R;
  p.ell = ell;
  p.seed = seed;
  p.inst = inst;
  p.cap = cap;
  p.round = 0;
  p.iter = L.iter;
  p.ntiles = L.ntiles;
  p.ctl = reinterpret_cast<Ctl*>(w);
  p.kc = reinterpret_cast<KparCtl*>(w + L.kc);
  p.round_end = out_round_end ? out_round_end : reinterpret_cast<int32_t*>(w + L.round_end);
  p.phi = reinterpret_cast<double*>(w + L.phi);
  p.D = reinterpret_cast<float*>(w + L.D);
  p.labels = out_labels ? out_labels : reinterpret_cast<int32_t*>(w + L.labels);
  p.tsum = reinterpret_cast<double*>(w + L.tsum);
  p.tcount = reinterpret_cast<int32_t*>(w + L.tcount);
  p.toff = reinterpret_cast<int32_t*>(w + L.toff);
  p.cand = out_cand ? out_cand : reinterpret_cast<int64_t*>(w + L.cand);
  p.w = out_weights ? out_weights : reinterpret_cast<int32_t*>(w + L.w);
  p.Cg = reinterpret_cast<float*>(w + L.Cg);
  p.lab_new = reinterpret_cast<int32_t*>(w + L.lab_new);
  p.mind_new = reinterpret_cast<float*>(w + L.mind_new);
  p.idx_c = reinterpret_cast<int64_t*>(w + L.idx_c);
  p.out_idx = out_idx;
  p.from = 0;
  p.first = 1;

  auto gather = [&](int from, int n) {
    p.from = from;
    const unsigned g = (unsigned)std::min<int64_t>(((int64_t)n * d + 255) / 256, 4096);
    hipLaunchKernelGGL(kmpar_gather_kernel, dim3(std::max(1u, g)), dim3(256), 0, stream, p, n);
  };
  // every point against the candidates [from, to): assignment, then merge
  auto fold = [&](int from, int to) -> int {
    gather(from, to - from);
    const int rc = launch_assign(X, nullptr, KMPP_F32, p.Cg, N, d, to - from, p.lab_new, p.mind_new, w + L.aws,
                                 L.aws_bytes, stream);
    if (rc != KMPP_OK) return rc;
    hipLaunchKernelGGL(kmpar_merge_kernel, dim3((unsigned)p.ntiles), dim3(kPNT), 0, stream, p);
    p.first = 0;
    return hipGetLastError() == hipSuccess ? KMPP_OK : KMPP_E_HIP;
  };

  hipLaunchKernelGGL(kmpar_init_kernel, dim3(1), dim3(1), 0, stream, p);
  int m = 1;
  int rc = fold(0, 1);
  if (rc != KMPP_OK) return rc;
  for (int r = 0; r < R; ++r) {
    p.round = r;
    hipLaunchKernelGGL(kmpar_phi_kernel, dim3(1), dim3(256), 0, stream, p);
    hipLaunchKernelGGL(kmpar_count_kernel, dim3((unsigned)p.ntiles), dim3(kPNT), 0, stream, p);
    hipLaunchKernelGGL(kmpar_scan_kernel, dim3(1), dim3(256), 0, stream, p);
    hipLaunchKernelGGL(kmpar_write_kernel, dim3((unsigned)p.ntiles), dim3(kPNT), 0, stream, p);
    if (hipGetLastError() != hipSuccess) return KMPP_E_HIP;
    int32_t next = 0;
    if (hipMemcpyAsync(&next, p.round_end + r + 1, sizeof(int32_t), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return KMPP_E_HIP;
    if (next < m || next > cap) return KMPP_E_HIP;
    if (next > m) {
      rc = fold(m, next);
      if (rc != KMPP_OK) return rc;
    }
    m = next;
  }
  hipLaunchKernelGGL(kmpar_wclear_kernel, dim3(64), dim3(256), 0, stream, p);
  const int lds = cap <= 12288 ? 1 : 0;
  hipLaunchKernelGGL(kmpar_weights_kernel, dim3((unsigned)p.ntiles), dim3(kPNT), lds ? sizeof(int) * (size_t)cap : 0,
                     stream, p, lds);
  if (hipGetLastError() != hipSuccess) return KMPP_E_HIP;
  // weighted k-means++ over the m gathered candidates
  gather(0, m);
  rc = seed_run(p.Cg, m, d, K, seed, inst, 2u, p.w, out_centers, nullptr, p.idx_c, nullptr, nullptr, KMPP_F32,
                nullptr, w + L.sws, L.sws_bytes, stream);
  if (rc != KMPP_OK) return rc;
  hipLaunchKernelGGL(kmpar_status_kernel, dim3(1), dim3(1), 0, stream, p, reinterpret_cast<const Ctl*>(w + L.sws));
  if (out_idx) hipLaunchKernelGGL(kmpar_map_kernel, dim3(1), dim3(256), 0, stream, p);
  return hipGetLastError() == hipSuccess ? KMPP_OK : KMPP_E_HIP;
}

}  // namespace kmpp
