// assign.hip -- nearest-seed assignment, the partition O of the paper's
// Algorithm 1 (Section II), as a dense contraction on the matrix cores.
//
// score(i, j) = ||c_j||^2 - 2 <x_i, c_j> has the same argmin over j as
// ||x_i - c_j||^2.  The products run on MFMA with FP32 accumulation:
//   FP32 rows: v_mfma_f32_16x16x4_f32;
//   BF16 rows: v_mfma_f32_16x16x32_bf16 against the centres split into a
//              BF16 high part and a BF16 remainder (two products), so only
//              the rows carry storage rounding;
//   FP8 rows:  each E4M3 code converted exactly to BF16, the BF16 path, and
//              the row's power-of-two scale applied to the product.
// A wave owns RB blocks of 16 rows, keeps their operand fragments in
// registers for the whole loop over centre tiles of 16, and keeps a running
// best and second-best score per row.  The contraction index is permuted
// (lane group q of a row takes the q-th contiguous quarter of the padded
// row) so fragment loads are contiguous; the centres are packed once into
// exactly that order.
//
// A row's best index is final when its score gap to the second best exceeds
// twice the products' error bound
//   E = (c1 d + c2) u (max_j ||c_j||^2 + 2 ||x|| max_j ||c_j||) * 1.05,
// u = 2^-24 (FP32 accumulation; BF16 adds 2^-16 for the centre split).
// Other rows are queued and re-evaluated against every centre in the direct
// FP32 form sum_k (x_k - c_jk)^2, ties to the smallest index.
#include "kmpp_dev.h"
#include "kmpp_impl.h"

namespace kmpp {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

struct AssignParams {
  const void* X;
  const int8_t* xexp;
  const float* C;       // [K, d] FP32
  const void* Cp;       // packed B fragments
  float* cn;            // [Kp] ||c_j||^2 (FP32, direct)
  Ctl* ctl;             // nflag counter
  int32_t* flags;       // [N] queued rows
  int32_t* labels;
  float* mind;
  float* cmax2;         // max_j ||c_j||^2 (workspace scalar)
  int64_t N;
  int32_t d, K, Kp, dp; // dp = padded d: 4 * VPL * (steps per tile)
  int32_t nblk;         // number of 16-row blocks
  int32_t all_rows;     // recheck kernel: every row instead of the queue
};

// ---- per-format row fragment handling
template <int FMT>
struct Frag;

// FP32: one MFMA contracts 4 values, one per lane group.
template <>
struct Frag<FMT_F32> {
  static constexpr int VPL = 1;  // values per lane per step
  using A = float;
};
// BF16 / FP8 (as BF16): one MFMA contracts 32 values, 8 per lane group.
template <>
struct Frag<FMT_BF16> {
  static constexpr int VPL = 8;
  using A = v8bf;
};
template <>
struct Frag<FMT_FP8> : Frag<FMT_BF16> {};

__device__ __forceinline__ __bf16 bf_from_bits(uint16_t b) { return __builtin_bit_cast(__bf16, b); }

// Merge (s1, i1, s2) with another lane's (t1, j1, t2): ties on the best
// score keep the smaller index and make the gap zero.
__device__ __forceinline__ void top2_merge(float& s1, int& i1, float& s2, float t1, int j1, float t2) {
  if (t1 < s1 || (t1 == s1 && j1 < i1)) {
    s2 = fminf(s1, t2);
    s1 = t1;
    i1 = j1;
  } else {
    s2 = fminf(s2, t1);
  }
}

// Load the FP32-valued x_k (dequantised) of row `row`, columns [k0, k0+n).
template <int FMT>
__device__ __forceinline__ float x_at(const AssignParams& p, int64_t row, int k);

template <>
__device__ __forceinline__ float x_at<FMT_F32>(const AssignParams& p, int64_t row, int k) {
  return static_cast<const float*>(p.X)[row * p.d + k];
}
template <>
__device__ __forceinline__ float x_at<FMT_BF16>(const AssignParams& p, int64_t row, int k) {
  return __uint_as_float((uint32_t) static_cast<const uint16_t*>(p.X)[row * p.d + k] << 16);
}
template <>
__device__ __forceinline__ float x_at<FMT_FP8>(const AssignParams& p, int64_t row, int k) {
  const uint8_t q = static_cast<const uint8_t*>(p.X)[row * p.d + k];
  return __builtin_amdgcn_cvt_f32_fp8((int)q, 0) * exp2i((int)p.xexp[row]);
}

// ---------------------------------------------------------------- prep
// ||c_j||^2 (direct FP32), its maximum, and the packed B fragments.
// FP32: Cp[jt][s][lane] = C[16 jt + lane%16][q*DQ + s], q = lane/16,
//       DQ = dp/4 (steps per lane group), s < DQ.
// BF16: Cp[jt][h][s][lane] = 8 BF16 of part h (0 high, 1 remainder) of
//       C[16 jt + lane%16][q*DQ + 8 s + 0..7], DQ = dp/4, s < DQ/8.
__global__ __launch_bounds__(256) void assign_prep_kernel(AssignParams p, int fmt) {
  const int Kt = p.Kp / 16;
  const int DQ = p.dp / 4;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = tid; j < p.Kp; j += stride) {
    float a = 0.0f;
    if (j < p.K)
      for (int k = 0; k < p.d; ++k) {
        const float c = p.C[j * p.d + k];
        a = fmaf(c, c, a);
      }
    p.cn[j] = a;
    if (j < p.K) atomicMax(reinterpret_cast<unsigned int*>(p.cmax2), __float_as_uint(a));
  }
  if (fmt == FMT_F32) {
    float* Cp = (float*)const_cast<void*>(p.Cp);
    const int64_t total = (int64_t)Kt * DQ * 64;
    for (int64_t e = tid; e < total; e += stride) {
      const int lane = (int)(e % 64);
      const int s = (int)((e / 64) % DQ);
      const int jt = (int)(e / 64 / DQ);
      const int j = 16 * jt + lane % 16, k = (lane / 16) * DQ + s;
      Cp[e] = (j < p.K && k < p.d) ? p.C[(int64_t)j * p.d + k] : 0.0f;
    }
  } else {
    uint16_t* Cp = (uint16_t*)const_cast<void*>(p.Cp);
    const int S = DQ / 8;
    const int64_t total = (int64_t)Kt * 2 * S * 64 * 8;
    for (int64_t e = tid; e < total; e += stride) {
      const int t = (int)(e % 8);
      const int lane = (int)((e / 8) % 64);
      const int s = (int)((e / 512) % S);
      const int h = (int)((e / 512 / S) % 2);
      const int jt = (int)(e / 512 / S / 2);
      const int j = 16 * jt + lane % 16, k = (lane / 16) * DQ + 8 * s + t;
      const float c = (j < p.K && k < p.d) ? p.C[(int64_t)j * p.d + k] : 0.0f;
      const uint32_t hb = __float_as_uint(c);
      const uint32_t hi = ((hb + 0x7FFFu + ((hb >> 16) & 1u)) >> 16) & 0xFFFFu;  // RNE
      const float rem = c - __uint_as_float(hi << 16);                              // exact
      const uint32_t rb = __float_as_uint(rem);
      const uint32_t lo = ((rb + 0x7FFFu + ((rb >> 16) & 1u)) >> 16) & 0xFFFFu;
      Cp[e] = (uint16_t)(h == 0 ? hi : lo);
    }
  }
}

// ---------------------------------------------------------------- main
template <int FMT, int DQK, int RB>
__global__ __launch_bounds__(256) void assign_mfma_kernel(AssignParams p) {
  using F = Frag<FMT>;
  constexpr int S = DQK;  // MFMA steps per centre tile (per product): dp / (4 * VPL)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, col = lane & 15;
  const int DQ = p.dp / 4;  // contraction elements per lane group
  const int Kt = p.Kp / 16;
  __shared__ float s_gap[4][RB * 16];
  __shared__ int s_best[4][RB * 16];

  const int64_t blk0 = ((int64_t)blockIdx.x * 4 + wave) * RB;  // first 16-row block of this wave
  if (blk0 >= p.nblk) return;                                  // whole wave idle (no barriers below)

  // ---- row fragments (registers for the whole centre loop) and ||x||^2
  typename F::A a[RB][S];
  float xs[RB];  // partial sum of x^2 over this lane's quarter
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    int64_t row = (blk0 + rb) * 16 + col;
    const bool ok = row < p.N;
    row = ok ? row : p.N - 1;
    float acc = 0.0f;
    if constexpr (FMT == FMT_F32) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int k = q * DQ + s;
        const float v = (ok && k < p.d) ? static_cast<const float*>(p.X)[row * p.d + k] : 0.0f;
        a[rb][s] = v;
        acc = fmaf(v, v, acc);
      }
    } else {
      const float sc = (FMT == FMT_FP8) ? exp2i((int)p.xexp[row]) : 1.0f;
#pragma unroll
      for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int k = q * DQ + 8 * s + t;
          uint16_t bits = 0;
          float xv = 0.0f;
          if (ok && k < p.d) {
            if constexpr (FMT == FMT_BF16) {
              bits = static_cast<const uint16_t*>(p.X)[row * p.d + k];
              xv = __uint_as_float((uint32_t)bits << 16);
            } else {
              const uint8_t c8 = static_cast<const uint8_t*>(p.X)[row * p.d + k];
              const float f = __builtin_amdgcn_cvt_f32_fp8((int)c8, 0);  // exact in BF16
              bits = (uint16_t)(__float_as_uint(f) >> 16);
              xv = f * sc;
            }
          }
          a[rb][s][t] = bf_from_bits(bits);
          acc = fmaf(xv, xv, acc);
        }
      }
    }
    xs[rb] = acc;
  }

  // ---- running top-2 per (row block, accumulator row)
  float s1[RB][4], s2[RB][4];
  int i1[RB][4];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      s1[rb][v] = INFINITY;
      s2[rb][v] = INFINITY;
      i1[rb][v] = INT_MAX;
    }

  for (int jt = 0; jt < Kt; ++jt) {
    v4f acc[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) acc[rb] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (FMT == FMT_F32) {
      const float* bp = static_cast<const float*>(p.Cp) + ((int64_t)jt * DQ) * 64 + lane;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const float b = bp[s * 64];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][s], b, acc[rb], 0, 0, 0);
      }
    } else {
      const uint4* bp = static_cast<const uint4*>(p.Cp) + ((int64_t)jt * 2 * S) * 64 + lane;
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const uint4 bw = bp[(h * S + s) * 64];
          const v8bf b = __builtin_bit_cast(v8bf, bw);
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rb][s], b, acc[rb], 0, 0, 0);
        }
    }
    const int j = jt * 16 + col;
    const float cnj = j < p.K ? p.cn[j] : INFINITY;
    if constexpr (FMT == FMT_FP8) {
      // accumulator v holds row 16*blk + 4q + v: apply its scale
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          int64_t row = (blk0 + rb) * 16 + 4 * q + v;
          row = row < p.N ? row : p.N - 1;
          acc[rb][v] *= exp2i((int)p.xexp[row]);
        }
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float sc = fmaf(-2.0f, acc[rb][v], cnj);
        if (sc < s1[rb][v]) {
          s2[rb][v] = s1[rb][v];
          s1[rb][v] = sc;
          i1[rb][v] = j;
        } else if (sc < s2[rb][v]) {
          s2[rb][v] = sc;
        }
      }
  }

  // ---- merge across the 16 lanes that share rows (different centres)
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        const float t1 = __shfl_xor(s1[rb][v], o, 64);
        const int j1 = __shfl_xor(i1[rb][v], o, 64);
        const float t2 = __shfl_xor(s2[rb][v], o, 64);
        top2_merge(s1[rb][v], i1[rb][v], s2[rb][v], t1, j1, t2);
      }
      if (col == 0) {
        s_gap[wave][rb * 16 + 4 * q + v] = s2[rb][v] - s1[rb][v];
        s_best[wave][rb * 16 + 4 * q + v] = i1[rb][v];
      }
    }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

  // ---- per row (lanes of a row: same col, q = 0..3): ||x||, bound, direct
  // distance to the best centre over this lane's quarter
  const float cmax2 = *p.cmax2;
  const float cmax = sqrtf(cmax2);
  constexpr float kGrowth = 1.05f;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    float x2 = xs[rb];
    x2 += __shfl_xor(x2, 16, 64);
    x2 += __shfl_xor(x2, 32, 64);
    const int64_t row = (blk0 + rb) * 16 + col;
    const int best = s_best[wave][rb * 16 + col];
    const float gap = s_gap[wave][rb * 16 + col];
    const float xn = sqrtf(x2) * 1.0001f;
    const float mag = cmax2 + 2.0f * xn * cmax;
    const float unit =
        (FMT == FMT_F32) ? (float)(p.dp + 8) * 0x1p-24f : (float)(2 * p.dp + 8) * 0x1p-24f + 0x1p-16f;
    const float E = unit * mag * kGrowth;
    const bool sure = gap > 2.0f * E && best < p.K;
    // direct distance to the best centre: this lane's quarter
    float dd = 0.0f;
    const int bj = best < p.K ? best : 0;
    if (row < p.N) {
      for (int s = 0; s < DQ; ++s) {
        const int k = q * DQ + s;
        if (k < p.d) {
          const float df = x_at<FMT>(p, row, k) - p.C[(int64_t)bj * p.d + k];
          dd = fmaf(df, df, dd);
        }
      }
    }
    dd += __shfl_xor(dd, 16, 64);
    dd += __shfl_xor(dd, 32, 64);
    if (q == 0 && row < p.N) {
      if (sure) {
        p.labels[row] = best;
        if (p.mind) p.mind[row] = dd;
      } else {
        const uint32_t slot = atomicAdd(&p.ctl->nflag, 1u);
        p.flags[slot] = (int32_t)row;
      }
    }
  }
}

// ---------------------------------------------------------------- recheck
// One wave per queued row: direct FP32 distances to every centre, lanes
// split over centres, ties to the smallest index.
template <int FMT>
__global__ __launch_bounds__(256) void assign_recheck_kernel(AssignParams p) {
  const int lane = threadIdx.x & 63;
  const int64_t n = p.all_rows ? p.N : (int64_t)p.ctl->nflag;
  const int64_t waves = (int64_t)gridDim.x * 4;
  for (int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); w < n; w += waves) {
    const int64_t row = p.all_rows ? w : (int64_t)p.flags[w];
    float best = INFINITY;
    int bi = INT_MAX;
    for (int j = lane; j < p.K; j += 64) {
      float a = 0.0f;
      for (int k = 0; k < p.d; ++k) {
        const float df = x_at<FMT>(p, row, k) - p.C[(int64_t)j * p.d + k];
        a = fmaf(df, df, a);
      }
      if (a < best) {
        best = a;
        bi = j;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const float tb = __shfl_xor(best, o, 64);
      const int ti = __shfl_xor(bi, o, 64);
      if (tb < best || (tb == best && ti < bi)) {
        best = tb;
        bi = ti;
      }
    }
    if (lane == 0) {
      // no comparable distance (NaN in the row or the centres): label -1
      p.labels[row] = bi < p.K ? bi : -1;
      if (p.mind) p.mind[row] = bi < p.K ? best : __builtin_nanf("");
    }
  }
}

__global__ void assign_reset_kernel(Ctl* ctl, float* cmax2) {
  ctl->status = KMPP_OK;
  ctl->nflag = 0u;
  *cmax2 = 0.0f;
}

// ---------------------------------------------------------------- host
namespace {
inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }
inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

struct AssignLayout {
  size_t cn, cmax, cp, flags, total;
  int Kp, dp;
};

// MFMA steps per centre tile for width d: a power of two so the padded row
// splits evenly over the 4 lane groups; 0 if d is beyond the MFMA path.
int assign_steps(int d, int dtype) {
  const int vpl = dtype == KMPP_F32 ? 1 : 8;
  const int maxs = dtype == KMPP_F32 ? 32 : 8;
  int s = 1;
  while (4 * vpl * s < d) s <<= 1;
  return s <= maxs ? s : 0;
}

AssignLayout assign_layout(int64_t N, int d, int K, int dtype) {
  AssignLayout L;
  L.Kp = round_up(K, 16);
  const int steps = assign_steps(d, dtype);
  L.dp = steps ? 4 * (dtype == KMPP_F32 ? 1 : 8) * steps : round_up(d, 4);
  size_t off = sizeof(Ctl);
  L.cn = off;
  off += a256(sizeof(float) * L.Kp);
  L.cmax = off;
  off += 256;
  L.cp = off;
  off += a256(dtype == KMPP_F32 ? sizeof(float) * (size_t)L.Kp * L.dp : sizeof(uint16_t) * 2 * (size_t)L.Kp * L.dp);
  L.flags = off;
  off += a256(sizeof(int32_t) * (size_t)N);
  L.total = off;
  return L;
}

template <int FMT, int DQK, int RB>
hipError_t launch_main(const AssignParams& p, hipStream_t stream) {
  const int64_t waves = (p.nblk + RB - 1) / RB;
  const int64_t blocks = (waves + 3) / 4;
  hipLaunchKernelGGL((assign_mfma_kernel<FMT, DQK, RB>), dim3((unsigned)blocks), dim3(256), 0, stream, p);
  return hipGetLastError();
}

// RB row blocks per wave: fragment registers RB * steps * (1 or 4) <= 64
template <int FMT>
hipError_t dispatch_main(const AssignParams& p, int steps, hipStream_t stream) {
  if constexpr (FMT == FMT_F32) {
    switch (steps) {
      case 1: return launch_main<FMT, 1, 4>(p, stream);
      case 2: return launch_main<FMT, 2, 4>(p, stream);
      case 4: return launch_main<FMT, 4, 4>(p, stream);
      case 8: return launch_main<FMT, 8, 4>(p, stream);
      case 16: return launch_main<FMT, 16, 2>(p, stream);
      case 32: return launch_main<FMT, 32, 1>(p, stream);
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (steps) {
      case 1: return launch_main<FMT, 1, 4>(p, stream);
      case 2: return launch_main<FMT, 2, 4>(p, stream);
      case 4: return launch_main<FMT, 4, 2>(p, stream);
      case 8: return launch_main<FMT, 8, 1>(p, stream);
      default: return hipErrorInvalidValue;
    }
  }
}
}  // namespace

size_t assign_workspace(int64_t N, int d, int K, int dtype) { return assign_layout(N, d, K, dtype).total; }

int launch_assign(const void* X, const int8_t* X_exp, int dtype, const float* C, int64_t N, int d, int K,
                  int32_t* labels, float* mind, void* ws, size_t ws_bytes, hipStream_t stream) {
  const AssignLayout L = assign_layout(N, d, K, dtype);
  if (ws_bytes < L.total) return KMPP_E_WORKSPACE;
  char* w = static_cast<char*>(ws);
  AssignParams p;
  p.X = X;
  p.xexp = X_exp;
  p.C = C;
  p.Cp = w + L.cp;
  p.cn = reinterpret_cast<float*>(w + L.cn);
  p.ctl = reinterpret_cast<Ctl*>(w);
  p.flags = reinterpret_cast<int32_t*>(w + L.flags);
  p.labels = labels;
  p.mind = mind;
  p.cmax2 = reinterpret_cast<float*>(w + L.cmax);
  p.N = N;
  p.d = d;
  p.K = K;
  p.Kp = L.Kp;
  p.dp = L.dp;
  p.nblk = (int)((N + 15) / 16);

  p.all_rows = 0;

  hipLaunchKernelGGL(assign_reset_kernel, dim3(1), dim3(1), 0, stream, p.ctl, p.cmax2);
  const int steps = assign_steps(d, dtype);
  if (steps) {
    hipLaunchKernelGGL(assign_prep_kernel, dim3(256), dim3(256), 0, stream, p, dtype);
    hipError_t e;
    if (dtype == KMPP_F32)
      e = dispatch_main<FMT_F32>(p, steps, stream);
    else if (dtype == KMPP_BF16)
      e = dispatch_main<FMT_BF16>(p, steps, stream);
    else
      e = dispatch_main<FMT_FP8>(p, steps, stream);
    if (e != hipSuccess) return KMPP_E_HIP;
  } else {
    p.all_rows = 1;  // wider than the MFMA path: every row in the direct form
  }
  const unsigned rb = 2048;
  if (dtype == KMPP_F32)
    hipLaunchKernelGGL(assign_recheck_kernel<FMT_F32>, dim3(rb), dim3(256), 0, stream, p);
  else if (dtype == KMPP_BF16)
    hipLaunchKernelGGL(assign_recheck_kernel<FMT_BF16>, dim3(rb), dim3(256), 0, stream, p);
  else
    hipLaunchKernelGGL(assign_recheck_kernel<FMT_FP8>, dim3(rb), dim3(256), 0, stream, p);
  return hipGetLastError() == hipSuccess ? KMPP_OK : KMPP_E_HIP;
}

}  // namespace kmpp
