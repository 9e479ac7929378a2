// quant.hip -- storage formats of the precision forms: FP32 rows to BF16
// (round to nearest even) or to FP8 E4M3FN with one power-of-two scale per
// row.  Runs once, before the seed loop; the seed passes then stream 2 or 1
// bytes per coordinate instead of 4.
#include "kmpp_dev.h"
#include "kmpp_impl.h"

namespace kmpp {

__device__ __forceinline__ uint32_t bf16_rne(float x) {
  const uint32_t b = __float_as_uint(x);
  if ((b & 0x7FFFFFFFu) > 0x7F800000u) return (b >> 16) | 0x40u;  // quiet NaN
  return (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
}

// 4 floats per thread, grid-stride.
__global__ __launch_bounds__(256) void quant_bf16_kernel(const float* __restrict__ X, uint16_t* __restrict__ Q,
                                                         int64_t n) {
  const int64_t n4 = n / 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
    const float4 v = reinterpret_cast<const float4*>(X)[i];
    uint2 o;
    o.x = bf16_rne(v.x) | (bf16_rne(v.y) << 16);
    o.y = bf16_rne(v.z) | (bf16_rne(v.w) << 16);
    reinterpret_cast<uint2*>(Q)[i] = o;
  }
  for (int64_t i = n4 * 4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    Q[i] = (uint16_t)bf16_rne(X[i]);
}

// Smallest e with amax <= 448 * 2^e (amax = f * 2^k, f in [0.5, 1)):
// e = k - 9 if f <= 0.875, else k - 8; 0 for a zero or non-finite row;
// clamped to [-117, 127] so 2^e and 2^(e-9) are normal floats.
__device__ __forceinline__ int fp8_row_exponent(float amax) {
  if (!(amax > 0.0f) || !isfinite(amax)) return 0;
  int k;
  const float f = frexpf(amax, &k);
  int e = k - 9 + (f > 0.875f ? 1 : 0);
  e = e < -117 ? -117 : e;
  e = e > 127 ? 127 : e;
  return e;
}

// One wave per row: max |x| by wave reduction, then E4M3FN(x * 2^-e).
__global__ __launch_bounds__(256) void quant_fp8_kernel(const float* __restrict__ X, uint8_t* __restrict__ Q,
                                                        int8_t* __restrict__ E, int64_t N, int d) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); r < N; r += waves) {
    const float* x = X + r * d;
    float amax = 0.0f;
    for (int j = lane; j < d; j += 64) amax = fmaxf(amax, fabsf(x[j]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
    const int e = fp8_row_exponent(amax);
    if (lane == 0) E[r] = (int8_t)e;
    uint8_t* q = Q + r * d;
    if ((d & 3) == 0) {
      for (int j = 4 * lane; j < d; j += 256) {
        const float4 v = *reinterpret_cast<const float4*>(x + j);
        int w = __builtin_amdgcn_cvt_pk_fp8_f32(ldexpf(v.x, -e), ldexpf(v.y, -e), 0, false);
        w = __builtin_amdgcn_cvt_pk_fp8_f32(ldexpf(v.z, -e), ldexpf(v.w, -e), w, true);
        *reinterpret_cast<uint32_t*>(q + j) = (uint32_t)w;
      }
    } else {
      for (int j = lane; j < d; j += 64) {
        const int w = __builtin_amdgcn_cvt_pk_fp8_f32(ldexpf(x[j], -e), 0.0f, 0, false);
        q[j] = (uint8_t)(w & 0xFF);
      }
    }
  }
}

// Widths that are a multiple of 4, up to 256: G lanes per row, each holding
// one 16-byte chunk (G = the power of two >= d / 4), so the row is read
// once; max |x| is reduced over the row's G lanes, and U row groups per lane
// are loaded before any is converted.  Same arithmetic as quant_fp8_kernel.
template <int G>
__global__ __launch_bounds__(256) void quant_fp8_rows_kernel(const float* __restrict__ X, uint8_t* __restrict__ Q,
                                                             int8_t* __restrict__ E, int64_t N, int d) {
  constexpr int U = 4;
  constexpr int RPW = 64 / G;  // rows per wave and row group
  const int lane = threadIdx.x & 63, sub = lane % G, rg = lane / G;
  const int nc = d / 4;        // chunks per row (<= G)
  const bool mine = sub < nc;
  const int64_t wave0 = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t base = wave0 * RPW * U; base < N; base += waves * RPW * U) {
    float4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = base + (int64_t)u * RPW + rg;
      // rows past N and lanes past the row read an in-bounds chunk, unused
      const int64_t rr = r < N ? r : N - 1;
      v[u] = *reinterpret_cast<const float4*>(X + rr * d + 4 * (mine ? sub : 0));
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = base + (int64_t)u * RPW + rg;
      float amax = mine ? fmaxf(fmaxf(fabsf(v[u].x), fabsf(v[u].y)), fmaxf(fabsf(v[u].z), fabsf(v[u].w))) : 0.0f;
#pragma unroll
      for (int o = G / 2; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
      const int e = fp8_row_exponent(amax);
      if (r < N) {
        if (sub == 0) E[r] = (int8_t)e;
        if (mine) {
          int w = __builtin_amdgcn_cvt_pk_fp8_f32(ldexpf(v[u].x, -e), ldexpf(v[u].y, -e), 0, false);
          w = __builtin_amdgcn_cvt_pk_fp8_f32(ldexpf(v[u].z, -e), ldexpf(v[u].w, -e), w, true);
          *reinterpret_cast<uint32_t*>(Q + r * d + 4 * sub) = (uint32_t)w;
        }
      }
    }
  }
}

int launch_quantize(const float* X, int64_t N, int d, int dtype, void* Xq, int8_t* Xq_exp, hipStream_t stream) {
  const int64_t n = N * (int64_t)d;
  if (dtype == KMPP_BF16) {
    const int64_t blocks = std::min<int64_t>(65536, (n / 4 + 255) / 256 + 1);
    hipLaunchKernelGGL(quant_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, X,
                       static_cast<uint16_t*>(Xq), n);
  } else if ((d & 3) == 0 && d <= 256) {
    int g = 1;
    while (g < d / 4) g <<= 1;
    // rows per workgroup per loop step: 4 waves x (64 / g) rows x 4 row groups
    const int64_t rows_per_block = 4 * (64 / g) * 4;
    const int64_t blocks = std::min<int64_t>(65536, (N + rows_per_block - 1) / rows_per_block);
    uint8_t* q = static_cast<uint8_t*>(Xq);
    switch (g) {
      case 1: hipLaunchKernelGGL(quant_fp8_rows_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, stream, X, q, Xq_exp, N, d); break;
      case 2: hipLaunchKernelGGL(quant_fp8_rows_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, stream, X, q, Xq_exp, N, d); break;
      case 4: hipLaunchKernelGGL(quant_fp8_rows_kernel<4>, dim3((unsigned)blocks), dim3(256), 0, stream, X, q, Xq_exp, N, d); break;
      case 8: hipLaunchKernelGGL(quant_fp8_rows_kernel<8>, dim3((unsigned)blocks), dim3(256), 0, stream, X, q, Xq_exp, N, d); break;
      case 16: hipLaunchKernelGGL(quant_fp8_rows_kernel<16>, dim3((unsigned)blocks), dim3(256), 0, stream, X, q, Xq_exp, N, d); break;
      case 32: hipLaunchKernelGGL(quant_fp8_rows_kernel<32>, dim3((unsigned)blocks), dim3(256), 0, stream, X, q, Xq_exp, N, d); break;
      default: hipLaunchKernelGGL(quant_fp8_rows_kernel<64>, dim3((unsigned)blocks), dim3(256), 0, stream, X, q, Xq_exp, N, d); break;
    }
  } else {
    const int64_t blocks = std::min<int64_t>(65536, (N + 3) / 4);
    hipLaunchKernelGGL(quant_fp8_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, X,
                       static_cast<uint8_t*>(Xq), Xq_exp, N, d);
  }
  return hipGetLastError() == hipSuccess ? KMPP_OK : KMPP_E_HIP;
}

}  // namespace kmpp
