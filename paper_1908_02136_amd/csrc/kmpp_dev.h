// kmpp_dev.h -- device-side building blocks shared by the libkmpp kernels:
// the Philox4x32-10 stream, storage-format decoding, wavefront / workgroup
// reductions and scans, and the status word.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kmpp.h"

namespace kmpp {

enum : int { FMT_F32 = KMPP_F32, FMT_BF16 = KMPP_BF16, FMT_FP8 = KMPP_FP8_E4M3 };

template <int FMT>
struct ElemBytes;
template <>
struct ElemBytes<FMT_F32> { static constexpr int value = 4; };
template <>
struct ElemBytes<FMT_BF16> { static constexpr int value = 2; };
template <>
struct ElemBytes<FMT_FP8> { static constexpr int value = 1; };

// First 256 bytes of every workspace.
struct Ctl {
  int32_t status;      // KMPP_OK, a warning (>0) or an error (<0)
  uint32_t arrive;     // reserved (0)
  uint32_t nflag;      // assignment: rows queued for the direct-form recheck
  uint32_t nqueue;     // assignment, BF16/FP8 rows: rows the first stage left to the second
  uint64_t lead;       // seed loop, lead-workgroup draw: (pass << 32) | drawn row
  uint32_t pad[58];
};
static_assert(sizeof(Ctl) == 256, "control block is 256 bytes");

// Errors replace OK or a warning; a warning replaces only OK.
__device__ inline void raise_status(Ctl* ctl, int32_t code) {
  int32_t* st = &ctl->status;
  int32_t cur = __hip_atomic_load(st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  while (true) {
    if (cur < 0 || (code > 0 && cur != KMPP_OK)) return;
    if (__hip_atomic_compare_exchange_strong(st, &cur, code, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return;
  }
}

// ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 products with a Weyl key schedule.
__device__ __forceinline__ uint4 philox4x32_10(uint4 x, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t ha = __umulhi(0xD2511F53u, x.x), la = 0xD2511F53u * x.x;
    const uint32_t hb = __umulhi(0xCD9E8D57u, x.z), lb = 0xCD9E8D57u * x.z;
    x = make_uint4(hb ^ x.y ^ k0, lb, ha ^ x.w ^ k1, la);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return x;
}

// u in [0,1) with 53 random bits: counter (step, instance, 0, tag); tag 0
// is the k-means++ stream, other tags separate other streams of a run.
__device__ __forceinline__ double draw_uniform(uint64_t seed, uint32_t step, uint32_t inst, uint32_t tag = 0u) {
  const uint4 r = philox4x32_10(make_uint4(step, inst, 0u, tag), (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t m = ((uint64_t)(r.x >> 5) << 26) | (uint64_t)(r.y >> 6);
  return (double)m * 0x1p-53;
}

__device__ __forceinline__ int64_t uniform_index(double u, int64_t N) {
  const int64_t i = (int64_t)floor(__dmul_rn(u, (double)N));
  return i < N - 1 ? i : N - 1;
}

// Pointers into device memory as global-address-space pointers, so loads
// through pointers read from memory (not kernel arguments) still compile to
// global rather than flat instructions.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> as_global(T* p) {
  return (gptr<T>)p;
}

// 2^e as a float for e in [-126, 127].
__device__ __forceinline__ float exp2i(int e) { return __int_as_float((e + 127) << 23); }

// ---- raw chunk types by byte width
template <int CB>
struct Raw;
template <>
struct Raw<16> { using T = uint4; };
template <>
struct Raw<8> { using T = uint2; };
template <>
struct Raw<4> { using T = uint32_t; };
template <>
struct Raw<2> { using T = uint16_t; };
template <>
struct Raw<1> { using T = uint8_t; };

typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));

// Where a pass reads the point rows from (the seed-pass kernels take one as
// a template parameter):
//   ROW_CACHED       plain global loads, cached in L2 and the last-level cache;
//   ROW_NONTEMPORAL  non-temporal global loads, for rows read once per pass
//                    that do not fit the caches;
//   ROW_BUFFER       loads through a buffer resource: a 128-bit descriptor
//                    (base, size) held in scalar registers, 32-bit offsets,
//                    and a hardware range check that returns 0 outside it --
//                    the read-only, descriptor-addressed path nearest to a
//                    texture fetch.
enum : int { ROW_CACHED = 0, ROW_NONTEMPORAL = 1, ROW_BUFFER = 2 };

// Where every lane of a seed pass takes the current centre from (Section II
// compares keeping the centroids in global and in constant memory):
//   CEN_LDS     the workgroup copies the row into LDS once, lanes read their
//               slice from there (one barrier);
//   CEN_SCALAR  scalar loads of the whole row into SGPRs through the scalar
//               data cache (uniform, read-only: the constant-cache path),
//               exact widths only;
//   CEN_GLOBAL  every lane loads its own slice with vector loads (L2 hits
//               after the first workgroup).
enum : int { CEN_LDS = 0, CEN_SCALAR = 1, CEN_GLOBAL = 2 };

// One CB-byte chunk through a global pointer (ROW_CACHED, ROW_NONTEMPORAL).
template <int CB, int RL = ROW_CACHED>
__device__ __forceinline__ typename Raw<CB>::T load_raw(gptr<const char> p) {
  constexpr bool NTL = RL == ROW_NONTEMPORAL;
  if constexpr (CB == 16) {
    const v4u v = NTL ? __builtin_nontemporal_load((gptr<const v4u>)p) : *(gptr<const v4u>)p;
    return make_uint4(v.x, v.y, v.z, v.w);
  } else if constexpr (CB == 8) {
    const v2u v = NTL ? __builtin_nontemporal_load((gptr<const v2u>)p) : *(gptr<const v2u>)p;
    return make_uint2(v.x, v.y);
  } else {
    using T = typename Raw<CB>::T;
    return NTL ? __builtin_nontemporal_load((gptr<const T>)p) : *(gptr<const T>)p;
  }
}

// Buffer resource over `bytes` bytes at `base` (raw, stride 0; the third
// descriptor word selects 32-bit data on gfx9-family chips).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rows_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// One CB-byte chunk at byte offset `off` of a buffer resource (ROW_BUFFER);
// chunks past the resource's size read as zero.
template <int CB>
__device__ __forceinline__ typename Raw<CB>::T load_raw_buf(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (CB == 16) {
    const v4u v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    return make_uint4(v.x, v.y, v.z, v.w);
  } else if constexpr (CB == 8) {
    const v2u v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    return make_uint2(v.x, v.y);
  } else if constexpr (CB == 4) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
  } else if constexpr (CB == 2) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
  } else {
    return __builtin_amdgcn_raw_buffer_load_b8(r, off, 0, 0);
  }
}

template <int CB>
__device__ __forceinline__ uint32_t raw_word(const typename Raw<CB>::T& r, int w) {
  if constexpr (CB == 16) {
    return w == 0 ? r.x : w == 1 ? r.y : w == 2 ? r.z : r.w;
  } else if constexpr (CB == 8) {
    return w == 0 ? r.x : r.y;
  } else {
    return (uint32_t)r;
  }
}

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// Decode one chunk of CB bytes in format FMT into VEC floats (FP8 unscaled).
template <int FMT, int CB>
__device__ __forceinline__ void decode(const typename Raw<CB>::T& r, float* v) {
  if constexpr (FMT == FMT_F32) {
#pragma unroll
    for (int w = 0; w < CB / 4; ++w) v[w] = __uint_as_float(raw_word<CB>(r, w));
  } else if constexpr (FMT == FMT_BF16) {
    if constexpr (CB >= 4) {
#pragma unroll
      for (int w = 0; w < CB / 4; ++w) {
        const uint32_t x = raw_word<CB>(r, w);
        v[2 * w] = bf16_lo(x);
        v[2 * w + 1] = bf16_hi(x);
      }
    } else {
      v[0] = __uint_as_float((uint32_t)r << 16);
    }
  } else {  // FP8 E4M3FN, the gfx950 native 8-bit float format
    if constexpr (CB >= 4) {
#pragma unroll
      for (int w = 0; w < CB / 4; ++w) {
        const int x = (int)raw_word<CB>(r, w);
        const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8(x, false);
        const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8(x, true);
        v[4 * w] = lo[0];
        v[4 * w + 1] = lo[1];
        v[4 * w + 2] = hi[0];
        v[4 * w + 3] = hi[1];
      }
    } else {
      v[0] = __builtin_amdgcn_cvt_f32_fp8((int)(uint32_t)r, 0);
    }
  }
}

// ---- wavefront (64 lanes) and workgroup reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int64_t wave_min(int64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t w = __shfl_xor(v, o, 64);
    v = w < v ? w : v;
  }
  return v;
}
__device__ __forceinline__ int64_t wave_max(int64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}
__device__ __forceinline__ float wave_minf(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  return v;
}

// Exclusive prefix over the workgroup of one double per thread, in a fixed
// association order (wave-level Hillis-Steele, then wave offsets in order),
// so every call on the same inputs gives the same bits.  `sh` holds at least
// NT/64 + 1 doubles.  Returns the exclusive prefix; *total = sum of all.
template <int NT>
__device__ __forceinline__ double block_exclusive_scan(double v, double* sh, double* total) {
  constexpr int NW = NT / 64;
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
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < NW; ++w) {
      const double t = sh[w];
      sh[w] = r;
      r += t;
    }
    sh[NW] = r;
  }
  __syncthreads();
  const double res = sh[wave] + ex;
  *total = sh[NW];
  __syncthreads();
  return res;
}

template <int NT>
__device__ __forceinline__ int64_t block_min(int64_t v, int64_t* sh) {
  constexpr int NW = NT / 64;
  v = wave_min(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  int64_t r = sh[0];
  for (int w = 1; w < NW; ++w) r = sh[w] < r ? sh[w] : r;
  __syncthreads();
  return r;
}

template <int NT>
__device__ __forceinline__ int64_t block_max(int64_t v, int64_t* sh) {
  constexpr int NW = NT / 64;
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  int64_t r = sh[0];
  for (int w = 1; w < NW; ++w) r = sh[w] > r ? sh[w] : r;
  __syncthreads();
  return r;
}

template <int NT>
__device__ __forceinline__ float block_minf(float v, float* sh) {
  constexpr int NW = NT / 64;
  v = wave_minf(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = sh[0];
  for (int w = 1; w < NW; ++w) r = fminf(r, sh[w]);
  __syncthreads();
  return r;
}

}  // namespace kmpp
