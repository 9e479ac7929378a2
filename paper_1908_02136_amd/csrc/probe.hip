// probe.hip -- read-bandwidth probe: a measurement helper, not part of the
// method.  It reads a buffer once with 8 16-byte loads per lane in flight
// (grid-stride) and writes one FP32 partial sum per workgroup, the
// attainable-bandwidth denominator for the seed pass's rate.
#include "kmpp_dev.h"
#include "kmpp_impl.h"

namespace kmpp {

template <int RL>
__global__ __launch_bounds__(256) void read_probe_kernel(const char* buf, size_t n16, float* out) {
  __shared__ double red[4];
  const gptr<const char> x = as_global(buf);
  const size_t stride = (size_t)gridDim.x * 256;
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  float a = 0.0f;
  for (; i + 7 * stride < n16; i += 8 * stride) {
    uint4 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = load_raw<16, RL>(x + (i + k * stride) * 16);
#pragma unroll
    for (int k = 0; k < 8; ++k)
      a += (__uint_as_float(v[k].x) + __uint_as_float(v[k].y)) + (__uint_as_float(v[k].z) + __uint_as_float(v[k].w));
  }
  for (; i < n16; i += stride) {
    const uint4 v = load_raw<16, RL>(x + i * 16);
    a += (__uint_as_float(v.x) + __uint_as_float(v.y)) + (__uint_as_float(v.z) + __uint_as_float(v.w));
  }
  const double s = wave_sum((double)a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (float)((red[0] + red[1]) + (red[2] + red[3]));
}

}  // namespace kmpp

using namespace kmpp;

extern "C" int kmpp_read_probe(const void* buf, size_t bytes, int32_t blocks, int32_t nontemporal,
                               float* out_partial, void* stream) {
  if (!buf || !out_partial || bytes == 0 || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(buf) % 16 != 0 ||
      blocks < 1 || blocks > 65536 || (nontemporal != 0 && nontemporal != 1))
    return KMPP_E_INVALID;
  const void* fn = nontemporal ? reinterpret_cast<const void*>(&read_probe_kernel<ROW_NONTEMPORAL>)
                               : reinterpret_cast<const void*>(&read_probe_kernel<ROW_CACHED>);
  const char* b = static_cast<const char*>(buf);
  size_t n16 = bytes / 16;
  void* args[] = {&b, &n16, &out_partial};
  return hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(256), args, 0, static_cast<hipStream_t>(stream)) ==
                 hipSuccess
             ? KMPP_OK
             : KMPP_E_HIP;
}
