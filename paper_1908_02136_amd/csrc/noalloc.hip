// noalloc.hip -- kmpp_seed_noalloc: the seed loop of kmpp_seed for callers
// that cannot allocate device memory (code under graph capture, serving
// loops, harnesses that forbid allocation).
//
// The workspace kmpp_seed takes from its caller (the control block with the
// status word, the FP64 tile sums, the D buffers and indices a call does not
// bring) lives here in a file-scope device array, sized for the largest
// accepted input, N = K = KMPP_NOALLOC_MAX_N rows.  Each device the library
// runs on holds its own copy from the load of the library's code object
// until the process ends.  In host code the array's name is a host-side
// stand-in, not a device address: the address of the current device's copy
// comes from hipGetSymbolAddress, taken once per device and kept below, and
// only that address is handed to the kernels.
//
// Every call on a device shares that device's copy and leaves its contents
// behind.  Nothing in it has to start at zero: the first-seed kernel resets
// the control block, and every pass writes the tile sums and D values
// before any later kernel reads them.  Calls that overlap on one device (on
// different streams, or from different threads without ordering) race on
// the array.
#include <mutex>

#include "kmpp_dev.h"
#include "kmpp_impl.h"

namespace kmpp {

constexpr size_t kNoAllocScratchBytes = seed_layout(KMPP_NOALLOC_MAX_N, KMPP_NOALLOC_MAX_N).total;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// The current device's copy of `scratch`, looked up on the first call made
// with that device current.
int scratch_on_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return KMPP_E_HIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return KMPP_E_HIP;
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return KMPP_OK;
}

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }
}  // namespace

}  // namespace kmpp

using namespace kmpp;

extern "C" int kmpp_seed_noalloc(const float* X, int64_t N, int32_t d, int32_t K, uint64_t seed,
                                 float* out_centers, float* out_D, int64_t* out_idx, const void* Xq,
                                 const int8_t* Xq_exp, int32_t dtype, const kmpp_seed_opts* opts,
                                 int32_t* out_status, void* stream) {
  if (!X || !out_centers) return KMPP_E_INVALID;
  if (N < 1 || K < 1 || K > N || N > INT32_MAX || d < 1 || d > KMPP_MAX_D) return KMPP_E_INVALID;
  if (dtype != KMPP_F32 && dtype != KMPP_BF16 && dtype != KMPP_FP8_E4M3) return KMPP_E_INVALID;
  if (!aligned16(X)) return KMPP_E_INVALID;
  if (dtype != KMPP_F32) {
    if (!Xq || !aligned16(Xq)) return KMPP_E_INVALID;
    if (dtype == KMPP_FP8_E4M3 && !Xq_exp) return KMPP_E_INVALID;
  }
  if (opts && (opts->draw < KMPP_DRAW_AUTO || opts->draw > KMPP_DRAW_SINGLE)) return KMPP_E_INVALID;
  if (N > KMPP_NOALLOC_MAX_N) return KMPP_E_TOO_LARGE;
  void* ws = nullptr;
  const int rc = scratch_on_current_device(&ws);
  if (rc != KMPP_OK) return rc;
  return seed_run(X, N, d, K, seed, opts ? opts->instance : 0u, 0u, nullptr, out_centers, out_D, out_idx, Xq,
                  Xq_exp, dtype, opts, ws, kNoAllocScratchBytes, static_cast<hipStream_t>(stream), out_status);
}
