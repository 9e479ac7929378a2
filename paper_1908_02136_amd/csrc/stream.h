// stream.h -- the row streamer shared by the seed pass and the batched
// kernel: D = min(D, ||x - c||^2) over a range of rows.
#pragma once

#include "kmpp_dev.h"
#include "kmpp_impl.h"

namespace kmpp {

// A row of d elements is split into chunks of CB bytes; a group of G lanes
// covers one row (G*CPL chunks), so one wave-wide load reads 64/G whole
// consecutive rows.  Each lane keeps the centre slice of its chunks in
// registers, the row distance is reduced across the G lanes with xor
// shuffles, and U loads per lane are issued before any is consumed.
// iter() handles the R = U*64/G rows of one wave starting at `base` and
// hands every row's new nearest distance to `sink(row, dnew, changed)`; a row's
// arithmetic depends only on the template parameters, not on where the
// rows (RL: ROW_CACHED, ROW_NONTEMPORAL or ROW_BUFFER) or the centre come
// from.
template <int FMT, int CB, int G, int CPL, int U, bool FULL, int NT, int RL = ROW_CACHED>
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
  // ROW_BUFFER: a resource over this workgroup's rows [rfirst, r1)
  __amdgpu_buffer_rsrc_t rs;
  int64_t rfirst;

  // The loaded state of one iteration: rows, FP8 row scales, old D.
  struct Batch {
    RawT raw[U][CPL];
    float sc[U];
    float dold[NJ];
  };

  __device__ __forceinline__ void layout() {
    const int lane = threadIdx.x & 63;
    wave = threadIdx.x >> 6;
    sub = lane % G;
    rg = lane / G;
  }

  // Each lane reads its own slice of the centre (from LDS, or per lane from
  // global memory).
  template <class Ptr>
  __device__ __forceinline__ void set_centre(Ptr cs, int d) {
    const int nchunk = d / VEC;
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
      const int c = sub + G * k;
#pragma unroll
      for (int e = 0; e < VEC; ++e) cen[k][e] = (FULL || c < nchunk) ? cs[c * VEC + e] : 0.0f;
    }
  }

  // The whole centre through the scalar unit: the same address in every
  // lane, so the loads are scalar (scalar data cache, values in SGPRs), then
  // each lane selects its slice.  Exact widths only (d = G * CPL * VEC).
  __device__ __forceinline__ void set_centre_uniform(const float* cg) {
    static_assert(FULL, "scalar centre loads need a compile-time width");
    constexpr int DD = G * CPL * VEC;
    float c[DD];
#pragma unroll
    for (int j = 0; j < DD; ++j) c[j] = cg[j];
#pragma unroll
    for (int k = 0; k < CPL; ++k)
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        float v = c[(G * k) * VEC + e];
#pragma unroll
        for (int s = 1; s < G; ++s) v = (sub == s) ? c[(s + G * k) * VEC + e] : v;
        cen[k][e] = v;
      }
  }

  // ROW_BUFFER: bind the rows [r0, r1) (at most 2^31 bytes).
  __device__ __forceinline__ void set_rows(const void* xs, int64_t r0, int64_t r1, int d) {
    if constexpr (RL == ROW_BUFFER) {
      const int64_t rb = (int64_t)d * EB;
      rs = make_rows_rsrc(static_cast<const char*>(xs) + r0 * rb, (uint32_t)((r1 - r0) * rb));
      rfirst = r0;
    }
  }

  __device__ __forceinline__ void init(const float* cs, int d) {
    layout();
    set_centre(cs, d);
  }

  // Issue the loads of this wave's R rows starting at `base` (rows >= r1
  // are clamped in bounds and later discarded); needs no centre.
  __device__ __forceinline__ void load(const SeedParams& p, int64_t base, int64_t r1, bool first, Batch& b) const {
    const int d = p.d;
    const int nchunk = d / VEC;
    const gptr<const char> xb = as_global(static_cast<const char*>(p.xs));
    const gptr<const float> Dg = as_global(static_cast<const float*>(p.D));
    const gptr<const int8_t> xe = as_global(p.xexp);
    const int64_t rb = (int64_t)d * EB;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int uu = sub + G * j;
      const int64_t row = base + (int64_t)uu * RPL + rg;
      b.dold[j] = (!first && uu < U && row < r1) ? Dg[row] : INFINITY;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int64_t row = base + u * RPL + rg;
      if constexpr (RL == ROW_BUFFER) {
        // rows past the tile read as zero through the range check
        const uint32_t ro = (uint32_t)((row - rfirst) * rb);
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
          const int c = sub + G * k;
          if (FULL || c < nchunk)
            b.raw[u][k] = load_raw_buf<CB>(rs, ro + (uint32_t)(c * CB));
          else
            b.raw[u][k] = RawT{};
        }
        row = row < r1 ? row : r1 - 1;
      } else {
        row = row < r1 ? row : r1 - 1;  // in bounds; the value is discarded
        const gptr<const char> rp = xb + row * rb;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
          const int c = sub + G * k;
          if (FULL || c < nchunk)
            b.raw[u][k] = load_raw<CB, RL>(rp + (int64_t)c * CB);
          else
            b.raw[u][k] = RawT{};
        }
      }
      if constexpr (FMT == FMT_FP8) b.sc[u] = exp2i((int)xe[row]);
    }
  }

  // Distances of a loaded batch to the centre, new D to `sink(row, dnew)`.
  template <class Sink>
  __device__ __forceinline__ void compute(int64_t base, int64_t r1, bool first, int64_t prev, const Batch& b,
                                          Sink&& sink) const {
    float delta[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      float a = 0.0f;
#pragma unroll
      for (int k = 0; k < CPL; ++k) {
        float v[VEC];
        decode<FMT, CB>(b.raw[u][k], v);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const float df = (FMT == FMT_FP8) ? fmaf(v[e], b.sc[u], -cen[k][e]) : v[e] - cen[k][e];
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
        float dn = first ? dv : fminf(b.dold[j], dv);
        if constexpr (FMT != FMT_F32) dn = (row == prev) ? 0.0f : dn;
        // most rows keep their nearest distance once a few seeds exist:
        // `changed` lets the sink skip their store
        sink(row, dn, first || !(dn == b.dold[j]));
      }
    }
  }

  // One iteration: load, then compute.
  template <class Sink>
  __device__ __forceinline__ void iter(const SeedParams& p, int64_t base, int64_t r1, bool first, int64_t prev,
                                       Sink&& sink) const {
    Batch b;
    load(p, base, r1, first, b);
    compute(base, r1, first, prev, b, sink);
  }
};

}  // namespace kmpp
