// batched.hip -- many independent k-means++ seedings (paper, Section II,
// Algorithms 1-2, one instance each) in ONE persistent launch.
//
// Schedule (host, kmpp_seed_batched_prepare): every instance b gets a gang
// of w_b workgroups (a power of two, 1 for small instances), chosen from a
// cost model so no instance's critical path dominates; gangs are placed
// longest-first onto the W co-resident workgroups (list scheduling).  Each
// workgroup runs its list of (instance, member) items in one global order,
// so the first unfinished item of that order always has all its members
// present: the gang waits cannot cycle.
//
// Member r of a gang owns rows [N r / w, N (r+1) / w); its 4 waves take
// contiguous quarters of that range.  Per seed step a member streams its
// rows (D = min(D, ||x - c||^2)), keeps FP64 sums of blocks of rows in LDS,
// and, for w > 1, publishes its FP64 total in a 64-bit slot whose low 16
// mantissa bits carry the step number (the sum is perturbed by < 2^-36
// relative; every member sees the same values; two banks of slots by step
// parity, since no member can be two steps ahead).  All members read the w
// slots, scan them in a fixed order and compute t = u * total; the member
// whose prefix interval holds t scans its own block sums and rows (its own
// writes: no cross-workgroup visibility of D is needed) and publishes the
// index in a 64-bit flag tagged with the step.  Waits are bounded; an
// expired wait sets KMPP_E_TIMEOUT.
//
// The rows streamed are FP32, BF16 or FP8 (one format per launch, a kernel
// per format); the centres are always the FP32 rows, and with BF16 / FP8
// rows the row of the current centre gets D = 0, as in the single-instance
// seeding.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <queue>
#include <vector>

#include "kmpp_dev.h"
#include "kmpp_impl.h"
#include "stream.h"

namespace kmpp {

constexpr int kBNT = 256;           // threads per workgroup
constexpr int kBNW = kBNT / 64;
constexpr int kBMaxD = 256;         // widest instance (centre row in LDS)
constexpr int kBMaxBlocks = 2048;   // FP64 block sums in LDS per member
constexpr int kBIT = 4;             // wave iterations per block
constexpr int kBMaxGang = 64;

struct BInst {
  const float* X;      // FP32 rows: the centres
  const void* xs;      // the rows the passes stream (X, or BF16 / FP8 rows)
  const int8_t* xexp;  // FP8 row exponents
  float* C;
  float* D;
  int64_t* idx;
  int64_t N;
  int32_t d, K;
  int32_t w;        // gang size
  int32_t slot0;    // first of 2w member slots (two banks by step parity)
};

struct BItem {
  int32_t b;
  int16_t r, w;
};

struct BPlan {
  const BInst* inst;
  const BItem* items;
  const int32_t* begin;  // [W+1] item ranges per workgroup
  uint64_t* mslots;      // member sums (tagged)
  uint64_t* iflag;       // per instance: (step << 32) | index
  Ctl* ctl;
  uint64_t seed;
  uint64_t wait_ticks;   // budget of one gang wait in real-time counter ticks; 0: give up at once
  int32_t n_inst, W, n_mslots;
  int32_t fmt;           // the row format of every instance
};

__device__ __forceinline__ uint64_t tag16(int m) { return 0x8000u | ((uint32_t)m & 0x7FFFu); }

// Bounded wait until (*addr & mask) == want.  The budget (BPlan.wait_ticks,
// on the constant-rate real-time counter) is set by the host from the
// plan's estimated length, so a member that waits for peers still busy with
// earlier items of their lists is not cut off; 0 makes every wait give up at
// once (a host-forced expiry, for testing the error path).  Once any wait of
// the launch has expired, later waits return at once, so the grid drains
// quickly; the results are then undefined and the status says so.
__device__ __forceinline__ uint64_t wait_for(uint64_t* addr, uint64_t mask, uint64_t want, const BPlan& P) {
  if (P.wait_ticks == 0) {
    raise_status(P.ctl, KMPP_E_TIMEOUT);
    return want;
  }
  uint64_t v = __hip_atomic_load(addr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  for (uint32_t i = 0; (v & mask) != want; ++i) {
    if ((i & 255) == 255) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (__builtin_amdgcn_s_memrealtime() - t0 > P.wait_ticks ||
          __hip_atomic_load(&P.ctl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == KMPP_E_TIMEOUT) {
        raise_status(P.ctl, KMPP_E_TIMEOUT);
        return want;
      }
    }
    // the shortest sleep between polls: a gang's members wait for each
    // other every seed step, and longer sleeps (40 x 64 clocks after the
    // first 64 polls) measured 51.7 against 49.3 ms for the 512-instance
    // batch
    __builtin_amdgcn_s_sleep(1);
    v = __hip_atomic_load(addr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return v;
}

struct BShared {
  float cs[kBMaxD];
  double bs[kBMaxBlocks];
  double sh[kBNW];
  int2 shm[kBNW];
  double s_T, s_E, s_lo;
  int64_t s_next;
  int s_owner;
};

// Exclusive scan of one double per thread (fixed order); returns (ex, total).
__device__ __forceinline__ double2 bscan(double v, double* sh) {
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
  for (int w = 0; w < kBNW; ++w) {
    if (w == wave) off = tot;
    tot += sh[w];
  }
  __syncthreads();
  return make_double2(off + ex, tot);
}

__device__ __forceinline__ int2 bminmax(int a, int b, int2* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a = min(a, __shfl_xor(a, o, 64));
    b = max(b, __shfl_xor(b, o, 64));
  }
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = make_int2(a, b);
  __syncthreads();
  int2 r = sh[0];
#pragma unroll
  for (int w = 1; w < kBNW; ++w) r = make_int2(min(r.x, sh[w].x), max(r.y, sh[w].y));
  __syncthreads();
  return r;
}

template <int FMT, int CB, int G, int CPL, int U, bool FULL>
__device__ __forceinline__ void run_member(const BPlan& P, int b, int r, BShared& S) {
  using St = Streamer<FMT, CB, G, CPL, U, FULL, kBNT>;
  constexpr int R = St::R;
  constexpr int BR = kBIT * R;  // rows per block
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const BInst I = P.inst[b];
  const int w = I.w;
  const int64_t N = I.N;
  const int d = I.d, K = I.K;
  const int64_t r0 = N * r / w, r1 = N * (r + 1) / w;
  const int64_t span = ((r1 - r0 + kBNW - 1) / kBNW + R - 1) / R * R;
  const int64_t wb = min(r1, r0 + wave * span), we = min(r1, wb + span);
  const int nbw = (int)((span + BR - 1) / BR);
  const int nb = kBNW * nbw;

  SeedParams sp;
  sp.xs = I.xs;
  sp.xexp = I.xexp;
  sp.X = I.X;
  sp.D = I.D;
  sp.N = N;
  sp.d = d;

  int64_t ci = uniform_index(draw_uniform(P.seed, 0u, (uint32_t)b), N);
  for (int m = 0; m < K; ++m) {
    const float* crow = I.X + ci * (int64_t)d;
    for (int j = tid; j < d; j += kBNT) {
      const float c = crow[j];
      S.cs[j] = c;
      if (r == 0) I.C[(int64_t)m * d + j] = c;
    }
    if (r == 0 && tid == 0) I.idx[m] = ci;
    __syncthreads();
    St st;
    st.init(S.cs, d);
    const bool first = m == 0;
    const gptr<float> D = as_global(I.D);
    for (int blk = 0; blk < nbw; ++blk) {
      double acc = 0.0;
#pragma unroll 1
      for (int it = 0; it < kBIT; ++it) {
        const int64_t base = wb + (int64_t)(blk * kBIT + it) * R;
        if (base < we)
          // BF16 / FP8 rows: the row of the centre gets D = 0 (its FP32 row,
          // not its stored one, is the centre)
          st.iter(sp, base, we, first, FMT != FMT_F32 ? ci : -1, [&](int64_t row, float dn, bool changed) {
            if (changed) D[row] = dn;
            acc += (double)dn;
          });
      }
      acc = wave_sum(acc);
      if (lane == 0) S.bs[wave * nbw + blk] = acc;
    }
    __syncthreads();
    if (m == K - 1) break;

    // block sums: per-thread contiguous runs, fixed-order scan
    const int per = (nb + kBNT - 1) / kBNT;  // <= 8
    const int q0 = min(nb, tid * per), q1 = min(nb, q0 + per);
    double part = 0.0;
    for (int q = q0; q < q1; ++q) part += S.bs[q];
    const double2 sc = bscan(part, S.sh);
    const double u = draw_uniform(P.seed, (uint32_t)(m + 1), (uint32_t)b);

    // gang exchange of member totals
    if (w > 1) {
      if (tid == 0) {
        const uint64_t bits = ((uint64_t)__double_as_longlong(sc.y) & ~0xFFFFull) | tag16(m);
        __hip_atomic_store(&P.mslots[I.slot0 + (m & 1) * w + r], bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (wave == 0) {
        double val = 0.0;
        if (lane < w) {
          const uint64_t bits = wait_for(&P.mslots[I.slot0 + (m & 1) * w + lane], 0xFFFFull, tag16(m), P);
          val = __longlong_as_double((long long)(bits & ~0xFFFFull));
        }
        // fixed-order wave scan of member totals
        double x = val;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const double y = __shfl_up(x, o, 64);
          if (lane >= o) x += y;
        }
        double ex = __shfl_up(x, 1, 64);
        if (lane == 0) ex = 0.0;
        const double T = __shfl(x, 63, 64);
        const double t = __dmul_rn(u, T);
        // owner: first member whose inclusive prefix exceeds t; else last positive
        const uint64_t hit = __ballot(lane < w && x > t);
        const uint64_t pos = __ballot(lane < w && val > 0.0);
        int owner = hit ? __builtin_ctzll(hit) : (pos ? 63 - __builtin_clzll(pos) : w - 1);
        const double Eo = __shfl(ex, owner, 64);
        if (lane == 0) {
          S.s_T = T;
          S.s_E = hit ? Eo : -1.0;  // -1: rounding put t past the total
          S.s_owner = owner;
        }
      }
      __syncthreads();
    } else if (tid == 0) {
      S.s_T = sc.y;
      S.s_E = 0.0;
      S.s_owner = 0;
    }
    __syncthreads();
    const double T = S.s_T;
    int64_t next;
    if (!isfinite(T)) {
      if (tid == 0) raise_status(P.ctl, KMPP_E_NONFINITE);
      next = 0;
    } else if (T == 0.0) {
      if (tid == 0) raise_status(P.ctl, KMPP_W_DEGENERATE);
      next = uniform_index(u, N);
    } else if (S.s_owner == r) {
      const double t = __dmul_rn(u, T);
      const bool inside = S.s_E >= 0.0 && (w > 1 || t < T);
      // block holding t: walk this thread's blocks from its prefix
      const double Er = inside ? S.s_E : 0.0;
      const int NONE = INT_MAX;
      int cand = NONE, lastpos = -1;
      double run = Er + sc.x, lo = 0.0;
      for (int q = q0; q < q1; ++q) {
        const double nr = run + S.bs[q];
        if (cand == NONE && inside && nr > t) {
          cand = q;
          lo = run;
        }
        if (S.bs[q] > 0.0) lastpos = q;
        run = nr;
      }
      const int2 bm = bminmax(cand, lastpos, S.shm);
      if (cand != NONE && cand == bm.x) S.s_lo = lo;
      __syncthreads();
      const bool found_blk = bm.x != NONE;
      const int blk = found_blk ? bm.x : max(bm.y, 0);
      const int bw = blk / nbw, bi = blk % nbw;
      const int64_t bwb = min(r1, r0 + bw * span), bwe = min(r1, bwb + span);
      const int64_t rb0 = min(bwe, bwb + (int64_t)bi * BR), rb1 = min(bwe, rb0 + BR);
      // rows of the block in wave 0: contiguous runs per lane
      int64_t pick = -1;
      if (wave == 0) {
        const int n = (int)(rb1 - rb0);
        const int per2 = (n + 63) / 64;
        const int64_t a0 = rb0 + min(n, lane * per2), a1 = min(rb1, a0 + per2);
        double p2 = 0.0;
        int64_t lp = -1;
        for (int64_t q = a0; q < a1; ++q) {
          const float dq = D[q];
          p2 += (double)dq;
          if (dq > 0.0f) lp = q;
        }
        double x = p2;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const double y = __shfl_up(x, o, 64);
          if (lane >= o) x += y;
        }
        double ex = __shfl_up(x, 1, 64);
        if (lane == 0) ex = 0.0;
        int64_t f = INT64_MAX;
        if (found_blk) {
          double rr = S.s_lo + ex;
          for (int64_t q = a0; q < a1; ++q) {
            rr += (double)D[q];
            if (rr > t) {
              f = q;
              break;
            }
          }
        }
        f = wave_min(f);
        lp = wave_max(lp);
        pick = f != INT64_MAX ? f : (lp >= 0 ? lp : rb1 - 1);
        if (pick < r0 || pick >= r1) pick = r0;
        if (lane == 0) {
          S.s_next = pick;
          if (w > 1)
            __hip_atomic_store(&P.iflag[b], ((uint64_t)(m + 1) << 32) | (uint64_t)pick, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      __syncthreads();
      next = S.s_next;
    } else {
      if (tid == 0) {
        const uint64_t v = wait_for(&P.iflag[b], 0xFFFFFFFF00000000ull, (uint64_t)(m + 1) << 32, P);
        S.s_next = (int64_t)(v & 0xFFFFFFFFull);
      }
      __syncthreads();
      next = S.s_next;
    }
    ci = next < N ? next : N - 1;
    __syncthreads();
  }
  __syncthreads();
}

// The streamer of each (format, width): 16-byte chunks where the width
// divides into them (G lanes per row), else one element per chunk.  Keep
// rows_per_block() in step with these choices.  One kernel per row format
// (each keeps only its own streamers' registers).
template <int FMT>
__device__ __forceinline__ void run_item(const BPlan& P, int b, int r, BShared& S) {
  const int d = P.inst[b].d;
  if constexpr (FMT == FMT_BF16) {
    switch (d) {
      case 8: run_member<FMT_BF16, 16, 1, 1, 8, true>(P, b, r, S); return;
      case 16: run_member<FMT_BF16, 16, 2, 1, 8, true>(P, b, r, S); return;
      case 32: run_member<FMT_BF16, 16, 4, 1, 8, true>(P, b, r, S); return;
      case 64: run_member<FMT_BF16, 16, 8, 1, 8, true>(P, b, r, S); return;
      case 128: run_member<FMT_BF16, 16, 16, 1, 8, true>(P, b, r, S); return;
      default:
        if (d <= 8)
          run_member<FMT_BF16, 2, 8, 1, 8, false>(P, b, r, S);
        else if (d <= 64)
          run_member<FMT_BF16, 2, 64, 1, 8, false>(P, b, r, S);
        else
          run_member<FMT_BF16, 2, 64, 4, 4, false>(P, b, r, S);
    }
  } else if constexpr (FMT == FMT_FP8) {
    switch (d) {
      case 8: run_member<FMT_FP8, 8, 1, 1, 8, true>(P, b, r, S); return;
      case 16: run_member<FMT_FP8, 16, 1, 1, 8, true>(P, b, r, S); return;
      case 32: run_member<FMT_FP8, 16, 2, 1, 8, true>(P, b, r, S); return;
      case 64: run_member<FMT_FP8, 16, 4, 1, 8, true>(P, b, r, S); return;
      case 128: run_member<FMT_FP8, 16, 8, 1, 8, true>(P, b, r, S); return;
      default:
        if (d <= 8)
          run_member<FMT_FP8, 1, 8, 1, 8, false>(P, b, r, S);
        else if (d <= 64)
          run_member<FMT_FP8, 1, 64, 1, 8, false>(P, b, r, S);
        else
          run_member<FMT_FP8, 1, 64, 4, 4, false>(P, b, r, S);
    }
  } else {
    switch (d) {
      case 2: run_member<FMT_F32, 8, 1, 1, 8, true>(P, b, r, S); return;
      case 4: run_member<FMT_F32, 16, 1, 1, 8, true>(P, b, r, S); return;
      case 8: run_member<FMT_F32, 16, 2, 1, 8, true>(P, b, r, S); return;
      case 16: run_member<FMT_F32, 16, 4, 1, 8, true>(P, b, r, S); return;
      case 32: run_member<FMT_F32, 16, 8, 1, 8, true>(P, b, r, S); return;
      case 64: run_member<FMT_F32, 16, 16, 1, 8, true>(P, b, r, S); return;
      case 128: run_member<FMT_F32, 16, 32, 1, 8, true>(P, b, r, S); return;
      default:
        if (d <= 8)
          run_member<FMT_F32, 4, 8, 1, 8, false>(P, b, r, S);
        else if (d <= 64)
          run_member<FMT_F32, 4, 64, 1, 8, false>(P, b, r, S);
        else
          run_member<FMT_F32, 4, 64, 4, 4, false>(P, b, r, S);
    }
  }
}

template <int FMT>
__global__ __launch_bounds__(kBNT) void batched_kernel(BPlan P) {
  __shared__ BShared S;
  const int e = P.begin[blockIdx.x + 1];
  for (int it = P.begin[blockIdx.x]; it < e; ++it) {
    const BItem item = P.items[it];
    run_item<FMT>(P, item.b, item.r, S);
    __syncthreads();
  }
}

const void* batched_fn(int fmt) {
  return fmt == FMT_BF16 ? reinterpret_cast<const void*>(&batched_kernel<FMT_BF16>)
         : fmt == FMT_FP8 ? reinterpret_cast<const void*>(&batched_kernel<FMT_FP8>)
                          : reinterpret_cast<const void*>(&batched_kernel<FMT_F32>);
}

__global__ void batched_reset_kernel(BPlan P) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (tid == 0) P.ctl->status = KMPP_OK;
  for (int64_t i = tid; i < P.n_mslots; i += stride) P.mslots[i] = 0;
  for (int64_t i = tid; i < P.n_inst; i += stride) P.iflag[i] = 0;
}

// ---------------------------------------------------------------- host
namespace {
inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

struct PlanHost {
  BPlan plan;
  int W;
  bool cooperative;
};
std::mutex g_mu;
std::map<const void*, PlanHost> g_plans;

struct Tune {
  int wg_per_cu = 2;
  double chip_gbs = 5000.0;  // streaming rate of the whole chip, GB/s
  double sync1_us = 2.5;     // per seed step, gang of one
  double syncw_us = 6.0;     // per seed step, larger gangs
  double alpha = 1.0;        // cap of one instance's time, as a multiple of the mean load
  double wait_ms = -1.0;     // gang wait budget: < 0 automatic (from the plan), 0 give up at once
};
Tune g_tune;

struct Layout {
  size_t inst, items, begin, mslots, iflag, D, idx, total;
  int n_items, n_mslots, W;
  std::vector<int> gang;
};

int rows_per_block(int fmt, int d) {
  // R * kBIT for the streamer chosen in run_item: G lanes per row, U loads
  // per lane
  int G = 0, U = 8;
  const int eb = fmt == FMT_F32 ? 4 : fmt == FMT_BF16 ? 2 : 1;
  // exact widths: bytes per chunk (8 for FP32 d = 2 and FP8 d = 8)
  const int cb = (fmt == FMT_F32 && d == 2) || (fmt == FMT_FP8 && d == 8) ? 8 : 16;
  const bool exact = fmt == FMT_F32 ? (d == 2 || d == 4 || d == 8 || d == 16 || d == 32 || d == 64 || d == 128)
                                    : fmt == FMT_BF16 ? (d == 8 || d == 16 || d == 32 || d == 64 || d == 128)
                                                      : (d == 8 || d == 16 || d == 32 || d == 64 || d == 128);
  if (exact) {
    G = d * eb / cb;
  } else {
    G = d <= 8 ? 8 : 64;
    if (d > 64) U = 4;
  }
  return U * (64 / G) * kBIT;
}

int num_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
  return n;
}

int inst_fmt(const kmpp_instance& I) { return I.dtype == KMPP_BF16 ? FMT_BF16 : I.dtype == KMPP_FP8_E4M3 ? FMT_FP8 : FMT_F32; }

double inst_time_us(const kmpp_instance& I, int w, const Tune& T, int W) {
  // bytes streamed per seed step: the rows in their format (FP8: plus the
  // exponent byte)
  const double eb = I.dtype == KMPP_BF16 ? 2.0 : I.dtype == KMPP_FP8_E4M3 ? 1.0 + 1.0 / I.d : 4.0;
  const double bytes = (double)I.N * I.d * eb * I.K;
  const double per_wg = T.chip_gbs * 1e3 / W;  // bytes per us per workgroup when all stream
  return bytes / w / per_wg + I.K * (w > 1 ? T.syncw_us : T.sync1_us);
}

Layout plan_layout(const kmpp_instance* inst, int n, int W, const Tune& T) {
  Layout L;
  L.W = W;
  L.gang.resize(n);
  double total = 0.0;
  for (int b = 0; b < n; ++b) total += inst_time_us(inst[b], 1, T, W);
  const double cap = std::max(1.0, T.alpha * total / W);
  L.n_items = 0;
  L.n_mslots = 0;
  for (int b = 0; b < n; ++b) {
    const int rpb = rows_per_block(inst_fmt(inst[b]), inst[b].d);
    const int64_t blocks1 = (inst[b].N + rpb - 1) / rpb;
    int w = 1;
    // smallest gang within the time cap, enough LDS for the block sums, and
    // at least one block of rows per member
    while (w < kBMaxGang && w * 2 <= inst[b].N &&
           (inst_time_us(inst[b], w, T, W) > cap || blocks1 / w + kBNW > kBMaxBlocks))
      w *= 2;
    L.gang[b] = w;
    L.n_items += w;
    L.n_mslots += 2 * w;
  }
  size_t off = sizeof(Ctl);
  L.inst = off;
  off += a256(sizeof(BInst) * n);
  L.items = off;
  off += a256(sizeof(BItem) * L.n_items);
  L.begin = off;
  off += a256(sizeof(int32_t) * (W + 1));
  L.mslots = off;
  off += a256(sizeof(uint64_t) * L.n_mslots);
  L.iflag = off;
  off += a256(sizeof(uint64_t) * n);
  int64_t nD = 0, nI = 0;
  for (int b = 0; b < n; ++b) {
    if (!inst[b].out_D) nD += inst[b].N;
    if (!inst[b].out_idx) nI += inst[b].K;
  }
  L.D = off;
  off += a256(sizeof(float) * nD);
  L.idx = off;
  off += a256(sizeof(int64_t) * nI);
  L.total = off;
  return L;
}

int workgroups(int fmt) {
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, batched_fn(fmt), kBNT, 0) != hipSuccess || occ <= 0)
    occ = 1;
  return num_cus() * std::min(occ, g_tune.wg_per_cu);
}

// Every instance of a batch streams rows of one format (the first one's).
bool one_format(const kmpp_instance* inst, int n) {
  for (int b = 1; b < n; ++b)
    if (inst[b].dtype != inst[0].dtype) return false;
  return true;
}

// The budget of one gang wait, in ticks of the device's constant-rate
// real-time counter: a wait can last as long as the peers' earlier list
// items, at most the plan's estimated length, so eight times that with a
// floor of one second (the cost model is an estimate); the tuning table's
// wait_ms overrides it (0: every wait gives up at once).
uint64_t wait_budget_ticks(const Tune& T, double makespan_us) {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    khz = 100000;  // the 100 MHz counter of the Instinct family
  const double ms = T.wait_ms >= 0.0 ? T.wait_ms : std::max(1000.0, 8.0 * makespan_us * 1e-3);
  return (uint64_t)(ms * (double)khz);
}
}  // namespace

int batched_tune_set(const char* key, double v) {
  if (!strcmp(key, "wg_per_cu")) g_tune.wg_per_cu = std::max(1, (int)v);
  else if (!strcmp(key, "chip_gbs")) g_tune.chip_gbs = v;
  else if (!strcmp(key, "sync1_us")) g_tune.sync1_us = v;
  else if (!strcmp(key, "syncw_us")) g_tune.syncw_us = v;
  else if (!strcmp(key, "alpha")) g_tune.alpha = v;
  else if (!strcmp(key, "wait_ms")) g_tune.wait_ms = v;
  else return KMPP_E_INVALID;
  return KMPP_OK;
}

// An instance fits when its rows, split over the largest gang, leave every
// member's block sums within LDS.
bool batched_fits(const kmpp_instance& I) {
  if (I.N < 1 || I.K < 1 || I.K > I.N || I.d < 1 || I.d > kBMaxD || I.N > INT32_MAX) return false;
  if (I.dtype != KMPP_F32 && I.dtype != KMPP_BF16 && I.dtype != KMPP_FP8_E4M3) return false;
  const int rpb = rows_per_block(inst_fmt(I), I.d);
  const int64_t blocks = (I.N + rpb - 1) / rpb;
  return blocks / kBMaxGang + kBNW <= kBMaxBlocks;
}

size_t batched_workspace(const kmpp_instance* inst, int n) {
  for (int b = 0; b < n; ++b)
    if (!batched_fits(inst[b])) return 0;
  if (!one_format(inst, n)) return 0;
  return plan_layout(inst, n, workgroups(inst_fmt(inst[0])), g_tune).total;
}

int batched_prepare(const kmpp_instance* inst, int n, uint64_t seed, void* ws, size_t ws_bytes, hipStream_t stream) {
  for (int b = 0; b < n; ++b) {
    const kmpp_instance& I = inst[b];
    if (!I.X || !I.out_centers || I.N < 1 || I.K < 1 || I.K > I.N || I.N > INT32_MAX || I.d < 1 ||
        (reinterpret_cast<uintptr_t>(I.X) & 15))
      return KMPP_E_INVALID;
    if (I.dtype != KMPP_F32 && I.dtype != KMPP_BF16 && I.dtype != KMPP_FP8_E4M3) return KMPP_E_INVALID;
    if (I.dtype != KMPP_F32 && (!I.Xq || (reinterpret_cast<uintptr_t>(I.Xq) & 15))) return KMPP_E_INVALID;
    if (I.dtype == KMPP_FP8_E4M3 && !I.Xq_exp) return KMPP_E_INVALID;
    if (!batched_fits(I)) return KMPP_E_UNSUPPORTED;
  }
  if (!one_format(inst, n)) return KMPP_E_UNSUPPORTED;
  const int fmt = inst_fmt(inst[0]);
  const int W = workgroups(fmt);
  const Tune T = g_tune;
  const Layout L = plan_layout(inst, n, W, T);
  if (ws_bytes < L.total) return KMPP_E_WORKSPACE;
  char* w = static_cast<char*>(ws);

  // longest-first list scheduling of gangs onto W workgroup slots
  std::vector<int> order(n);
  for (int b = 0; b < n; ++b) order[b] = b;
  std::vector<double> tb(n);
  for (int b = 0; b < n; ++b) tb[b] = inst_time_us(inst[b], L.gang[b], T, W);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return tb[a] > tb[b]; });
  std::vector<double> avail(W, 0.0);
  std::vector<std::vector<BItem>> lists(W);
  using Slot = std::pair<double, int>;
  std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> heap;
  for (int s = 0; s < W; ++s) heap.push({0.0, s});
  std::vector<BInst> hinst(n);
  int slot0 = 0;
  int64_t offD = 0, offI = 0;
  for (int b = 0; b < n; ++b) {
    const kmpp_instance& I = inst[b];
    BInst& H = hinst[b];
    H.X = I.X;
    H.xs = I.dtype == KMPP_F32 ? static_cast<const void*>(I.X) : I.Xq;
    H.xexp = I.dtype == KMPP_FP8_E4M3 ? I.Xq_exp : nullptr;
    H.C = I.out_centers;
    H.D = I.out_D ? I.out_D : reinterpret_cast<float*>(w + L.D) + offD;
    if (!I.out_D) offD += I.N;
    H.idx = I.out_idx ? I.out_idx : reinterpret_cast<int64_t*>(w + L.idx) + offI;
    if (!I.out_idx) offI += I.K;
    H.N = I.N;
    H.d = I.d;
    H.K = I.K;
    H.w = L.gang[b];
    H.slot0 = slot0;
    slot0 += 2 * L.gang[b];
  }
  double makespan_us = 0.0;
  for (int b : order) {
    const int g = L.gang[b];
    std::vector<Slot> got;
    double start = 0.0;
    for (int k = 0; k < g; ++k) {
      got.push_back(heap.top());
      heap.pop();
      start = std::max(start, got.back().first);
    }
    for (int k = 0; k < g; ++k) {
      lists[got[k].second].push_back(BItem{b, (int16_t)k, (int16_t)g});
      heap.push({start + tb[b], got[k].second});
    }
    makespan_us = std::max(makespan_us, start + tb[b]);
  }
  std::vector<BItem> items;
  std::vector<int32_t> begin(W + 1, 0);
  for (int s = 0; s < W; ++s) {
    begin[s] = (int32_t)items.size();
    items.insert(items.end(), lists[s].begin(), lists[s].end());
  }
  begin[W] = (int32_t)items.size();
  std::vector<char> host(L.mslots - sizeof(Ctl), 0);
  memcpy(host.data() + (L.inst - sizeof(Ctl)), hinst.data(), sizeof(BInst) * n);
  memcpy(host.data() + (L.items - sizeof(Ctl)), items.data(), sizeof(BItem) * items.size());
  memcpy(host.data() + (L.begin - sizeof(Ctl)), begin.data(), sizeof(int32_t) * begin.size());
  if (hipMemcpyAsync(w + sizeof(Ctl), host.data(), host.size(), hipMemcpyHostToDevice, stream) != hipSuccess)
    return KMPP_E_HIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return KMPP_E_HIP;

  PlanHost ph;
  ph.W = W;
  ph.plan.inst = reinterpret_cast<const BInst*>(w + L.inst);
  ph.plan.items = reinterpret_cast<const BItem*>(w + L.items);
  ph.plan.begin = reinterpret_cast<const int32_t*>(w + L.begin);
  ph.plan.mslots = reinterpret_cast<uint64_t*>(w + L.mslots);
  ph.plan.iflag = reinterpret_cast<uint64_t*>(w + L.iflag);
  ph.plan.ctl = reinterpret_cast<Ctl*>(w);
  ph.plan.seed = seed;
  ph.plan.wait_ticks = wait_budget_ticks(T, makespan_us);
  ph.plan.n_inst = n;
  ph.plan.W = W;
  ph.plan.n_mslots = L.n_mslots;
  ph.plan.fmt = fmt;
  ph.cooperative = true;
  std::lock_guard<std::mutex> lk(g_mu);
  g_plans[ws] = ph;
  return KMPP_OK;
}

int batched_launch(void* ws, hipStream_t stream) {
  PlanHost ph;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_plans.find(ws);
    if (it == g_plans.end()) return KMPP_E_INVALID;
    ph = it->second;
  }
  hipLaunchKernelGGL(batched_reset_kernel, dim3(64), dim3(256), 0, stream, ph.plan);
  if (hipGetLastError() != hipSuccess) return KMPP_E_HIP;
  void* args[] = {&ph.plan};
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return KMPP_E_HIP;
  hipError_t e;
  if (cs == hipStreamCaptureStatusNone)
    e = hipLaunchCooperativeKernel(batched_fn(ph.plan.fmt), dim3(ph.W), dim3(kBNT), args, 0, stream);
  else  // under capture: a plain launch of the same occupancy-sized grid
    e = hipLaunchKernel(batched_fn(ph.plan.fmt), dim3(ph.W), dim3(kBNT), args, 0, stream);
  return e == hipSuccess ? KMPP_OK : KMPP_E_HIP;
}

}  // namespace kmpp
