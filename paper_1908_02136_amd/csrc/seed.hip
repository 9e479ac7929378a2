// seed.hip -- the k-means++ seed loop (paper, Section II, Algorithms 1-2).
//
// The pass kernel m (1..K) streams the point rows once, updates every
// point's nearest squared distance
// D = min(D, ||x - c_{m-1}||^2) and reduces D per workgroup tile into an FP64
// tile sum.  For m < K seed m is then taken by inverting the FP64
// cumulative distribution of D (tile sums, then the owning tile's rows) at
// t = u_m * sum(D), either by every workgroup of pass m+1 at its start (one
// launch per seed; pass m+1 then writes D and its tile sums to the other of
// two buffers, so pass m's stay intact while any workgroup still draws), by
// workgroup 0 of pass m+1 alone, which publishes the index to the others
// (one launch per seed, D in place: nobody writes D or a tile sum before the
// index is out), or by a one-workgroup draw kernel between the passes (two
// launches per seed; weighted seeding, or where the tuning table says so).
// Pass m+1 reads that original FP32 row, broadcasts it from LDS and stores
// it in out_centers[m].  Nothing returns to the host between seeds.
//
// Row streaming: a row of d elements is split into 16-byte chunks; a group
// of G lanes covers one row (G*CPL chunks), so one wave-wide load reads 64/G
// whole consecutive rows (1 KiB contiguous).  Each lane keeps the centre
// slice of its chunks in registers and the row distance is reduced across
// the G lanes with xor shuffles.  U loads per lane are issued before any is
// consumed.  D is read once per row per pass, 64 rows per coalesced
// access, and written back only where it changed (every row, to the other
// buffer, when the next pass draws at its start).
#include <type_traits>

#include "kmpp_dev.h"
#include "kmpp_impl.h"
#include "stream.h"

namespace kmpp {

// ---------------------------------------------------------------- S1
// First seed: i0 = min(floor(u_0 N), N-1); resets the status word.
__global__ __launch_bounds__(256) void seed_init_kernel(SeedParams p) {
  __shared__ int64_t s_i0;
  if (threadIdx.x == 0) {
    p.ctl->status = KMPP_OK;
    p.ctl->arrive = 0u;
    p.ctl->lead = 0ull;
    if (p.sumD) p.sumD[0] = 0.0;
    const double u0 = draw_uniform(p.seed, 0u, p.inst);
    const int64_t i0 = uniform_index(u0, p.N);
    p.idx[0] = i0;
    s_i0 = i0;
  }
  __syncthreads();
  const float* src = p.X + s_i0 * (int64_t)p.d;
  for (int j = threadIdx.x; j < p.d; j += blockDim.x) p.centers[j] = src[j];
}

// Weighted seeding, before the first draw: D := 1 for every row and the
// tile sums := FP64 sums of the weights, so the draw kernel (pass 0) picks
// the first centre with probability proportional to w.
__global__ __launch_bounds__(256) void seed_wfirst_kernel(SeedParams p) {
  __shared__ double red[4];
  const int64_t t0 = (int64_t)blockIdx.x * p.rows_per_tile;
  const int64_t t1 = min(p.N, t0 + (int64_t)p.rows_per_tile);
  double acc = 0.0;
  for (int64_t i = t0 + threadIdx.x; i < t1; i += 256) {
    p.D[i] = 1.0f;
    acc += (double)p.wts[i];
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) p.tsum[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// ---------------------------------------------------------------- S3-S5
// Draw seed p.pass from the pass just finished, in one workgroup (the
// kernel boundary makes every D and tile sum of the pass visible):
//  1. each thread loads a contiguous block of at most kDrawPer FP64 tile
//     sums (all loads in flight together); the blocks are exclusive-scanned
//     in a fixed order; t = u * total;
//  2. each thread walks its block in registers from its prefix; the first
//     tile whose inclusive prefix exceeds t owns the draw;
//  3. the owner tile's D values (at most kDrawRows per thread) are loaded,
//     scanned the same way from the tile's prefix, and the first row whose
//     inclusive prefix exceeds t is the seed;
//  4. the index is written; the next pass copies the row into out_centers
//     (every draw is followed by a pass).
// If rounding leaves no prefix above t, the last row with D > 0 is taken.
constexpr int kDrawNT = 256;
constexpr int kDrawPer = 32;   // tile sums per thread: kMaxTiles <= kDrawNT * kDrawPer
constexpr int kDrawRows = 16;  // D values per thread kept in registers

// Exclusive scan of one double per thread over NT threads with a single
// barrier; fixed association order.  Returns (exclusive, total).
template <int NT>
__device__ __forceinline__ double2 draw_scan(double v, double* sh) {
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
  double off = 0.0, tot = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    if (w == wave) off = tot;
    tot += sh[w];
  }
  __syncthreads();
  return make_double2(off + ex, tot);
}

// (min a, max b) over the workgroup with one barrier.
template <int NT>
__device__ __forceinline__ int2 draw_minmax(int a, int b, int2* sh) {
  constexpr int NW = NT / 64;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a = min(a, __shfl_xor(a, o, 64));
    b = max(b, __shfl_xor(b, o, 64));
  }
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = make_int2(a, b);
  __syncthreads();
  int2 r = sh[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) r = make_int2(min(r.x, sh[w].x), max(r.y, sh[w].y));
  __syncthreads();
  return r;
}

template <bool WEIGHTED>
__global__ __launch_bounds__(kDrawNT) void seed_draw_kernel(SeedParams p) {
  constexpr int NT = kDrawNT;
  constexpr int NW = NT / 64;
  __shared__ double sh[NW];
  __shared__ int2 shm[NW];
  __shared__ float shf[NW];
  __shared__ double s_lo;
  const int tid = threadIdx.x;
  const int G = p.ntiles;
  const int NONE = INT_MAX;

  const int per = (G + NT - 1) / NT;  // <= kDrawPer
  const int b0 = min(G, tid * per);
  const int nb = max(0, min(per, G - b0));
  double v[kDrawPer];
#pragma unroll
  for (int k = 0; k < kDrawPer; ++k) v[k] = k < nb ? p.tsum[b0 + k] : 0.0;
  double part = 0.0;
  int lastpos = -1;
#pragma unroll
  for (int k = 0; k < kDrawPer; ++k) {
    part += v[k];
    if (v[k] > 0.0) lastpos = b0 + k;
  }
  const double2 sc = draw_scan<NT>(part, sh);
  const double T = sc.y;
  const double u = draw_uniform(p.seed, (uint32_t)p.pass, p.inst, p.tag);
  if (tid == 0 && p.sumD) p.sumD[p.pass] = T;

  int64_t seed_row;
  if (!isfinite(T)) {
    if (tid == 0) raise_status(p.ctl, KMPP_E_NONFINITE);
    seed_row = 0;
  } else if (T == 0.0) {
    if (tid == 0) raise_status(p.ctl, KMPP_W_DEGENERATE);
    seed_row = uniform_index(u, p.N);
  } else {
    const double t = __dmul_rn(u, T);
    int cand = NONE;
    double run = sc.x, lo = 0.0;
#pragma unroll
    for (int k = 0; k < kDrawPer; ++k) {
      const double nr = run + v[k];
      if (cand == NONE && k < nb && nr > t) {
        cand = b0 + k;
        lo = run;
      }
      run = nr;
    }
    const int2 tm = draw_minmax<NT>(cand, lastpos, shm);
    if (cand != NONE && cand == tm.x) s_lo = lo;
    const bool inside = tm.x != NONE;  // else rounding put t at or past the total
    int tile = inside ? tm.x : tm.y;
    if (tile < 0 || tile >= G) tile = G - 1;
    __syncthreads();
    const double tlo = inside ? s_lo : 0.0;
    const int64_t r0 = (int64_t)tile * p.rows_per_tile;
    const int64_t r1 = min(p.N, r0 + (int64_t)p.rows_per_tile);
    const int n = (int)(r1 - r0);
    const int per2 = (n + NT - 1) / NT;
    const int64_t q0 = r0 + min(n, tid * per2);
    const int nq = max(0, min(per2, (int)(r1 - q0)));
    int found = NONE, lastrow = -1;
    // a row's share: D, or w * D (FP64) for weighted seeding
    using Share = typename std::conditional<WEIGHTED, double, float>::type;
    auto share = [&](int64_t i, float dk) -> Share {
      if constexpr (WEIGHTED)
        return (double)dk * (double)p.wts[i];
      else
        return dk;
    };
    if (per2 <= kDrawRows) {
      Share dv[kDrawRows];
#pragma unroll
      for (int k = 0; k < kDrawRows; ++k) dv[k] = k < nq ? share(q0 + k, p.D[q0 + k]) : Share(0);
      double part2 = 0.0;
#pragma unroll
      for (int k = 0; k < kDrawRows; ++k) {
        part2 += (double)dv[k];
        if (dv[k] > Share(0)) lastrow = (int)(q0 - r0) + k;
      }
      const double2 sc2 = draw_scan<NT>(part2, sh);
      if (inside) {
        double r = tlo + sc2.x;
#pragma unroll
        for (int k = 0; k < kDrawRows; ++k) {
          r += (double)dv[k];
          if (found == NONE && k < nq && r > t) found = (int)(q0 - r0) + k;
        }
      }
    } else {  // very large tiles: same steps, values reloaded
      double part2 = 0.0;
      for (int k = 0; k < nq; ++k) {
        const double dk = (double)share(q0 + k, p.D[q0 + k]);
        part2 += dk;
        if (dk > 0.0) lastrow = (int)(q0 - r0) + k;
      }
      const double2 sc2 = draw_scan<NT>(part2, sh);
      if (inside) {
        double r = tlo + sc2.x;
        for (int k = 0; k < nq && found == NONE; ++k) {
          r += (double)share(q0 + k, p.D[q0 + k]);
          if (r > t) found = (int)(q0 - r0) + k;
        }
      }
    }
    const int2 fm = draw_minmax<NT>(found, lastrow, shm);
    seed_row = r0 + (fm.x != NONE ? fm.x : (fm.y >= 0 ? fm.y : n - 1));
  }

  // precision forms: the drawn row's D from the quantised rows, and its FP32
  // nearest distance recomputed from the original row against earlier seeds
  if (p.recheck != nullptr) {
    const float* xr = p.X + seed_row * (int64_t)p.d;
    float best = INFINITY;
    for (int j = tid; j < p.pass; j += NT) {
      const float* c = p.centers + (int64_t)j * p.d;
      float a = 0.0f;
      for (int k = 0; k < p.d; ++k) {
        const float df = xr[k] - c[k];
        a = fmaf(df, df, a);
      }
      best = fminf(best, a);
    }
    best = block_minf<NT>(best, shf);
    if (tid == 0) {
      p.recheck[2 * (int64_t)p.pass] = p.D[seed_row];
      p.recheck[2 * (int64_t)p.pass + 1] = best;
    }
  }
  if (tid == 0) p.idx[p.pass] = seed_row;
}

// The draw of seed step = pass - 1 at the start of every workgroup of the
// pass (the kernel boundary makes the previous pass's D and tile sums
// visible; this pass writes to the other buffers).  The same fixed-order
// steps as draw_seed on the same values, so every workgroup finds the same
// row, and for one NT the draw kernel finds it too; the tile sums and then
// the owner tile's D are staged in LDS (lds: max(8 ntiles, 4 rows_per_tile)
// bytes).  Workgroup 0 records the index (and the precision recheck) and
// raises the status.  Returns the row; lds is free again on return.
// Copy n values to LDS with up to 8 loads per thread in flight before the
// first store (one memory round trip per 8 * NT values).
template <int NT, typename T, typename L>
__device__ __forceinline__ void stage_to_lds(const T* __restrict__ src, L* dst, int n) {
  constexpr int kB = 8;
  for (int b = 0; b < n; b += kB * NT) {
    T v[kB];
#pragma unroll
    for (int k = 0; k < kB; ++k) {
      const int i = b + k * NT + (int)threadIdx.x;
      v[k] = i < n ? src[i] : T(0);
    }
#pragma unroll
    for (int k = 0; k < kB; ++k) {
      const int i = b + k * NT + (int)threadIdx.x;
      if (i < n) dst[i] = v[k];
    }
  }
}

template <int NT, bool STAGE = true>
__device__ int64_t draw_at_start(const SeedParams& p, float* lds) {
  constexpr int NW = NT / 64;
  __shared__ double sh[NW];
  __shared__ int2 shm[NW];
  __shared__ float shf[NW];
  __shared__ double s_lo;
  const double* ts = reinterpret_cast<const double*>(lds);
  const int tid = threadIdx.x;
  const int G = p.ntiles;
  const int NONE = INT_MAX;
  const int step = p.pass - 1;
  const bool lead = blockIdx.x == 0;

  if constexpr (STAGE) {
    stage_to_lds<NT>(p.tsum, reinterpret_cast<double*>(lds), G);
    __syncthreads();
  } else {
    ts = p.tsum;  // read in place (nothing writes them before the draw ends)
  }
  // the tiles: contiguous blocks per thread, fixed-order FP64 scan
  const int per = (G + NT - 1) / NT;
  const int b0 = min(G, tid * per);
  const int nb = max(0, min(per, G - b0));
  double part = 0.0;
  int lastpos = -1;
  for (int k = 0; k < nb; ++k) {
    const double v = ts[b0 + k];
    part += v;
    if (v > 0.0) lastpos = b0 + k;
  }
  const double2 sc = draw_scan<NT>(part, sh);
  const double T = sc.y;
  const double u = draw_uniform(p.seed, (uint32_t)step, p.inst, p.tag);
  if (lead && tid == 0 && p.sumD) p.sumD[step] = T;

  int64_t seed_row;
  if (!isfinite(T)) {
    if (lead && tid == 0) raise_status(p.ctl, KMPP_E_NONFINITE);
    seed_row = 0;
  } else if (T == 0.0) {
    if (lead && tid == 0) raise_status(p.ctl, KMPP_W_DEGENERATE);
    seed_row = uniform_index(u, p.N);
  } else {
    const double t = __dmul_rn(u, T);
    int cand = NONE;
    double run = sc.x, lo = 0.0;
    for (int k = 0; k < nb; ++k) {
      const double nr = run + ts[b0 + k];
      if (cand == NONE && nr > t) {
        cand = b0 + k;
        lo = run;
      }
      run = nr;
    }
    const int2 tm = draw_minmax<NT>(cand, lastpos, shm);  // ends with a barrier: ts is free
    if (cand != NONE && cand == tm.x) s_lo = lo;
    const bool inside = tm.x != NONE;
    int tile = inside ? tm.x : tm.y;
    if (tile < 0 || tile >= G) tile = G - 1;
    // the owner tile's D, staged in LDS, same blocks as draw_seed
    const int64_t r0 = (int64_t)tile * p.rows_per_tile;
    const int64_t r1 = min(p.N, r0 + (int64_t)p.rows_per_tile);
    const int n = (int)(r1 - r0);
    const float* dv = STAGE ? lds : p.D + r0;
    if constexpr (STAGE) stage_to_lds<NT>(p.D + r0, lds, n);
    __syncthreads();  // s_lo (and the staged D) are visible to every thread
    const double tlo = inside ? s_lo : 0.0;
    const int per2 = (n + NT - 1) / NT;
    const int j0 = min(n, tid * per2);
    const int nq = max(0, min(per2, n - j0));
    int found = NONE, lastrow = -1;
    double part2 = 0.0;
    for (int k = 0; k < nq; ++k) {
      const float dk = dv[j0 + k];
      part2 += (double)dk;
      if (dk > 0.0f) lastrow = j0 + k;
    }
    const double2 sc2 = draw_scan<NT>(part2, sh);
    if (inside) {
      double r = tlo + sc2.x;
      for (int k = 0; k < nq && found == NONE; ++k) {
        r += (double)dv[j0 + k];
        if (r > t) found = j0 + k;
      }
    }
    const int2 fm = draw_minmax<NT>(found, lastrow, shm);  // ends with a barrier: lds is free
    seed_row = r0 + (fm.x != NONE ? fm.x : (fm.y >= 0 ? fm.y : n - 1));
  }

  if (lead) {
    // precision forms: as in draw_seed
    if (p.recheck != nullptr) {
      const float* xr = p.X + seed_row * (int64_t)p.d;
      float best = INFINITY;
      for (int j = tid; j < step; j += NT) {
        const float* c = p.centers + (int64_t)j * p.d;  // written by earlier passes
        float a = 0.0f;
        for (int k = 0; k < p.d; ++k) {
          const float df = xr[k] - c[k];
          a = fmaf(df, df, a);
        }
        best = fminf(best, a);
      }
      best = block_minf<NT>(best, shf);
      if (tid == 0) {
        p.recheck[2 * (int64_t)step] = p.D[seed_row];
        p.recheck[2 * (int64_t)step + 1] = best;
      }
    }
    if (tid == 0) p.idx[step] = seed_row;
  }
  __syncthreads();
  return seed_row;
}

// ---------------------------------------------------------------- S2
// One pass: the row path RL and the centre source CS are template
// parameters (the memory spaces Section II compares).
// DRAWER: every workgroup first draws seed m-1 (m >= 2) from pass m-1's D
// and tile sums; this pass writes every row's D to Dw and its tile sums to
// tsum_w (the other buffers).  Else D is updated in place where it changed.
template <int FMT, int CB, int G, int CPL, int U, bool FULL, int NT, int RL, int CS, int DRAW>
__global__ __launch_bounds__(NT) void seed_pass_kernel(SeedParams p) {
  constexpr bool DRAWER = DRAW == 1;
  constexpr bool LEAD = DRAW == 2;
  using S = Streamer<FMT, CB, G, CPL, U, FULL, NT, RL>;
  constexpr int NW = NT / 64;
  extern __shared__ __align__(16) float cs[];  // centre row, d floats (CEN_LDS); the draw's staging (DRAWER)
  __shared__ double red[NW];

  const int tid = threadIdx.x;
  const int d = p.d;
  const bool first = p.pass == 1;
  const int64_t t0 = (int64_t)blockIdx.x * p.rows_per_tile;
  const int64_t t1 = min(p.N, t0 + (int64_t)p.rows_per_tile);

  S st;
  st.layout();
  st.set_rows(p.xs, t0, t1, d);
  // Narrow FP32 rows (at most 8 lanes per row), 512-thread workgroups,
  // without DRAWER: this wave's first rows (and their D) are requested before
  // the centre, so their latency overlaps the two dependent loads of the
  // centre (its index, then its row); measured -1 to -3 % per seed for d = 2
  // and 32.  Wider rows lose occupancy to the batch held meanwhile (+3 % at
  // d = 128), with DRAWER the draw's registers come on top, and the 256-thread
  // variants (those of the memory-space comparison) keep one code shape.
  constexpr bool kEarly = !DRAWER && FMT == FMT_F32 && G <= 8 && NT == 512;
  __shared__ int64_t s_cidx;
  const int64_t base0 = t0 + (int64_t)st.wave * S::R;
  typename S::Batch b0;
  const bool early = kEarly && base0 < t1;
  if (early) st.load(p, base0, t1, first, b0);
  // centre c_{pass-1}: the original FP32 row of the previous seed (drawn
  // here first with DRAWER)
  int64_t cidx;
  if constexpr (DRAWER) {
    cidx = p.pass >= 2 ? draw_at_start<NT>(p, cs) : p.idx[0];
  } else if constexpr (LEAD) {
    // workgroup 0 draws seed pass-1 from the previous pass's tile sums and
    // D, in place (no workgroup of this pass writes either before it has
    // the index), and publishes the index tagged with the pass; the others
    // wait for it (their first rows already in flight).  Workgroup 0 is
    // dispatched first and waits for nobody, so every wait ends; a wait
    // past its budget (p.lead_wait ticks of the real-time counter; 0: none)
    // raises KMPP_E_TIMEOUT and goes on with row 0.
    if (p.pass < 2) {
      cidx = p.idx[0];
    } else if (blockIdx.x == 0) {
      cidx = draw_at_start<NT, false>(p, cs);
      if (tid == 0)
        __hip_atomic_store(&p.ctl->lead, ((uint64_t)(uint32_t)p.pass << 32) | (uint64_t)cidx, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    } else {
      if (tid == 0) {
        const uint64_t want = (uint64_t)(uint32_t)p.pass;
        uint64_t v = p.lead_wait ? __hip_atomic_load(&p.ctl->lead, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        while ((v >> 32) != want) {
          if (p.lead_wait == 0 || __builtin_amdgcn_s_memrealtime() - t0 > p.lead_wait) {
            raise_status(p.ctl, KMPP_E_TIMEOUT);
            v = want << 32;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          v = __hip_atomic_load(&p.ctl->lead, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        s_cidx = (int64_t)(v & 0xFFFFFFFFull);
      }
      __syncthreads();
      cidx = s_cidx;
    }
  } else {
    cidx = p.idx[p.pass - 1];
  }
  // every draw has raised its status by now (the last one in this
  // workgroup's own thread 0 with DRAWER, else in an earlier launch)
  if (p.status_out && p.pass == p.K && blockIdx.x == 0 && tid == 0)
    *p.status_out = __hip_atomic_load(&p.ctl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const float* cg = p.X + cidx * (int64_t)d;
  const int64_t prev = (FMT != FMT_F32) ? cidx : -1;
  if constexpr (CS == CEN_SCALAR) {
    st.set_centre_uniform(cg);
  } else if constexpr (CS == CEN_GLOBAL) {
    // a zero the compiler cannot see as uniform keeps these vector loads
    // even where every lane reads the same address (one lane per row)
    int vzero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(vzero));
    st.set_centre(as_global(cg) + vzero, d);
  } else {
    for (int j = tid; j < d; j += NT) cs[j] = cg[j];
    __syncthreads();
    st.set_centre(cs, d);
  }
  // centre m-1 is stored by this pass (centre 0 by the init kernel, except
  // for weighted seeding, whose first centre comes from a draw)
  if (blockIdx.x == 0 && (p.pass > 1 || p.wts))
    for (int j = tid; j < d; j += NT) p.centers[(int64_t)(p.pass - 1) * d + j] = CS == CEN_LDS ? cs[j] : cg[j];

  double acc = 0.0;
  float* D = p.D;
  auto sink = [&](int64_t row, float dn, bool changed) {
    if constexpr (DRAWER)
      p.Dw[row] = dn;
    else if (changed)
      D[row] = dn;
    acc += p.wts ? (double)dn * (double)p.wts[row] : (double)dn;
  };
  for (int64_t base = base0; base < t1; base += (int64_t)NW * S::R) {
    if (early && base == base0)
      st.compute(base, t1, first, prev, b0, sink);
    else
      st.iter(p, base, t1, first, prev, sink);
  }

  acc = wave_sum(acc);
  if ((tid & 63) == 0) red[st.wave] = acc;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[w];
    (DRAWER ? p.tsum_w : p.tsum)[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------- registry
template <int FMT, int CB, int G, int CPL, int U, bool FULL, int NT, int RL, int CS = CEN_LDS, bool WITH_DRAWER = false>
static SeedVariant make_variant(int dexact) {
  SeedVariant v;
  v.fmt = FMT;
  v.dexact = dexact;
  v.cb = CB;
  v.g = G;
  v.cpl = CPL;
  v.u = U;
  v.full = FULL;
  v.nt = NT;
  v.rl = RL;
  v.cs = CS;
  v.rows_per_iter = (NT / 64) * U * (64 / G);
  v.fn = reinterpret_cast<const void*>(&seed_pass_kernel<FMT, CB, G, CPL, U, FULL, NT, RL, CS, 0>);
  if constexpr (WITH_DRAWER) {
    v.fn_drawer = reinterpret_cast<const void*>(&seed_pass_kernel<FMT, CB, G, CPL, U, FULL, NT, RL, CS, 1>);
    v.fn_lead = reinterpret_cast<const void*>(&seed_pass_kernel<FMT, CB, G, CPL, U, FULL, NT, RL, CS, 2>);
  } else {
    v.fn_drawer = nullptr;
    v.fn_lead = nullptr;
  }
  return v;
}

// Rows in 16-byte (d = 2: 8-byte) chunks for exact widths, U = 8 loads per
// lane; the widths of the named workloads also with U = 16; each also with
// the drawer.
#define KMPP_EXACT(NT, L)                                                                                   \
  make_variant<FMT_F32, 8, 1, 1, 8, true, NT, L, CEN_LDS, true>(2), make_variant<FMT_F32, 16, 1, 1, 8, true, NT, L, CEN_LDS, true>(4),      \
      make_variant<FMT_F32, 16, 2, 1, 8, true, NT, L, CEN_LDS, true>(8), make_variant<FMT_F32, 16, 4, 1, 8, true, NT, L, CEN_LDS, true>(16), \
      make_variant<FMT_F32, 16, 8, 1, 8, true, NT, L, CEN_LDS, true>(32), make_variant<FMT_F32, 16, 16, 1, 8, true, NT, L, CEN_LDS, true>(64), \
      make_variant<FMT_F32, 16, 32, 1, 8, true, NT, L, CEN_LDS, true>(128), make_variant<FMT_F32, 16, 64, 1, 8, true, NT, L, CEN_LDS, true>(256), \
      make_variant<FMT_F32, 16, 64, 2, 4, true, NT, L, CEN_LDS, true>(512),                                                \
      make_variant<FMT_F32, 16, 8, 1, 16, true, NT, L, CEN_LDS, true>(32), make_variant<FMT_F32, 16, 16, 1, 16, true, NT, L, CEN_LDS, true>(64), \
      make_variant<FMT_F32, 16, 32, 1, 16, true, NT, L, CEN_LDS, true>(128),                                               \
      make_variant<FMT_BF16, 16, 1, 1, 8, true, NT, L, CEN_LDS, true>(8), make_variant<FMT_BF16, 16, 2, 1, 8, true, NT, L, CEN_LDS, true>(16), \
      make_variant<FMT_BF16, 16, 4, 1, 8, true, NT, L, CEN_LDS, true>(32), make_variant<FMT_BF16, 16, 8, 1, 8, true, NT, L, CEN_LDS, true>(64), \
      make_variant<FMT_BF16, 16, 16, 1, 8, true, NT, L, CEN_LDS, true>(128), make_variant<FMT_BF16, 16, 32, 1, 8, true, NT, L, CEN_LDS, true>(256), \
      make_variant<FMT_BF16, 16, 8, 1, 16, true, NT, L, CEN_LDS, true>(64), make_variant<FMT_BF16, 16, 16, 1, 16, true, NT, L, CEN_LDS, true>(128), \
      make_variant<FMT_FP8, 16, 1, 1, 8, true, NT, L, CEN_LDS, true>(16), make_variant<FMT_FP8, 16, 2, 1, 8, true, NT, L, CEN_LDS, true>(32), \
      make_variant<FMT_FP8, 16, 4, 1, 8, true, NT, L, CEN_LDS, true>(64), make_variant<FMT_FP8, 16, 8, 1, 8, true, NT, L, CEN_LDS, true>(128), \
      make_variant<FMT_FP8, 16, 16, 1, 8, true, NT, L, CEN_LDS, true>(256),                                                \
      make_variant<FMT_FP8, 16, 4, 1, 16, true, NT, L, CEN_LDS, true>(64), make_variant<FMT_FP8, 16, 8, 1, 16, true, NT, L, CEN_LDS, true>(128)

// Any d: one element per chunk, G = min(64, pow2 >= d) lanes per row; FP32
// rows also with the drawer.
#define KMPP_GENERIC(NT)                                                                                    \
  make_variant<FMT_F32, 4, 1, 1, 8, false, NT, ROW_CACHED, CEN_LDS, true>(-1), make_variant<FMT_F32, 4, 2, 1, 8, false, NT, ROW_CACHED, CEN_LDS, true>(-2), \
      make_variant<FMT_F32, 4, 4, 1, 8, false, NT, ROW_CACHED, CEN_LDS, true>(-4), make_variant<FMT_F32, 4, 8, 1, 8, false, NT, ROW_CACHED, CEN_LDS, true>(-8), \
      make_variant<FMT_F32, 4, 16, 1, 8, false, NT, ROW_CACHED, CEN_LDS, true>(-16), make_variant<FMT_F32, 4, 32, 1, 8, false, NT, ROW_CACHED, CEN_LDS, true>(-32), \
      make_variant<FMT_F32, 4, 64, 1, 8, false, NT, ROW_CACHED, CEN_LDS, true>(-64), make_variant<FMT_F32, 4, 64, 4, 8, false, NT, ROW_CACHED, CEN_LDS, true>(-256), \
      make_variant<FMT_F32, 4, 64, 16, 2, false, NT, ROW_CACHED, CEN_LDS, true>(-1024),                                         \
      make_variant<FMT_F32, 4, 64, 64, 1, false, NT, ROW_CACHED, CEN_LDS, true>(-4096),                                         \
      make_variant<FMT_BF16, 2, 1, 1, 8, false, NT, ROW_CACHED>(-1), make_variant<FMT_BF16, 2, 2, 1, 8, false, NT, ROW_CACHED>(-2), \
      make_variant<FMT_BF16, 2, 4, 1, 8, false, NT, ROW_CACHED>(-4), make_variant<FMT_BF16, 2, 8, 1, 8, false, NT, ROW_CACHED>(-8), \
      make_variant<FMT_BF16, 2, 16, 1, 8, false, NT, ROW_CACHED>(-16), make_variant<FMT_BF16, 2, 32, 1, 8, false, NT, ROW_CACHED>(-32), \
      make_variant<FMT_BF16, 2, 64, 1, 8, false, NT, ROW_CACHED>(-64), make_variant<FMT_BF16, 2, 64, 4, 8, false, NT, ROW_CACHED>(-256), \
      make_variant<FMT_BF16, 2, 64, 16, 2, false, NT, ROW_CACHED>(-1024),                                        \
      make_variant<FMT_BF16, 2, 64, 64, 1, false, NT, ROW_CACHED>(-4096),                                        \
      make_variant<FMT_FP8, 1, 1, 1, 8, false, NT, ROW_CACHED>(-1), make_variant<FMT_FP8, 1, 2, 1, 8, false, NT, ROW_CACHED>(-2), \
      make_variant<FMT_FP8, 1, 4, 1, 8, false, NT, ROW_CACHED>(-4), make_variant<FMT_FP8, 1, 8, 1, 8, false, NT, ROW_CACHED>(-8), \
      make_variant<FMT_FP8, 1, 16, 1, 8, false, NT, ROW_CACHED>(-16), make_variant<FMT_FP8, 1, 32, 1, 8, false, NT, ROW_CACHED>(-32), \
      make_variant<FMT_FP8, 1, 64, 1, 8, false, NT, ROW_CACHED>(-64), make_variant<FMT_FP8, 1, 64, 4, 8, false, NT, ROW_CACHED>(-256), \
      make_variant<FMT_FP8, 1, 64, 16, 2, false, NT, ROW_CACHED>(-1024),                                         \
      make_variant<FMT_FP8, 1, 64, 64, 1, false, NT, ROW_CACHED>(-4096)

// Memory-space variants (FP32 rows, U = 8, 256 threads) of the widths of the
// two-dimensional points of the paper's experiments and of the 32-, 64- and
// 128-wide workloads: every centre source with every row path.
#define KMPP_SPACE_D(CB, G, DX)                                                                               \
  make_variant<FMT_F32, CB, G, 1, 8, true, 256, ROW_BUFFER, CEN_LDS>(DX),                                     \
      make_variant<FMT_F32, CB, G, 1, 8, true, 256, ROW_CACHED, CEN_SCALAR>(DX),                              \
      make_variant<FMT_F32, CB, G, 1, 8, true, 256, ROW_NONTEMPORAL, CEN_SCALAR>(DX),                         \
      make_variant<FMT_F32, CB, G, 1, 8, true, 256, ROW_BUFFER, CEN_SCALAR>(DX),                              \
      make_variant<FMT_F32, CB, G, 1, 8, true, 256, ROW_CACHED, CEN_GLOBAL>(DX),                              \
      make_variant<FMT_F32, CB, G, 1, 8, true, 256, ROW_NONTEMPORAL, CEN_GLOBAL>(DX),                         \
      make_variant<FMT_F32, CB, G, 1, 8, true, 256, ROW_BUFFER, CEN_GLOBAL>(DX)
#define KMPP_SPACES KMPP_SPACE_D(8, 1, 2), KMPP_SPACE_D(16, 8, 32), KMPP_SPACE_D(16, 16, 64), KMPP_SPACE_D(16, 32, 128)

const std::vector<SeedVariant>& seed_variants() {
  static const std::vector<SeedVariant> v = {KMPP_EXACT(256, ROW_CACHED), KMPP_EXACT(256, ROW_NONTEMPORAL),
                                             KMPP_EXACT(512, ROW_CACHED), KMPP_EXACT(512, ROW_NONTEMPORAL),
                                             KMPP_GENERIC(256),           KMPP_GENERIC(512),
                                             KMPP_SPACES};
  return v;
}

const void* seed_init_fn() { return reinterpret_cast<const void*>(&seed_init_kernel); }
const void* seed_wfirst_fn() { return reinterpret_cast<const void*>(&seed_wfirst_kernel); }
const void* seed_draw_fn(bool weighted) {
  return weighted ? reinterpret_cast<const void*>(&seed_draw_kernel<true>)
                  : reinterpret_cast<const void*>(&seed_draw_kernel<false>);
}
int seed_draw_threads() { return kDrawNT; }

}  // namespace kmpp
