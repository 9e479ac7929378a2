// assign.hip -- nearest-seed assignment, the partition O of the paper's
// Algorithm 1 (Section II), as a dense contraction on the matrix cores.
//
// score(i, j) = ||c_j||^2 - 2 <x_i, c_j> has the same argmin over j as
// ||x_i - c_j||^2.  The products run on MFMA with FP32 accumulation:
//   FP32 rows: v_mfma_f32_16x16x4_f32;
//   BF16 rows: v_mfma_f32_16x16x32_bf16 in two stages: every row against
//              the centres' BF16 high parts (one product, the high part's
//              rounding added to the bound), then the rows that leaves
//              undecided against high part plus BF16 remainder (two
//              products), so only the rows carry storage rounding;
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
// u = 2^-24 (FP32 accumulation; BF16 adds 2^-16 for the centre split, or
// 2^-8 ||x|| max_j ||c_j|| for the high part alone).
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
  float* cn;            // [Kp] -||c_j||^2 / 2 (FP32, direct; -inf for padding j >= K): each chain's start
  Ctl* ctl;             // status; nflag counts the rows queued for the recheck
  int32_t* labels;
  float* mind;
  float* cmax2;         // [3] workspace scalars: max_j ||c_j||^2, and (BF16 / FP8 rows)
                        // max_j ||c_j - hi_j||^2, max_j ||c_j - hi_j - lo_j||^2 (the
                        // residuals of the high part and of both parts)
  int64_t N;
  int32_t d, K, Kp, dp; // dp = padded d: 4 * VPL * (steps per tile)
  int32_t nblk;         // number of 16-row blocks
  int32_t all_rows;     // recheck kernel: every row instead of the queue
  float* Ct;            // [d, Kq] the centres transposed (zero past K)
  int32_t Kq;           // K rounded up to 64
  int32_t* cflags;      // [N] the rows queued for the recheck (nflag of them)
  int32_t* qa;          // [N] BF16/FP8 rows: the rows the first stage queued for the second (nqueue)
  uint64_t* pk;         // [kSplitCap] split recheck: (distance bits, index) minimum per queued row
};

// Queue positions below kSplitCap carry a 64-bit (distance, index) minimum
// for the split recheck, which spreads the centres over workgroups while the
// queue has fewer groups of rows than the recheck grid has workgroups.
constexpr int kSplitCap = 65536;
constexpr int kRecheckGrid = 2048;

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

// max(a, b, c, d) in two VALU operations (gfx950's three-input IEEE
// maximum; a NaN operand makes the result NaN, which the callers' compares
// then pass over).  No operand is canonicalised first, which the
// compiler's fmaxf would do to every MFMA result.
__device__ __forceinline__ float max4(float a, float b, float c, float d) {
  return __builtin_elementwise_maximum(__builtin_elementwise_maximum(a, b), __builtin_elementwise_maximum(c, d));
}

// Value e of a lane's quarter of a row from its MFMA fragments (FP32: one
// value per step; BF16 / FP8 as BF16: eight per step), exact in FP32.
template <int FMT, int S>
__device__ __forceinline__ float frag_value(const typename Frag<FMT>::A (&a)[S], int e) {
  if constexpr (FMT == FMT_F32) {
    return a[e];
  } else {
    // through the fragment's four 32-bit words (element 2w in the low half
    // of word w, 2w + 1 in the high half), as decode() reads them
    const uint4 w = __builtin_bit_cast(uint4, a[e / 8]);
    const int t = e % 8;
    const uint32_t word = (t >> 1) == 0 ? w.x : (t >> 1) == 1 ? w.y : (t >> 1) == 2 ? w.z : w.w;
    return (t & 1) ? bf16_hi(word) : bf16_lo(word);
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
// Every loop keeps kPrepU loads in flight per thread: indices are clamped
// into range so each load is issued unconditionally, and out-of-range values
// are masked afterwards (a guarded load would wait before the next one).
constexpr int kPrepU = 8;

// C[j][k] for a padded position (+0 outside K x d), loaded unconditionally
// and masked bitwise (a select on the loaded value may be turned back into
// a branch around the load).
__device__ __forceinline__ float c_at(const AssignParams& p, int64_t j, int64_t k) {
  const float v = p.C[min(j, (int64_t)p.K - 1) * p.d + min(k, (int64_t)p.d - 1)];
  const uint32_t keep = (j < p.K && k < p.d) ? 0xFFFFFFFFu : 0u;
  return __uint_as_float(__float_as_uint(v) & keep);
}

// out(e, val(e)) for e = tid, tid + stride, ... < total: whole batches of
// kPrepU elements per thread load everything first and store without a
// guard (a guarded store lets the compiler sink its load under the guard,
// one wait per element); the last partial batch goes one element at a time.
template <typename I, typename V, typename O>
__device__ __forceinline__ void strided_batched(I tid, I stride, I total, V&& val, O&& out) {
  const I full = total / (kPrepU * stride) * (kPrepU * stride);
  for (I e0 = tid; e0 < full; e0 += kPrepU * stride) {
    decltype(val(e0)) v[kPrepU];
#pragma unroll
    for (int u = 0; u < kPrepU; ++u) v[u] = val(e0 + u * stride);
#pragma unroll
    for (int u = 0; u < kPrepU; ++u) out(e0 + u * stride, v[u]);
  }
  for (I e = full + tid; e < total; e += stride) out(e, val(e));
}

// BF16 high part (round to nearest even) of c and BF16 remainder of c - hi
// (c - hi is exact in FP32), as 16-bit patterns.
__device__ __forceinline__ void split_bf16(float c, uint32_t& hi, uint32_t& lo) {
  const uint32_t hb = __float_as_uint(c);
  hi = ((hb + 0x7FFFu + ((hb >> 16) & 1u)) >> 16) & 0xFFFFu;
  const uint32_t rb = __float_as_uint(c - __uint_as_float(hi << 16));
  lo = ((rb + 0x7FFFu + ((rb >> 16) & 1u)) >> 16) & 0xFFFFu;
}

// A thread takes items tid, tid + stride, ...; it returns the bits of the
// largest ||c_j||^2 it saw and (BF16 / FP8 rows) of the largest squared
// residuals ||c_j - hi_j||^2 and ||c_j - hi_j - lo_j||^2 (as unsigned
// integers non-negative floats order like their values, and NaN above
// them).
// I: the index type (32-bit when every index fits, so the divisions below
// stay short and branch-free).
template <typename I>
__device__ uint3 prep_part(const AssignParams& p, int fmt, I tid, I stride) {
  const int Kt = p.Kp / 16;
  const int DQ = p.dp / 4;
  uint3 mx = make_uint3(0u, 0u, 0u);
  for (I j = tid; j < p.Kp; j += stride) {
    // ||c||^2 summed over k in order in FP64 and rounded once, so each chain
    // start carries a single FP32 rounding (at most 2^-25 ||c||^2), which the
    // error bound's slack covers; an FP32 sum would add up to d 2^-24 ||c||^2.
    // The residuals c - hi and c - hi - lo are exact in FP32 and their
    // squares are summed the same way.
    double a = 0.0, r1 = 0.0, r2 = 0.0;
    for (int k0 = 0; k0 < p.d; k0 += kPrepU) {
      float c[kPrepU];
#pragma unroll
      for (int u = 0; u < kPrepU; ++u) c[u] = c_at(p, j, k0 + u);
#pragma unroll
      for (int u = 0; u < kPrepU; ++u) {
        a = fma((double)c[u], (double)c[u], a);  // +0 past d: a unchanged
        if (fmt != FMT_F32) {
          uint32_t hi, lo;
          split_bf16(c[u], hi, lo);
          const float e1 = c[u] - __uint_as_float(hi << 16);
          const float e2 = e1 - __uint_as_float(lo << 16);
          r1 = fma((double)e1, (double)e1, r1);
          r2 = fma((double)e2, (double)e2, r2);
        }
      }
    }
    const float af = (float)a;
    p.cn[j] = j < p.K ? -0.5f * af : -INFINITY;  // exact scaling
    if (j < p.K) {
      mx.x = max(mx.x, __float_as_uint(af));
      mx.y = max(mx.y, __float_as_uint((float)r1));
      mx.z = max(mx.z, __float_as_uint((float)r2));
    }
  }
  if (fmt == FMT_F32) {
    float* Cp = (float*)const_cast<void*>(p.Cp);
    strided_batched(
        tid, stride, (I)Kt * DQ * 64,
        [&](I e) {
          const int lane = (int)(e % 64);
          const int s = (int)((e / 64) % DQ);
          const I jt = e / 64 / DQ;
          return c_at(p, 16 * jt + lane % 16, (lane / 16) * DQ + s);
        },
        [&](I e, float v) { Cp[e] = v; });
  } else {
    uint16_t* Cp = (uint16_t*)const_cast<void*>(p.Cp);
    const int S = DQ / 8;
    strided_batched(
        tid, stride, (I)Kt * 2 * S * 64 * 8,
        [&](I e) {
          const int t = (int)(e % 8);
          const int lane = (int)((e / 8) % 64);
          const int s = (int)((e / 512) % S);
          const I jt = e / 512 / S / 2;
          return c_at(p, 16 * jt + lane % 16, (lane / 16) * DQ + 8 * s + t);
        },
        [&](I e, float c) {
          uint32_t hi, lo;
          split_bf16(c, hi, lo);
          Cp[e] = (uint16_t)((e / 512 / S) % 2 == 0 ? hi : lo);  // part 0 high, 1 remainder
        });
  }
  return mx;
}

__global__ __launch_bounds__(256) void assign_prep_kernel(AssignParams p, int fmt) {
  const uint3 mx =
      prep_part<int64_t>(p, fmt, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
  unsigned int* const m = reinterpret_cast<unsigned int*>(p.cmax2);
  if (mx.x) atomicMax(m, mx.x);
  if (mx.y) atomicMax(m + 1, mx.y);
  if (mx.z) atomicMax(m + 2, mx.z);
}

// ---------------------------------------------------------------- main
// Workgroup: 4 waves x RB blocks of 16 rows.  The packed centre tiles are
// staged through LDS in chunks of TPC tiles, double-buffered: while the
// waves run the products of chunk c from one buffer, the next chunk's global
// loads are in flight and land in the other buffer at the end of the step,
// so every centre byte comes from L2 once per workgroup and is read from
// LDS by all four waves.
//
// The centres are the MFMA's first operand and the rows its second, so an
// accumulator holds centres 4q..4q+3 of the tile (q = lane / 16) for row
// lane % 16: each lane keeps one running top-2 per row block, and only the
// four lane groups of a row are merged at the end.  Each chain starts from
// the accumulator -||c_j||^2 / 2, so the running value is
// t = <x, c_j> - ||c_j||^2 / 2 = -score / 2 and the per-pair work is the
// top-2 update alone (largest t, ties to the smaller index).
// Waves per SIMD the compiler must allow: FP32 rows of width 97..128 fit 128
// registers, so four waves (measured faster than three); BF16 / FP8 rows of
// width 33..128 two (their two accumulator sets and the next tiles'
// operands take more registers than three waves allow, and each wave
// overlaps its own VALU and matrix work); no constraint otherwise.
constexpr int assign_min_waves(int fmt, int dqk) {
  return fmt == FMT_F32 && dqk == 32 ? 4 : (fmt != FMT_F32 && (dqk == 2 || dqk == 4) ? 2 : 1);
}

//
// BF16 / FP8 rows run in two stages (NP, the centre parts taken):
//   NP = 1: every row, products with the centres' BF16 high parts only (half
//           the matrix work); the bound adds 2 |x| max_j |c_j - hi_j|;
//           rows not decided go to queue qa;
//   NP = 2: only the rows in qa (gathered), products with both parts, the
//           bound adding 2 |x| max_j |c_j - hi_j - lo_j|; rows not decided
//           go to the recheck queue.
// FP32 rows take one stage (NP = 1, the FP32 product, tight bound).
template <int FMT, int DQK, int RB, int NP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(assign_min_waves(FMT, DQK))))
void assign_mfma_kernel(AssignParams p) {
  using F = Frag<FMT>;
  constexpr bool BF = FMT != FMT_F32;
  constexpr bool GATHER = BF && NP == 2;  // rows from qa
  constexpr bool FIRST = BF && NP == 1;   // undecided rows go to qa
  // BF16 / FP8 rows wider than 64 keep their best tile's values (SAVE): four
  // more VALU operations per tile and row block, which fit under the tile's
  // four or more MFMA steps; narrower rows' tiles have one or two steps, and
  // there the four direct distances of the tail cost less
  constexpr bool SAVE = BF && DQK >= 4;
  constexpr int S = DQK;                                  // MFMA steps per centre tile (per product)
  constexpr int TBG = BF ? 2 * S * 64 * 16 : S * 64 * 4;  // bytes of one packed centre tile (both parts)
  constexpr int TB = BF ? NP * S * 64 * 16 : TBG;         // bytes of the parts this stage stages in LDS
  constexpr int G = TB >= 16384 ? 2 : 4;                  // BF16 / FP8: tiles per group (see below)
  constexpr int TPC = BF ? (TB * G >= 16384 ? G : 16384 / TB) : (TB >= 16384 ? 1 : 16384 / TB);  // tiles per chunk
  constexpr int CHB = TPC * TB;                           // bytes per chunk
  constexpr int LPT = CHB / (256 * 16);                  // 16-byte loads per thread per chunk
  static_assert(CHB % (256 * 16) == 0, "chunk is a whole number of 16-byte loads per thread");
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int q = lane >> 4, col = lane & 15;
  const int DQ = p.dp / 4;  // contraction elements per lane group
  const int Kt = p.Kp / 16;
  __shared__ uint4 sbuf[2][CHB / 16];
  __shared__ uint4 scn[2][TPC * 4];  // chain starts -||c||^2 / 2 of the chunk's centres, 4 per entry
  __shared__ int s_nf;               // rows this workgroup queued for the recheck ...
  __shared__ int s_q[4 * RB * 16];   // ... and their indices
  __shared__ int s_base;             // where they go in the queue

  // first 16-row block of this wave; waves past the last block compute on
  // clamped rows and store nothing (they still take part in the barriers).
  // The second stage's rows are the first stage's queue; workgroups past it
  // leave at once.
  const int64_t nrows = GATHER ? (int64_t)p.ctl->nqueue : p.N;
  if (GATHER && (int64_t)blockIdx.x * 4 * RB * 16 >= nrows) return;
  const int64_t blk0 = ((int64_t)blockIdx.x * 4 + wave) * RB;
  int32_t rowv[RB];  // the row of each block for this lane's column, -1 past the end
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int64_t i = (blk0 + rb) * 16 + col;
    rowv[rb] = i < nrows ? (GATHER ? p.qa[i] : (int32_t)i) : -1;
  }

  // ---- row fragments (registers for the whole centre loop) and ||x||^2.
  // A lane's fragment values are consecutive in the row, so rows whose
  // width is a multiple of the fragment (4 FP32, 8 BF16/FP8 values) are read
  // with one vector load per fragment.
  typename F::A a[RB][S];
  float xs[RB];  // partial sum of x^2 over this lane's quarter
  const gptr<const char> xb = as_global(static_cast<const char*>(p.X));
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const bool ok = rowv[rb] >= 0;
    const int64_t row = ok ? rowv[rb] : p.N - 1;
    float acc = 0.0f;
    if constexpr (FMT == FMT_F32) {
      if (S % 4 == 0 && (p.d & 3) == 0) {
#pragma unroll
        for (int s4 = 0; s4 < S / 4; ++s4) {
          const int k = q * DQ + 4 * s4;
          const uint4 w = (ok && k < p.d) ? load_raw<16>(xb + (row * p.d + k) * 4) : make_uint4(0u, 0u, 0u, 0u);
          const float v[4] = {__uint_as_float(w.x), __uint_as_float(w.y), __uint_as_float(w.z), __uint_as_float(w.w)};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            a[rb][4 * s4 + e] = v[e];
            acc = fmaf(v[e], v[e], acc);
          }
        }
      } else {
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int k = q * DQ + s;
          const float v = (ok && k < p.d) ? static_cast<const float*>(p.X)[row * p.d + k] : 0.0f;
          a[rb][s] = v;
          acc = fmaf(v, v, acc);
        }
      }
    } else {
      // FP8: the row's power-of-two scale is applied here; q * 2^e is exact
      // in BF16 (3 mantissa bits, exponent within range)
      const float sc = (FMT == FMT_FP8) ? exp2i((int)p.xexp[row]) : 1.0f;
      if ((p.d & 7) == 0) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int k = q * DQ + 8 * s;
          const bool in = ok && k < p.d;
          float xv[8];
          if constexpr (FMT == FMT_BF16) {
            const uint4 w = in ? load_raw<16>(xb + (row * p.d + k) * 2) : make_uint4(0u, 0u, 0u, 0u);
            a[rb][s] = __builtin_bit_cast(v8bf, w);
            decode<FMT_BF16, 16>(w, xv);
          } else {
            const uint2 w = in ? load_raw<8>(xb + (row * p.d + k)) : make_uint2(0u, 0u);
            decode<FMT_FP8, 8>(w, xv);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
              xv[t] *= sc;
              a[rb][s][t] = bf_from_bits((uint16_t)(__float_as_uint(xv[t]) >> 16));
            }
          }
#pragma unroll
          for (int t = 0; t < 8; ++t) acc = fmaf(xv[t], xv[t], acc);
        }
      } else {
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int k = q * DQ + 8 * s + t;
            float xv = 0.0f;
            if (ok && k < p.d) {
              if constexpr (FMT == FMT_BF16) {
                xv = __uint_as_float((uint32_t) static_cast<const uint16_t*>(p.X)[row * p.d + k] << 16);
              } else {
                const uint8_t c8 = static_cast<const uint8_t*>(p.X)[row * p.d + k];
                xv = __builtin_amdgcn_cvt_f32_fp8((int)c8, 0) * sc;
              }
            }
            a[rb][s][t] = bf_from_bits((uint16_t)(__float_as_uint(xv) >> 16));
            acc = fmaf(xv, xv, acc);
          }
        }
      }
    }
    xs[rb] = acc;
  }

  // ---- per row block (this lane's centres): the largest t so far (m1),
  // the tile holding it (tb), this lane's four values of that tile (bv),
  // and the largest t outside those four values (m2)
  float m1[RB], m2[RB];
  int tb[RB];
  v4f bv[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    m1[rb] = -INFINITY;
    m2[rb] = -INFINITY;
    tb[rb] = -1;
    bv[rb] = v4f{-INFINITY, -INFINITY, -INFINITY, -INFINITY};
  }

  // ---- centre chunks through LDS
  const int nch = (Kt + TPC - 1) / TPC;
  const gptr<const char> cp = as_global(static_cast<const char*>(p.Cp));
  const gptr<const char> cnb = as_global(reinterpret_cast<const char*>(p.cn));
  uint4 pre[LPT];
  uint4 pcn = make_uint4(0u, 0u, 0u, 0u);
  // chunk c's word w: tile c * TPC + w / (TB / 16), the first TB bytes of the
  // tile's TBG (the high parts alone come first in each packed tile)
  auto gload = [&](int c) {
#pragma unroll
    for (int i = 0; i < LPT; ++i) {
      const int w = i * 256 + tid;
      const int64_t tile = (int64_t)c * TPC + w / (TB / 16);
      const int64_t idx = tile * (TBG / 16) + w % (TB / 16);
      pre[i] = tile < Kt ? load_raw<16>(cp + idx * 16) : make_uint4(0u, 0u, 0u, 0u);
    }
    const int64_t ci = (int64_t)c * TPC * 4 + tid;  // 16-byte entry of cn
    if (tid < TPC * 4) pcn = ci < (int64_t)Kt * 4 ? load_raw<16>(cnb + ci * 16) : make_uint4(0u, 0u, 0u, 0u);
  };
  auto sstore = [&](int b) {
#pragma unroll
    for (int i = 0; i < LPT; ++i) sbuf[b][i * 256 + tid] = pre[i];
    if (tid < TPC * 4) scn[b][tid] = pcn;
  };
  // tile tg's four values per row block enter as one: their maximum moves
  // (m1, tb, bv, m2) -- the new m2 is the median of (m1, m2, tile maximum);
  // six VALU operations per four values, ten where the values are saved
  // (FP32 rows keep none: their matrix-core work per tile is eight times
  // longer, and the registers would cost them a wave per SIMD).  A NaN value
  // makes the tile maximum NaN: no compare holds, and med3 then returns the
  // smaller of m1 and m2, so the state stays unchanged; a tile of -inf
  // values changes nothing.
  auto epilogue = [&](int tg, const v4f(&acc)[RB]) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      // both arms of each choice are plain values (so each compiles to a
      // select, not a branch)
      const v4f x = acc[rb];
      const float x0 = x[0], x1 = x[1], x2 = x[2], x3 = x[3];
      const float om1 = m1[rb], om2 = m2[rb];
      const int otb = tb[rb];
      const float tmax = max4(x0, x1, x2, x3);
      m2[rb] = __builtin_amdgcn_fmed3f(om1, om2, tmax);
      const bool gt = tmax > om1;
      tb[rb] = gt ? tg : otb;
      m1[rb] = gt ? tmax : om1;
      if constexpr (SAVE) {
        const v4f ob = bv[rb];
        const float b0 = ob[0], b1 = ob[1], b2 = ob[2], b3 = ob[3];
        const float n0 = gt ? x0 : b0, n1 = gt ? x1 : b1, n2 = gt ? x2 : b2, n3 = gt ? x3 : b3;
        bv[rb] = v4f{n0, n1, n2, n3};
      }
    }
  };
  gload(0);
  sstore(0);
  if (tid == 0) s_nf = 0;
  __syncthreads();
  if constexpr (BF) {
    // BF16 / FP8 rows: tiles in groups of G, the products of one tile issued
    // before the previous tile's values are folded in, so each wave's VALU
    // work overlaps its own matrix-core work (two accumulator sets).  The
    // centres are padded to a multiple of 64 (chain starts -inf), so every
    // chunk holds a whole number of groups.
    constexpr int NF = NP * S;
    for (int c = 0; c < nch; ++c) {
      if (c + 1 < nch) gload(c + 1);
      const int tn = min(TPC, Kt - c * TPC);  // a multiple of G
      const uint4* sb = &sbuf[c & 1][0];
      const uint4* sc = &scn[c & 1][0];
      auto frag = [&](int t, v8bf(&cf)[NF], v4f& init) {
        const uint4 c4 = sc[t * 4 + q];
        init = v4f{__uint_as_float(c4.x), __uint_as_float(c4.y), __uint_as_float(c4.z), __uint_as_float(c4.w)};
        const uint4* bp = sb + (t * NF) * 64 + lane;
#pragma unroll
        for (int f = 0; f < NF; ++f) cf[f] = __builtin_bit_cast(v8bf, bp[f * 64]);
      };
      auto products = [&](const v8bf(&cf)[NF], const v4f& init, v4f(&acc)[RB]) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cf[f], a[rb][f % S], f == 0 ? init : acc[rb], 0, 0, 0);
      };
      for (int t = 0; t < tn; t += G) {
        const int tg = c * TPC + t;
        v8bf f0[NF], f1[NF];
        v4f i0, i1, A[RB], B[RB];
        frag(t, f0, i0);
        frag(t + 1, f1, i1);
        products(f0, i0, A);
        if constexpr (G == 4) {
          frag(t + 2, f0, i0);
          products(f1, i1, B);
          epilogue(tg, A);
          frag(t + 3, f1, i1);
          products(f0, i0, A);
          epilogue(tg + 1, B);
          products(f1, i1, B);
          epilogue(tg + 2, A);
          epilogue(tg + 3, B);
        } else {
          products(f1, i1, B);
          epilogue(tg, A);
          epilogue(tg + 1, B);
        }
      }
      if (c + 1 < nch) sstore((c + 1) & 1);
      __syncthreads();
    }
  } else {
    for (int c = 0; c < nch; ++c) {
      if (c + 1 < nch) gload(c + 1);
      const int tn = min(TPC, Kt - c * TPC);
      for (int t = 0; t < tn; ++t) {
        // products of tile t (the chain starts from -||c_j||^2 / 2)
        const uint4 c4 = scn[c & 1][t * 4 + q];  // chain starts of this lane's centres j0..j0+3
        const v4f init = v4f{__uint_as_float(c4.x), __uint_as_float(c4.y), __uint_as_float(c4.z),
                             __uint_as_float(c4.w)};
        v4f acc[RB];
        const float* bp = reinterpret_cast<const float*>(&sbuf[c & 1][0]) + (t * S) * 64 + lane;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const float cv = bp[s * 64];
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(cv, a[rb][s], s == 0 ? init : acc[rb], 0, 0, 0);
        }
        epilogue(c * TPC + t, acc);
      }
      if (c + 1 < nch) sstore((c + 1) & 1);
      __syncthreads();
    }
  }

  // ---- per lane, the largest of its four saved values (ties: the smaller
  // index; it equals m1) and the largest of the other three; then merged
  // over the four lane groups of a row (lanes col + 16 q): the group with
  // the largest m1 (ties: the smaller centre index) gives the candidate bj.
  // Every other value of the row is at most oa (the owner's other saved
  // values and m2, the other groups' m1); every value outside the owner's
  // four saved centres is at most ot.  All four lanes of a row end with the
  // same b1, bj, oa, ot.
  float b1[RB], oa[RB], ot[RB];
  int bj[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    float v1 = bv[rb][0], v2 = -INFINITY;
    int ix = 0;
#pragma unroll
    for (int e = 1; e < 4; ++e) {
      const float v = bv[rb][e];
      if (v > v1) {
        v2 = v1;
        v1 = v;
        ix = e;
      } else {
        v2 = fmaxf(v2, v);
      }
    }
    b1[rb] = m1[rb];
    // (without saved values no row is decided without the direct
    // distances of its four candidates)
    oa[rb] = SAVE ? fmaxf(m2[rb], v2) : INFINITY;
    ot[rb] = m2[rb];
    bj[rb] = tb[rb] >= 0 ? tb[rb] * 16 + 4 * q + ix : INT_MAX;
#pragma unroll
    for (int o = 16; o < 64; o <<= 1) {
      const float o1 = __shfl_xor(b1[rb], o, 64);
      const int oj = __shfl_xor(bj[rb], o, 64);
      const float ooa = __shfl_xor(oa[rb], o, 64);
      const float oot = __shfl_xor(ot[rb], o, 64);
      if (o1 > b1[rb] || (o1 == b1[rb] && oj < bj[rb])) {
        oa[rb] = fmaxf(b1[rb], ooa);
        ot[rb] = fmaxf(b1[rb], oot);
        b1[rb] = o1;
        bj[rb] = oj;
      } else {
        oa[rb] = fmaxf(oa[rb], o1);
        ot[rb] = fmaxf(ot[rb], o1);
      }
    }
  }

  // ---- per row: ||x|| and the bound.  A row whose best score is ahead of
  // every other by more than the bound is decided (label bj); one ahead of
  // every score outside the owner's four saved centres is decided among
  // those four by their direct FP32 distances (ties: the smaller index);
  // other rows are queued.  The direct distance of the label is computed
  // when it is returned.  Direct distances run over this lane's quarter of
  // the row (the row values are the fragments in registers, exact) and are
  // summed over the four lane groups, so the branches around them are taken
  // by whole waves.
  const float cmax2 = p.cmax2[0];
  const float cmax = sqrtf(cmax2);
  // the centres' residual left out of the products: c - hi (first stage)
  // or c - hi - lo (second stage), its largest norm
  const float rmax = BF ? sqrtf(p.cmax2[FIRST ? 1 : 2]) : 0.0f;
  constexpr float kGrowth = 1.05f;
  constexpr int QV = F::VPL * S;  // values per lane quarter (= DQ)
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    float x2 = xs[rb];
    x2 += __shfl_xor(x2, 16, 64);
    x2 += __shfl_xor(x2, 32, 64);
    const int64_t row = rowv[rb];
    const float xn = sqrtf(x2) * 1.0001f;
    const float mag = cmax2 + 2.0f * xn * cmax;
    // E bounds the error of the difference of two t values (mag = max|c|^2
    // + 2 |x| max|c| spans both chains): FP32 accumulation over the
    // products and the chain start, (dp + 8) 2^-24 mag (2 dp products for
    // both centre parts; products of BF16 values are exact), plus, for
    // BF16 / FP8 rows, the centre residual r_j that the products leave out:
    // |<x, r_j>| <= |x| |r_j| per value, 2 |x| max|r| for a difference.
    // (Per value, the worst case is 2^-8 |c_k| for the high part, rounded to
    // 8 significant bits, and 2^-16 |c_k| for both parts; residual norms
    // are typically well under that.)
    const float unit = (FMT == FMT_F32 || NP == 1) ? (float)(p.dp + 8) * 0x1p-24f
                                                   : (float)(2 * p.dp + 8) * 0x1p-24f;
    const float E = (unit * mag + 2.0f * xn * rmax) * kGrowth;
    // t values: score gaps are twice the t gaps
    const bool sure_a = 2.0f * (b1[rb] - oa[rb]) > 2.0f * E && bj[rb] < p.K;
    const bool sure_t = 2.0f * (b1[rb] - ot[rb]) > 2.0f * E && bj[rb] < p.K;
    const bool four = sure_t && !sure_a;
    // direct distance of this row to centre j (clamped into range); a lane's
    // quarter of a centre row is contiguous, read with 16-byte loads where
    // it lies wholly inside the row, else element by element (positions
    // past d masked)
    auto qdist = [&](int j) {
      const float* crow = p.C + (int64_t)min(max(j, 0), p.K - 1) * p.d;
      float dd = 0.0f;
      if (QV % 4 == 0 && (p.d & 3) == 0 && (q + 1) * QV <= p.d) {
        const float4* c4 = reinterpret_cast<const float4*>(crow + q * QV);
#pragma unroll
        for (int i = 0; i < QV / 4; ++i) {
          const float4 cc = c4[i];
          const float cw[4] = {cc.x, cc.y, cc.z, cc.w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float df = frag_value<FMT>(a[rb], 4 * i + e) - cw[e];
            dd = fmaf(df, df, dd);
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < QV; ++e) {
          const int k = q * QV + e;
          const float df = frag_value<FMT>(a[rb], e) - crow[min(k, p.d - 1)];
          dd = k < p.d ? fmaf(df, df, dd) : dd;
        }
      }
      dd += __shfl_xor(dd, 16, 64);
      dd += __shfl_xor(dd, 32, 64);
      return dd;
    };
    int best = bj[rb];
    float dbest = 0.0f;
    if (__ballot(four) != 0ull) {
      const int j0 = four ? (bj[rb] & ~3) : 0;  // the owner's four saved centres
      float db = INFINITY;
      int bb = INT_MAX;
      for (int v = 0; v < 4; ++v) {
        const float dd = qdist(j0 + v);
        if (j0 + v < p.K && dd < db) {
          db = dd;
          bb = j0 + v;
        }
      }
      if (four) {
        best = bb;
        dbest = db;
      }
    }
    if (p.mind != nullptr && __ballot(sure_a) != 0ull) {
      const float dd = qdist(sure_a ? bj[rb] : 0);
      if (sure_a) dbest = dd;
    }
    const bool mine = q == 0 && row >= 0;
    if (mine && sure_t) {
      p.labels[row] = best;
      if (p.mind) p.mind[row] = dbest;
    }
    // rows for the recheck are collected in LDS
    const bool flag = mine && !sure_t;
    const unsigned long long fm = __ballot(flag);
    if (fm) {
      int base = 0;
      if (lane == 0) base = atomicAdd(&s_nf, __popcll(fm));
      base = __shfl(base, 0, 64);
      if (flag) s_q[base + __popcll(fm & ((1ull << lane) - 1ull))] = (int32_t)row;
    }
  }
  // ... and appended to the queue at a range reserved with one atomic per
  // workgroup (the queue's order does not matter: each row's recheck is
  // independent of the others)
  __syncthreads();
  uint32_t* const counter = FIRST ? &p.ctl->nqueue : &p.ctl->nflag;
  int32_t* const queue = FIRST ? p.qa : p.cflags;
  if (tid == 0) s_base = s_nf ? (int)atomicAdd(counter, (uint32_t)s_nf) : 0;
  __syncthreads();
  for (int i = tid; i < s_nf; i += 256) {
    queue[s_base + i] = s_q[i];
    // the split recheck's minimum for this queue position starts above every
    // (distance, index) pair
    if (!FIRST && s_base + i < kSplitCap) p.pk[s_base + i] = ~0ull;
  }
}

// ---------------------------------------------------------------- recheck
// Direct FP32 distances sum_k (x_k - c_jk)^2 (k in order) of the queued
// rows (every row in all-rows mode) to every centre, ties to the smallest
// index.  A wave takes kRR rows at once: lanes run over 64 centres at a
// time, read coalesced from the transposed copy Ct[k][j], and every centre
// value serves all kRR rows, whose values are the same for all lanes.
// kRR: 4 rows for FP32 (few rows are queued, and smaller groups spread
// them over more workgroups: 210 -> 181 us on 4.2M x 128), 8 for BF16 /
// FP8 rows, whose wider error bound queues many more (301 us with 8,
// 359 us with 4; 16 rows measured slower for both).
template <int FMT>
constexpr int recheck_rows() { return FMT == FMT_F32 ? 4 : 8; }

template <typename I>
__device__ void transpose_part(const AssignParams& p, I tid, I stride) {
  strided_batched(
      tid, stride, (I)p.d * p.Kq, [&](I e) { return c_at(p, e % p.Kq, e / p.Kq); },
      [&](I e, float v) { p.Ct[e] = v; });
}

__global__ __launch_bounds__(256) void assign_transpose_kernel(AssignParams p) {
  transpose_part<int64_t>(p, (int64_t)blockIdx.x * 256 + threadIdx.x, (int64_t)gridDim.x * 256);
}

// A workgroup takes kRR rows at once and its four waves split the centres
// (64 per step, wave w from step w on).  XL: the rows' values are first
// copied into LDS (interleaved by row, so one 16-byte read returns four
// rows' value at one k); rows wider than kRecheckLdsD are read through the
// scalar unit instead.  The waves' results are combined in wave order with
// ties to the smaller index.
constexpr int kRecheckLdsD = 256;

template <int FMT, bool XL>
__global__ __launch_bounds__(256) void assign_recheck_kernel(AssignParams p) {
  constexpr int kRR = recheck_rows<FMT>();
  static_assert(kRR % 4 == 0, "rows are staged in LDS four to a 16-byte word");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ float4 sx[XL ? kRecheckLdsD * (kRR / 4) : 1];
  __shared__ float s_b[4][kRR];
  __shared__ int s_i[4][kRR];
  const int64_t n = p.all_rows ? p.N : (int64_t)p.ctl->nflag;
  const int64_t groups = (n + kRR - 1) / kRR;
  for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
    int64_t rows[kRR];
#pragma unroll
    for (int r = 0; r < kRR; ++r) {
      const int64_t i = min(g * kRR + r, n - 1);  // a short last group repeats its last row
      rows[r] = p.all_rows ? i : (int64_t)p.cflags[i];
    }
    if constexpr (XL) {
      float* xw = reinterpret_cast<float*>(&sx[0]);
      for (int e = tid; e < p.d * kRR; e += 256) {
        const int k = e / kRR, r = e % kRR;
        int64_t rr = rows[0];
#pragma unroll
        for (int q = 1; q < kRR; ++q) rr = r == q ? rows[q] : rr;
        xw[e] = x_at<FMT>(p, rr, k);
      }
      __syncthreads();
    }
    float best[kRR];
    int bi[kRR];
#pragma unroll
    for (int r = 0; r < kRR; ++r) {
      best[r] = INFINITY;
      bi[r] = INT_MAX;
    }
    for (int j0 = wave * 64; j0 < p.K; j0 += 256) {
      const int j = j0 + lane;
      const float* ct = p.Ct + j;
      float acc[kRR];
#pragma unroll
      for (int r = 0; r < kRR; ++r) acc[r] = 0.0f;
#pragma unroll 8
      for (int k = 0; k < p.d; ++k) {
        const float cv = ct[(int64_t)k * p.Kq];
        float xv[kRR];
        if constexpr (XL) {
#pragma unroll
          for (int r4 = 0; r4 < kRR / 4; ++r4) {
            const float4 v = sx[k * (kRR / 4) + r4];
            xv[4 * r4] = v.x;
            xv[4 * r4 + 1] = v.y;
            xv[4 * r4 + 2] = v.z;
            xv[4 * r4 + 3] = v.w;
          }
        } else {
#pragma unroll
          for (int r = 0; r < kRR; ++r) xv[r] = x_at<FMT>(p, rows[r], k);
        }
#pragma unroll
        for (int r = 0; r < kRR; ++r) {
          const float df = xv[r] - cv;
          acc[r] = fmaf(df, df, acc[r]);
        }
      }
#pragma unroll
      for (int r = 0; r < kRR; ++r)
        if (j < p.K && acc[r] < best[r]) {
          best[r] = acc[r];
          bi[r] = j;
        }
    }
#pragma unroll
    for (int r = 0; r < kRR; ++r) {
      float b = best[r];
      int ib = bi[r];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const float tb = __shfl_xor(b, o, 64);
        const int ti = __shfl_xor(ib, o, 64);
        if (tb < b || (tb == b && ti < ib)) {
          b = tb;
          ib = ti;
        }
      }
      if (lane == 0) {
        s_b[wave][r] = b;
        s_i[wave][r] = ib;
      }
    }
    __syncthreads();
    if (tid < kRR && g * kRR + tid < n) {
      float b = s_b[0][tid];
      int ib = s_i[0][tid];
#pragma unroll
      for (int w = 1; w < 4; ++w) {
        const float tb = s_b[w][tid];
        const int ti = s_i[w][tid];
        if (tb < b || (tb == b && ti < ib)) {
          b = tb;
          ib = ti;
        }
      }
      int64_t row = rows[0];
#pragma unroll
      for (int q = 1; q < kRR; ++q) row = tid == q ? rows[q] : row;
      // no comparable distance (NaN in the row or the centres): label -1
      p.labels[row] = ib < p.K ? ib : -1;
      if (p.mind) p.mind[row] = ib < p.K ? b : __builtin_nanf("");
    }
    __syncthreads();  // LDS is rewritten by the next group
  }
}

// The recheck for rows of width d <= 128 (the MFMA path's queue): a
// workgroup takes kTR = 32 queued rows at once.  Their values go to LDS as
// [k][row]; the centres stream through LDS in tiles of kTC = 32 from the
// transposed copy Ct (128 contiguous bytes per k), double-buffered (the next
// tile's loads are in flight while the current one is used).  Thread
// (wave w, lane l) takes centre l % 32 of each tile and the four rows
// 8w + 4 (l / 32) .. +3, whose values at one k are a single 16-byte LDS read;
// every centre value serves four rows.  Per thread, centres come in index
// order (strict comparison keeps the smaller index), and the 32 lanes of a
// half-wave are merged with ties to the smaller index.
//
// A short queue has fewer groups of rows than the grid has workgroups; the
// centre tiles are then split into ranges, one work item per (group, range),
// and each row's result is the minimum of its ranges' (distance bits,
// index) pairs, taken with a 64-bit atomic minimum (distances are >= 0, so
// their bit patterns order like the values; equal distances keep the
// smaller index) and written out by assign_recheck_finish_kernel.
constexpr int kTR = 32, kTC = 32, kTDMax = 128;
constexpr int kMinTilesPerSplit = 2;

// centre tiles per work item: all of them (no split) for long queues,
// all-rows mode or a queue beyond the split slots
__device__ __forceinline__ int recheck_tiles_per_item(int64_t n, int ntile, int all_rows) {
  const int64_t groups = (n + kTR - 1) / kTR;
  if (all_rows || groups == 0 || groups >= kRecheckGrid || n > kSplitCap) return ntile;
  const int want = (int)((kRecheckGrid + groups - 1) / groups);  // ranges wanted per group
  return max((ntile + want - 1) / want, min(kMinTilesPerSplit, ntile));
}

template <int FMT>
__global__ __launch_bounds__(256) void assign_recheck_tiled_kernel(AssignParams p) {
  __shared__ float4 xs4[kTDMax * kTR / 4];           // row values, [k][row]
  __shared__ float4 cs4[2][kTDMax * kTC / 4];        // centre tiles, [k][centre]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cj = lane & 31;                           // centre within the tile
  const int r0 = wave * 8 + (lane >> 5) * 4;          // first of this thread's four rows
  const int d = p.d;
  const int64_t n = p.all_rows ? p.N : (int64_t)p.ctl->nflag;
  const int64_t groups = (n + kTR - 1) / kTR;
  const int ntile = (p.K + kTC - 1) / kTC;            // Kq >= ntile * kTC (Kq is a multiple of 64)
  const int tpi = recheck_tiles_per_item(n, ntile, p.all_rows);
  const int splits = (ntile + tpi - 1) / tpi;
  const int64_t items = groups * splits;
  const int tw = d * (kTC / 4);                       // 16-byte words of one centre tile
  const gptr<const char> ctb = as_global(reinterpret_cast<const char*>(p.Ct));
  float* xs = reinterpret_cast<float*>(xs4);
  // tile t's words: word w = (k, j4) -> Ct[k][t * kTC + 4 j4 .. +3]
  constexpr int kPer = kTDMax * kTC / 4 / 256;        // words per thread at most
  // every load in bounds (word clamped) and issued unconditionally; only
  // the words of the tile are stored
  uint4 pre[kPer];
  auto tload = [&](int t) {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int w = min(i * 256 + tid, tw - 1);
      const int k = w / (kTC / 4), j4 = w % (kTC / 4);
      pre[i] = load_raw<16>(ctb + ((int64_t)k * p.Kq + (int64_t)t * kTC + 4 * j4) * 4);
    }
  };
  auto tstore = [&](int b) {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int w = i * 256 + tid;
      if (w < tw) cs4[b][w] = __builtin_bit_cast(float4, pre[i]);
    }
  };
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int64_t g = it / splits;
    const int t0 = (int)(it % splits) * tpi, t1 = min(ntile, t0 + tpi);
    // rows of the group (a short last group repeats its last row)
    for (int e = tid; e < d * kTR; e += 256) {
      const int k = e / kTR, r = e % kTR;
      const int64_t i = min(g * kTR + r, n - 1);
      const int64_t row = p.all_rows ? i : (int64_t)p.cflags[i];
      xs[e] = x_at<FMT>(p, row, k);
    }
    tload(t0);
    tstore(0);
    __syncthreads();
    float best[4];
    int bi[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      best[r] = INFINITY;
      bi[r] = INT_MAX;
    }
    for (int t = t0; t < t1; ++t) {
      if (t + 1 < t1) tload(t + 1);
      const float* cs = reinterpret_cast<const float*>(cs4[(t - t0) & 1]);
      float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
      for (int k = 0; k < d; ++k) {
        const float c = cs[k * kTC + cj];
        const float4 x = xs4[(k * kTR + r0) / 4];
        const float xv[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float df = xv[r] - c;
          acc[r] = fmaf(df, df, acc[r]);
        }
      }
      const int j = t * kTC + cj;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (j < p.K && acc[r] < best[r]) {
          best[r] = acc[r];
          bi[r] = j;
        }
      if (t + 1 < t1) tstore((t + 1 - t0) & 1);
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float b = best[r];
      int ib = bi[r];
#pragma unroll
      for (int o = 16; o > 0; o >>= 1) {
        const float tb = __shfl_xor(b, o, 64);
        const int ti = __shfl_xor(ib, o, 64);
        if (tb < b || (tb == b && ti < ib)) {
          b = tb;
          ib = ti;
        }
      }
      const int64_t i = g * kTR + r0 + r;
      if (cj == 0 && i < n) {
        if (splits == 1) {
          const int64_t row = p.all_rows ? i : (int64_t)p.cflags[i];
          // no comparable distance (NaN in the row or the centres): label -1
          p.labels[row] = ib < p.K ? ib : -1;
          if (p.mind) p.mind[row] = ib < p.K ? b : __builtin_nanf("");
        } else {
          // b is +inf or a distance >= 0 here (NaN never wins a comparison)
          atomicMin(reinterpret_cast<unsigned long long*>(p.pk + i),
                    ((unsigned long long)__float_as_uint(b) << 32) | (uint32_t)ib);
        }
      }
    }
    __syncthreads();  // the next item rewrites the row values
  }
}

// The split recheck's results: the minimum pair of each queued row becomes
// its label and distance (nothing to do when the queue was not split).
__global__ __launch_bounds__(256) void assign_recheck_finish_kernel(AssignParams p) {
  const int64_t n = p.all_rows ? p.N : (int64_t)p.ctl->nflag;
  const int ntile = (p.K + kTC - 1) / kTC;
  if (recheck_tiles_per_item(n, ntile, p.all_rows) >= ntile) return;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const uint64_t v = p.pk[i];
    const int ib = (int)(uint32_t)v;
    const int32_t row = p.cflags[i];
    p.labels[row] = ib < p.K ? ib : -1;
    if (p.mind) p.mind[row] = ib < p.K ? __uint_as_float((uint32_t)(v >> 32)) : __builtin_nanf("");
  }
}

__global__ void assign_reset_kernel(Ctl* ctl, float* cmax2) {
  ctl->status = KMPP_OK;
  ctl->nflag = 0u;
  ctl->nqueue = 0u;
  cmax2[0] = 0.0f;
  cmax2[1] = 0.0f;
  cmax2[2] = 0.0f;
}

// Small centre sets: the reset, the transposed copy, the chain starts and
// the packed fragments in one workgroup (one launch instead of three).
__global__ __launch_bounds__(1024) void assign_setup_kernel(AssignParams p, int fmt) {
  __shared__ uint3 smx[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) {
    p.ctl->status = KMPP_OK;
    p.ctl->nflag = 0u;
    p.ctl->nqueue = 0u;
  }
  // every index fits 32 bits here (Kp * dp <= 65536, d <= 256)
  transpose_part<uint32_t>(p, (uint32_t)tid, 1024u);
  uint3 mx = prep_part<uint32_t>(p, fmt, (uint32_t)tid, 1024u);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mx.x = max(mx.x, (uint32_t)__shfl_xor((int)mx.x, o, 64));
    mx.y = max(mx.y, (uint32_t)__shfl_xor((int)mx.y, o, 64));
    mx.z = max(mx.z, (uint32_t)__shfl_xor((int)mx.z, o, 64));
  }
  if (lane == 0) smx[wave] = mx;
  __syncthreads();
  if (tid == 0) {
    uint3 m = make_uint3(0u, 0u, 0u);
    for (int w = 0; w < 16; ++w) {
      m.x = max(m.x, smx[w].x);
      m.y = max(m.y, smx[w].y);
      m.z = max(m.z, smx[w].z);
    }
    uint32_t* const o = reinterpret_cast<uint32_t*>(p.cmax2);
    o[0] = m.x;
    o[1] = m.y;
    o[2] = m.z;
  }
}

// ---------------------------------------------------------------- host
namespace {
inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }
inline int round_up(int x, int m) { return (x + m - 1) / m * m; }
// padded centre elements (Kp * dp) up to which one workgroup prepares the centres
constexpr int64_t kSetupOneWg = 1 << 16;

struct AssignLayout {
  size_t cn, cmax, cp, ct, cflags, qa, pk, total;
  int Kp, dp, Kq;
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
  // BF16 / FP8: a multiple of 64, so the main loop's groups of tiles are whole
  L.Kp = round_up(K, dtype == KMPP_F32 ? 16 : 64);
  const int steps = assign_steps(d, dtype);
  L.dp = steps ? 4 * (dtype == KMPP_F32 ? 1 : 8) * steps : round_up(d, 4);
  size_t off = sizeof(Ctl);
  L.cn = off;
  off += a256(sizeof(float) * L.Kp);
  L.cmax = off;
  off += 256;
  L.cp = off;
  off += a256(dtype == KMPP_F32 ? sizeof(float) * (size_t)L.Kp * L.dp : sizeof(uint16_t) * 2 * (size_t)L.Kp * L.dp);
  L.Kq = round_up(K, 64);
  L.ct = off;
  off += a256(sizeof(float) * (size_t)L.Kq * (size_t)d);
  L.cflags = off;
  off += a256(sizeof(int32_t) * (size_t)N);
  L.qa = off;
  if (dtype != KMPP_F32) off += a256(sizeof(int32_t) * (size_t)N);
  L.pk = off;
  off += sizeof(uint64_t) * kSplitCap;
  L.total = off;
  return L;
}

// One stage over all rows (FP32), or the two stages of BF16 / FP8 rows (the
// second's grid covers every row; its workgroups past the queue leave at once).
template <int FMT, int DQK, int RB>
hipError_t launch_main(AssignParams& p, hipStream_t stream) {
  const int64_t waves = (p.nblk + RB - 1) / RB;
  const int64_t blocks = (waves + 3) / 4;
  hipLaunchKernelGGL((assign_mfma_kernel<FMT, DQK, RB, 1>), dim3((unsigned)blocks), dim3(256), 0, stream, p);
  if constexpr (FMT != FMT_F32)
    hipLaunchKernelGGL((assign_mfma_kernel<FMT, DQK, RB, 2>), dim3((unsigned)blocks), dim3(256), 0, stream, p);
  return hipGetLastError();
}

template <int FMT>
void launch_recheck(const AssignParams& p, hipStream_t stream) {
  const unsigned grid = kRecheckGrid;
  if (p.d <= kTDMax) {
    hipLaunchKernelGGL((assign_recheck_tiled_kernel<FMT>), dim3(grid), dim3(256), 0, stream, p);
    hipLaunchKernelGGL(assign_recheck_finish_kernel, dim3(kSplitCap / 256), dim3(256), 0, stream, p);
  } else if (p.d <= kRecheckLdsD)
    hipLaunchKernelGGL((assign_recheck_kernel<FMT, true>), dim3(grid), dim3(256), 0, stream, p);
  else
    hipLaunchKernelGGL((assign_recheck_kernel<FMT, false>), dim3(grid), dim3(256), 0, stream, p);
}

// RB row blocks per wave: fragment registers RB * steps * (1 or 4) <= 64
// (BF16 / FP8 rows of width 33..64 take 8 blocks, 2 % faster than 4 at two
// waves per SIMD; for widths 65..128, 6 or 8 blocks measured slower, and so
// did 2 blocks at three waves per SIMD: 1.37 -> 1.50 ms on 4.2M x 128)
template <int FMT>
hipError_t dispatch_main(AssignParams& p, int steps, hipStream_t stream) {
  if constexpr (FMT == FMT_F32) {
    switch (steps) {
      case 1: return launch_main<FMT, 1, 4>(p, stream);
      case 2: return launch_main<FMT, 2, 8>(p, stream);
      case 4: return launch_main<FMT, 4, 4>(p, stream);
      case 8: return launch_main<FMT, 8, 4>(p, stream);
      case 16: return launch_main<FMT, 16, 4>(p, stream);
      case 32: return launch_main<FMT, 32, 2>(p, stream);
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (steps) {
      case 1: return launch_main<FMT, 1, 4>(p, stream);
      case 2: return launch_main<FMT, 2, 8>(p, stream);
      case 4: return launch_main<FMT, 4, 4>(p, stream);
      case 8: return launch_main<FMT, 8, 2>(p, stream);
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
  p.labels = labels;
  p.mind = mind;
  p.cmax2 = reinterpret_cast<float*>(w + L.cmax);
  p.N = N;
  p.d = d;
  p.K = K;
  p.Kp = L.Kp;
  p.dp = L.dp;
  p.nblk = (int)((N + 15) / 16);
  p.Ct = reinterpret_cast<float*>(w + L.ct);
  p.Kq = L.Kq;
  p.cflags = reinterpret_cast<int32_t*>(w + L.cflags);
  p.qa = reinterpret_cast<int32_t*>(w + L.qa);
  p.pk = reinterpret_cast<uint64_t*>(w + L.pk);

  p.all_rows = 0;

  const int steps = assign_steps(d, dtype);
  if (steps && (int64_t)L.Kp * L.dp <= kSetupOneWg) {
    hipLaunchKernelGGL(assign_setup_kernel, dim3(1), dim3(1024), 0, stream, p, dtype);
  } else {
    hipLaunchKernelGGL(assign_reset_kernel, dim3(1), dim3(1), 0, stream, p.ctl, p.cmax2);
    hipLaunchKernelGGL(assign_transpose_kernel, dim3(256), dim3(256), 0, stream, p);
    if (steps) hipLaunchKernelGGL(assign_prep_kernel, dim3(256), dim3(256), 0, stream, p, dtype);
  }
  if (steps) {
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
  if (dtype == KMPP_F32)
    launch_recheck<FMT_F32>(p, stream);
  else if (dtype == KMPP_BF16)
    launch_recheck<FMT_BF16>(p, stream);
  else
    launch_recheck<FMT_FP8>(p, stream);
  return hipGetLastError() == hipSuccess ? KMPP_OK : KMPP_E_HIP;
}

}  // namespace kmpp
