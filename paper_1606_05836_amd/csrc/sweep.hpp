// Gray-code sweep of the BB/FG (Glynn) and Ryser permanent formulas on gfx950.
//
// Formulas (Supplementary "Parallelization and Optimization"):
//   Ryser, Eq. (S1):  Per(A) = (-1)^n sum_{S} (-1)^{|S|} prod_i sum_{j in S} a_ij
//   BB/FG, Eq. (S2):  Per(A) = 2^{-(n-1)} sum_delta (prod_k delta_k) prod_i sum_j delta_j a_ij,
//                     delta_0 = +1, delta_k = +-1.
// The paper evaluates every term from scratch (O(n^2) per term) and notes that
// Gray-code order would cut this to O(n) but serialises the sweep.  Here the
// 2^nb terms (nb = n-1 for BB/FG, n for Ryser) are walked in reflected Gray
// order g(k) = k ^ (k >> 1), and the serial dependency is broken by cutting
// [0, 2^nb) into contiguous chunks of L = 2^c terms -- the contiguous
// per-process ranges of the parallel listings, pushed down to one GPU lane --
// with the row sums seeded from scratch at each chunk start.
//
// Table (built by the prep kernel, staged into LDS per workgroup): n columns
// T[0..n-1] of n complex entries each.
//   BB/FG:  T[0] = a_{.,0};  T[b+1] = -2 a_{.,b+1}   (Gray bit b <-> column b+1)
//   Ryser:  T[b] = a_{.,b}                            (Gray bit b <-> column b)
// The update column of Gray bit b is U_b = T[b + off] (off = 1 for BB/FG, 0
// for Ryser).  A Gray bit set means delta = -1 (BB/FG) or the column is in S
// (Ryser); a step that sets bit b adds U_b to every row sum, one that clears
// it subtracts U_b.  (BB/FG: flipping delta_c changes r_i by 2 delta_c(new)
// a_ic, and 2 a_ic scaled by -1 is exact.)
//
// Term sign: prod delta = (-1)^|S| = (-1)^popcount(g(k)) = (-1)^k.  Chunks
// start at multiples of L (L even), so in a chunk the sign is (-1)^t, t the
// offset in the chunk.
//
// Every lane of a wavefront walks its own chunk, all in lockstep: the step to
// offset t flips Gray bit ctz(t), the same on every lane, so the column to add
// is wave-uniform.  The low columns U_0..U_{D-1}, used by 1 - 2^-D of all
// steps, live in VGPRs laid out for 64-bit DPP row broadcast (row_newbcast);
// each row-sum update is one v_fmac_f64 whose first operand is the broadcast
// column entry and whose second is +-1.0 (the same rounding as an add).  The
// remaining steps read their column from a staged buffer in the same layout,
// refilled from the LDS table ahead of them (stage_column), or, in sweeps
// without registers to spare, from LDS at the step (all lanes the same
// address).
// The new value of the flipped bit is "set" iff bit ctz(t)+1 of k is clear;
// that bit comes from t except at t = L/2, where it is the chunk parity and
// differs between neighbouring lanes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

#include "dd.hpp"

namespace ph {

enum { ALGO_GLYNN = 0, ALGO_RYSER = 1 };

// Largest n whose sweep keeps update columns in VGPRs (larger n are register
// bound and take every column from LDS).
constexpr int DPP_NMAX = 44;

template <int S, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (S < E) {
    f(std::integral_constant<int, S>{});
    static_for<S + 1, E>(f);
  }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}

// Sizes derived from n and the formula.
template <int N, int ALGO>
struct Shape {
  static constexpr int NB = ALGO == ALGO_GLYNN ? N - 1 : N;  // Gray bits
  static constexpr int OFF = ALGO == ALGO_GLYNN ? 1 : 0;     // U_b = T[b + OFF]
  // unrolled block of 2^LOGU steps (chunks with c < LOGU take a plain loop)
  static constexpr int LOGU = NB >= 4 ? 4 : (NB >= 1 ? 1 : 0);
  // number of DPP-resident update columns (register budget)
  static constexpr int D0 = N <= 40 ? 4 : (N <= 44 ? 2 : 0);
  static_assert(D0 == 0 || N <= DPP_NMAX, "DPP-resident columns need a spill-free kernel");
  static constexpr int D = D0 < LOGU ? D0 : LOGU;
  static constexpr int NP = (2 * N + 15) / 16;  // VGPR pairs per resident column
};

// r_d += bcast(col lane K of the row) * sgn  (v_fmac_f64, DPP row_newbcast).
template <int K>
__device__ __forceinline__ void dpp_fmac(double& r, double col, double sgn) {
#define PH_DPP(k)                                                                               \
  if constexpr (K == k)                                                                         \
    asm("v_fmac_f64_dpp %0, %1, %2 row_newbcast:" #k " row_mask:0xf bank_mask:0xf" : "+v"(r) \
        : "v"(col), "v"(sgn));
  PH_DPP(0) PH_DPP(1) PH_DPP(2) PH_DPP(3) PH_DPP(4) PH_DPP(5) PH_DPP(6) PH_DPP(7)
  PH_DPP(8) PH_DPP(9) PH_DPP(10) PH_DPP(11) PH_DPP(12) PH_DPP(13) PH_DPP(14) PH_DPP(15)
#undef PH_DPP
}

// r += sgn * U (U resident: pair p holds doubles 16p..16p+15 of the column,
// re/im interleaved, lane l of each 16-lane row holding element l).
template <int N, int NP>
__device__ __forceinline__ void add_resident(double2 (&r)[N], const double (&col)[NP], double sgn) {
  static_for<0, 2 * N>([&](auto dc) {
    constexpr int d = decltype(dc)::value;
    if constexpr (d & 1)
      dpp_fmac<d & 15>(r[d >> 1].y, col[d >> 4], sgn);
    else
      dpp_fmac<d & 15>(r[d >> 1].x, col[d >> 4], sgn);
  });
}

// r += s * U from LDS (wave-uniform address, per-lane s): one rounding.
// Rows go in groups of 8 so that at most 8 loaded entries are live at once.
template <int N>
__device__ __forceinline__ void fma_lds(double2 (&r)[N], double s, const double2* col) {
  static_for<0, (N + 7) / 8>([&](auto gc) {
    constexpr int g = decltype(gc)::value;
#pragma unroll
    for (int i = 8 * g; i < (8 * g + 8 < N ? 8 * g + 8 : N); ++i) {
      const double2 v = col[i];
      r[i].x = fma(s, v.x, r[i].x);
      r[i].y = fma(s, v.y, r[i].y);
    }
    __builtin_amdgcn_sched_barrier(0);
  });
}

// sb += (+-) prod_i r_i.  K independent product chains (rows k, k+K, ...) give
// instruction-level parallelism; the last complex multiply is fused into the
// accumulation (4 FMAs).  n = 44 takes three chains: the fourth chain's
// registers hold the staged update column of the one-matrix sweep.
template <int N>
__device__ __forceinline__ void term(const double2 (&r)[N], double2& sb, bool neg) {
  constexpr int K = N < 4 ? N : (N == 44 ? 3 : 4);
  double2 ch[K];
#pragma unroll
  for (int k = 0; k < K; ++k) ch[k] = r[k];
#pragma unroll
  for (int i = K; i < N; ++i) ch[i % K] = cmul(ch[i % K], r[i]);
  if constexpr (K == 1) {
    sb.x += neg ? -ch[0].x : ch[0].x;
    sb.y += neg ? -ch[0].y : ch[0].y;
  } else {
    double2 x, y;
    if constexpr (K == 2) {
      x = ch[0];
      y = ch[1];
    } else if constexpr (K == 3) {
      x = cmul(ch[0], ch[1]);
      y = ch[2];
    } else {
      x = cmul(ch[0], ch[1]);
      y = cmul(ch[2], ch[3]);
    }
    if (neg) {
      x.x = -x.x;
      x.y = -x.y;
    }
    sb.x = fma(x.x, y.x, sb.x);
    sb.x = fma(-x.y, y.y, sb.x);
    sb.y = fma(x.x, y.y, sb.y);
    sb.y = fma(x.y, y.x, sb.y);
  }
}

// Row sums at the Gray word of index k0, from scratch, columns in order:
//   BB/FG  r_i = a_i0 + sum_{j>=1} delta_j a_ij   (delta_j a_ij = (-delta_j/2) T[j]_i, exact)
//   Ryser  r_i = sum_j [j in S] a_ij
// over the table's ncols columns (N for a square matrix).
template <int N, int ALGO>
__device__ __forceinline__ void seed(double2 (&r)[N], uint64_t k0, const double2* T, int ncols) {
  const uint64_t g = k0 ^ (k0 >> 1);
  if constexpr (ALGO == ALGO_GLYNN) {
#pragma unroll
    for (int i = 0; i < N; ++i) r[i] = T[i];
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) r[i] = make_double2(0.0, 0.0);
  }
#pragma unroll 1
  for (int j = (ALGO == ALGO_GLYNN ? 1 : 0); j < ncols; ++j) {
    const int bit = ALGO == ALGO_GLYNN ? j - 1 : j;
    const bool set = (g >> bit) & 1;
    const double w = ALGO == ALGO_GLYNN ? (set ? 0.5 : -0.5) : (set ? 1.0 : 0.0);
    fma_lds<N>(r, w, T + j * N);
  }
}

__device__ __forceinline__ void flush(dd2& acc, double2& sb, bool plain, bool active) {
  if (active) {
    if (plain) {
      acc.hr += sb.x;
      acc.hi += sb.y;
    } else {
      dd_accumulate(acc, sb.x, sb.y);
    }
  }
  sb = make_double2(0.0, 0.0);
}

// Per-wave sweep state: the DPP-resident update columns (DR of them; a
// caller with more live state of its own may ask for fewer than Shape::D).
template <int N, int ALGO, int DR = Shape<N, ALGO>::D>
struct Resident {
  using S = Shape<N, ALGO>;
  static_assert(DR <= S::D, "resident columns exceed the register budget");
  static constexpr int D = DR;
  double col[DR > 0 ? DR : 1][S::NP];

  // Load from the LDS table (after the block barrier).
  __device__ __forceinline__ void load(const double2* T) {
    const int l16 = threadIdx.x & 15;
#pragma unroll
    for (int b = 0; b < DR; ++b) {
      const double* c = reinterpret_cast<const double*>(T + (b + S::OFF) * N);
#pragma unroll
      for (int p = 0; p < S::NP; ++p) {
        const int d = p * 16 + l16;
        col[b][p] = d < 2 * N ? c[d] : 0.0;
      }
    }
  }
};

// Update column b in the lane-distributed layout of Resident::col, read from
// the LDS table.  A staged sweep fills one such buffer several steps before
// the step that flips bit b, so that step is a DPP update like a resident
// column's instead of a wave-uniform LDS read per row at the step itself.
template <int N, int ALGO, int NP>
__device__ __forceinline__ void stage_column(double (&x)[NP], const double2* T, int b) {
  using S = Shape<N, ALGO>;
  static_assert(NP == S::NP, "staged column of the resident layout");
  const int l16 = threadIdx.x & 15;
  const double* c = reinterpret_cast<const double*>(T + (b + S::OFF) * N);
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    // an in-range read on every lane (no branch in the sweep); lanes past the
    // column's 2N doubles are never broadcast by add_resident
    const int d = p * 16 + l16;
    x[p] = c[d < 2 * N ? d : 2 * N - 1];
  }
}

// The next step offset s' > s of an unrolled block of 2^LOGU steps whose
// flipped bit ctz(s') is not resident (>= DR); 0 if there is none.
template <int LOGU, int DR>
constexpr int next_staged(int s) {
  for (int t = s + 1; t < (1 << LOGU); ++t)
    if (__builtin_ctz(t) >= DR) return t;
  return 0;
}

// One lane sweeps the chunk [k0, k0 + 2^c) and folds it into acc.
// Requires LOGU <= c <= nb (c == 0 only when the formula has a single term);
// nb follows from the table's ncols columns (N for a square matrix).
// STAGE: the steps that flip a non-resident bit (and the block boundaries)
// take their column from one staged buffer (stage_column), refilled right
// after each use with the next such step's column.
template <int N, int ALGO, int DR, bool STAGE = false>
__device__ __forceinline__ void sweep_chunk(uint64_t k0, int c, const Resident<N, ALGO, DR>& res, const double2* T,
                                            dd2& acc, bool plain, bool active, int ncols = N) {
  using S = Shape<N, ALGO>;
  constexpr int LOGU = S::LOGU;
  constexpr int U = 1 << LOGU;
  double2 r[N];
  seed<N, ALGO>(r, k0, T, ncols);
  double2 sb = make_double2(0.0, 0.0);
  term<N>(r, sb, (k0 & 1) != 0);  // offset 0
  if constexpr (LOGU == 0) {
    flush(acc, sb, plain, active);
  } else {
    const double one = 1.0, mone = -1.0;
    const uint32_t nblk = 1u << (c - LOGU);
    constexpr int S1 = next_staged<LOGU, DR>(0);  // first staged step of a block
    // a staged load with no step left to use it reads table column 0 (present
    // in every table, even one of fewer columns than rows)
    constexpr int UNUSED = -S::OFF;
    double xs[S::NP];
    if constexpr (STAGE) {
      if constexpr (S1 != 0)
        stage_column<N, ALGO>(xs, T, __builtin_ctz(S1));
      else
        stage_column<N, ALGO>(xs, T, nblk > 1 ? LOGU : UNUSED);
    }
    for (uint32_t m = 0; m < nblk; ++m) {
      const uint32_t tb = m << LOGU;
      static_for<1, U>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        constexpr int b = __builtin_ctz(s);
        double sg;
        if constexpr (b + 1 < LOGU) {
          sg = (((s >> (b + 1)) & 1) == 0) ? one : mone;
        } else {
          // s = U/2: the next bit is bit 0 of the block index, or the chunk
          // parity when the chunk is a single block (then it differs by lane).
          const uint64_t k = k0 + tb + s;
          sg = ((k >> (b + 1)) & 1) ? mone : one;
        }
        if constexpr (b < DR) {
          add_resident<N, S::NP>(r, res.col[b], sg);
        } else if constexpr (STAGE) {
          add_resident<N, S::NP>(r, xs, sg);
          constexpr int sn = next_staged<LOGU, DR>(s);
          if constexpr (sn != 0)
            stage_column<N, ALGO>(xs, T, __builtin_ctz(sn));
          else  // this block's boundary column
            stage_column<N, ALGO>(xs, T, m + 1 < nblk ? LOGU + __builtin_ctz(m + 1) : UNUSED);
        } else {
          fma_lds<N>(r, sg, T + (b + S::OFF) * N);
        }
        term<N>(r, sb, (s & 1) != 0);
        // keep steps apart: overlapping the next update with this product
        // would need two copies of the row sums in registers
        __builtin_amdgcn_sched_barrier(0);
      });
      if (m + 1 < nblk) {
        // block boundary: offset t = (m+1) U flips bit LOGU + ctz(m+1)
        const int b = LOGU + __builtin_ctz(m + 1);
        const uint64_t k = k0 + tb + U;
        const double sgb = ((k >> (b + 1)) & 1) ? -1.0 : 1.0;
        if constexpr (STAGE) {
          add_resident<N, S::NP>(r, xs, sgb);
          if constexpr (S1 != 0)
            stage_column<N, ALGO>(xs, T, __builtin_ctz(S1));
          else
            stage_column<N, ALGO>(xs, T, m + 2 < nblk ? LOGU + __builtin_ctz(m + 2) : UNUSED);
        } else {
          fma_lds<N>(r, sgb, T + (b + S::OFF) * N);
        }
        term<N>(r, sb, false);
      }
      flush(acc, sb, plain, active);
    }
  }
}

__device__ __forceinline__ dd2 wave_reduce(dd2 a, bool plain) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    dd2 o;
    o.hr = __shfl_xor(a.hr, off, 64);
    o.lr = __shfl_xor(a.lr, off, 64);
    o.hi = __shfl_xor(a.hi, off, 64);
    o.li = __shfl_xor(a.li, off, 64);
    if (plain) {
      a.hr += o.hr;
      a.hi += o.hi;
    } else {
      a = dd_add(a, o);
    }
  }
  return a;
}

// Entry (i, j) of the table the sweep reads, from A (row-major, leading
// dimension lda):
//   BB/FG  T[0] = a_{.,0},  T[j] = -2 a_{.,j} (j >= 1)
//   Ryser  T[j] = a_{.,j}
// Scaling by -2 is exact, so the Gray step r_i += 2 delta_c(new) a_ic of
// Eq. (S2) is one correctly rounded add per component.
__device__ __forceinline__ double2 table_entry(const double2* __restrict__ a, int64_t lda, int algo, int i, int j) {
  const double2 v = a[(int64_t)i * lda + j];
  return (algo == ALGO_GLYNN && j >= 1) ? make_double2(-2.0 * v.x, -2.0 * v.y) : v;
}

// Stage the n x n table into LDS straight from A, column-major (column j is
// N contiguous entries); block-cooperative.
template <int N, int ALGO>
__device__ __forceinline__ void stage_table(double2* lds, const double2* __restrict__ a, int64_t lda) {
  for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
    const int i = e / N, j = e % N;  // row-major reads
    lds[j * N + i] = table_entry(a, lda, ALGO, i, j);
  }
  __syncthreads();
}

}  // namespace ph
