// Two lanes per term, for the orders whose n row sums no longer fit one
// lane's registers next to the update columns (the one-matrix sweep from
// n = PAIR_NMIN on), and for small sweeps that need more lanes than chunks.
//
// Lane l and lane l + 32 of a wavefront walk the same chunk.  The lower lane
// owns rows 0..R-1 and the upper lane rows R..2R-1, R = ceil(n/2); for odd n
// the last row of the upper half is padding whose row sum stays 1.  Each lane
// forms the product of its R row sums; one v_permlane32_swap per dword brings
// the upper lane's product to the lower lane, whose complex product of the two
// is the term of Eq. (S1) or (S2).  Only the lower lane accumulates it.
//
// Every 16-lane DPP row lies in one half, so the low update columns stay
// resident in VGPRs (row_newbcast), as in the one-lane sweep: each lane's row
// of 16 holds the 2R doubles of its own half of the column.
//
// Table (LDS): the n-column table of sweep.hpp with column stride 2R, rows
// N..2R-1 padded: a_{pad,0} = 1 (BB/FG), every other padded entry 0.  The
// Ryser seed sets the padded row sum to 1 itself.
#pragma once
#include "ph_internal.hpp"
#include "sweep.hpp"

namespace ph {

template <int N, int ALGO>
struct PairShape {
  static constexpr int R = (N + 1) / 2;  // rows per lane
  static constexpr int RS = 2 * R;       // column stride of the padded table
  static constexpr int NB = Shape<N, ALGO>::NB;
  static constexpr int OFF = Shape<N, ALGO>::OFF;
  static constexpr int LOGU = Shape<N, ALGO>::LOGU;
  static constexpr int D = LOGU < 4 ? LOGU : 4;  // resident update columns
  static constexpr int NP = (2 * R + 15) / 16;   // VGPR pairs per resident column
};

template <int N, int ALGO>
__device__ __forceinline__ void stage_table_pair(double2* lds, const double2* __restrict__ a, int64_t lda) {
  using P = PairShape<N, ALGO>;
  for (int e = threadIdx.x; e < N * P::RS; e += blockDim.x) {
    const int j = e / P::RS, q = e % P::RS;
    double2 v = make_double2(0.0, 0.0);
    if (q < N) v = table_entry(a, lda, ALGO, q, j);
    else if (ALGO == ALGO_GLYNN && j == 0) v = make_double2(1.0, 0.0);
    lds[e] = v;
  }
  __syncthreads();
}

template <int N, int ALGO>
struct ResidentPair {
  using P = PairShape<N, ALGO>;
  double col[P::D > 0 ? P::D : 1][P::NP];

  // Tl: this lane's half of the table (column j at Tl + j * RS).
  __device__ __forceinline__ void load(const double2* Tl) {
    const int l16 = threadIdx.x & 15;
#pragma unroll
    for (int b = 0; b < P::D; ++b) {
      const double* c = reinterpret_cast<const double*>(Tl + (b + P::OFF) * P::RS);
#pragma unroll
      for (int p = 0; p < P::NP; ++p) {
        const int d = p * 16 + l16;
        col[b][p] = d < 2 * P::R ? c[d] : 0.0;
      }
    }
  }
};

// This lane's half of update column b in the ResidentPair layout, read from
// the LDS table (stage_column's counterpart): an in-range read on every lane;
// lanes past the half's 2R doubles are never broadcast.
template <int N, int ALGO, int NP>
__device__ __forceinline__ void stage_column_pair(double (&x)[NP], const double2* Tl, int b) {
  using P = PairShape<N, ALGO>;
  static_assert(NP == P::NP, "staged column of the resident layout");
  const int l16 = threadIdx.x & 15;
  const double* c = reinterpret_cast<const double*>(Tl + (b + P::OFF) * P::RS);
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int d = p * 16 + l16;
    x[p] = c[d < 2 * P::R ? d : 2 * P::R - 1];
  }
}

// Row sums of this lane's half at the Gray word of k0 (as seed()).
template <int N, int ALGO, int R>
__device__ __forceinline__ void seed_pair(double2 (&r)[R], uint64_t k0, const double2* Tl, bool upper) {
  using P = PairShape<N, ALGO>;
  static_assert(R == P::R, "rows per lane");
  const uint64_t g = k0 ^ (k0 >> 1);
  if constexpr (ALGO == ALGO_GLYNN) {
#pragma unroll
    for (int i = 0; i < P::R; ++i) r[i] = Tl[i];
  } else {
#pragma unroll
    for (int i = 0; i < P::R; ++i) r[i] = make_double2(0.0, 0.0);
  }
#pragma unroll 1
  for (int j = (ALGO == ALGO_GLYNN ? 1 : 0); j < N; ++j) {
    const int bit = ALGO == ALGO_GLYNN ? j - 1 : j;
    const bool set = (g >> bit) & 1;
    const double w = ALGO == ALGO_GLYNN ? (set ? 0.5 : -0.5) : (set ? 1.0 : 0.0);
    fma_lds<P::R>(r, w, Tl + j * P::RS);
  }
  if constexpr (ALGO == ALGO_RYSER && (N & 1)) {
    if (upper) r[P::R - 1] = make_double2(1.0, 0.0);
  }
}

// On a lower lane l: x keeps its value and `from` receives x of lane l + 32.
// (v_permlane32_swap exchanges the upper half of its first operand with the
// lower half of its second; `from` enters with a dead value, the previous
// term's, so no copy is needed.  On upper lanes both results are unused.)
__device__ __forceinline__ void from_upper(double& x, double& from) {
  const unsigned xl = (unsigned)__double2loint(x), xh = (unsigned)__double2hiint(x);
  const unsigned fl = (unsigned)__double2loint(from), fh = (unsigned)__double2hiint(from);
  const auto pl = __builtin_amdgcn_permlane32_swap(xl, fl, false, false);
  const auto ph = __builtin_amdgcn_permlane32_swap(xh, fh, false, false);
  x = __hiloint2double((int)ph[0], (int)pl[0]);
  from = __hiloint2double((int)ph[1], (int)pl[1]);
}

// On lower lanes: sb += (+-) (product of the lower half's rows) * (product of
// the upper half's).  `up` carries the received product from term to term.
template <int R>
__device__ __forceinline__ void term_pair(const double2 (&r)[R], double2& sb, double2& up, bool neg) {
  constexpr int K = R < 4 ? R : 4;
  double2 ch[K];
#pragma unroll
  for (int k = 0; k < K; ++k) ch[k] = r[k];
#pragma unroll
  for (int i = K; i < R; ++i) ch[i % K] = cmul(ch[i % K], r[i]);
  double2 x = ch[0];
  if constexpr (K == 2) x = cmul(ch[0], ch[1]);
  if constexpr (K == 3) x = cmul(cmul(ch[0], ch[1]), ch[2]);
  if constexpr (K == 4) x = cmul(cmul(ch[0], ch[1]), cmul(ch[2], ch[3]));
  double2 lo = x;
  from_upper(lo.x, up.x);
  from_upper(lo.y, up.y);
  if (neg) {
    lo.x = -lo.x;
    lo.y = -lo.y;
  }
  sb.x = fma(lo.x, up.x, sb.x);
  sb.x = fma(-lo.y, up.y, sb.x);
  sb.y = fma(lo.x, up.y, sb.y);
  sb.y = fma(lo.y, up.x, sb.y);
}

// The pair of lanes sweeps the chunk [k0, k0 + 2^c); `active` folds it into
// acc (true on the lower lane of an in-range chunk only).  STAGE: each block
// boundary's column comes from a staged buffer filled right after the
// previous boundary (every other step's column is resident).
template <int N, int ALGO, bool STAGE = false>
__device__ __forceinline__ void sweep_chunk_pair(uint64_t k0, int c, const ResidentPair<N, ALGO>& res,
                                                 const double2* Tl, bool upper, dd2& acc, bool plain, bool active) {
  using P = PairShape<N, ALGO>;
  constexpr int R = P::R, LOGU = P::LOGU, U = 1 << LOGU;
  static_assert(LOGU == 4, "the pair sweep is for large orders");
  double2 r[R];
  seed_pair<N, ALGO>(r, k0, Tl, upper);
  double2 sb = make_double2(0.0, 0.0), up = make_double2(0.0, 0.0);
  const double one = 1.0, mone = -1.0;
  const uint32_t nblk = 1u << (c - LOGU);
  static_assert(!STAGE || P::D == LOGU, "staging covers the block boundaries only");
  double xs[P::NP];
  // block 0's boundary flips bit LOGU; with no boundary in the chunk the load
  // reads table column 0 and goes unused
  if constexpr (STAGE) stage_column_pair<N, ALGO>(xs, Tl, nblk > 1 ? LOGU : -P::OFF);
  term_pair<R>(r, sb, up, (k0 & 1) != 0);  // offset 0
  for (uint32_t m = 0; m < nblk; ++m) {
    const uint32_t tb = m << LOGU;
    static_for<1, U>([&](auto sc) {
      constexpr int s = decltype(sc)::value;
      constexpr int b = __builtin_ctz(s);
      double sg;
      if constexpr (b + 1 < LOGU) {
        sg = (((s >> (b + 1)) & 1) == 0) ? one : mone;
      } else {
        const uint64_t k = k0 + tb + s;
        sg = ((k >> (b + 1)) & 1) ? mone : one;
      }
      if constexpr (b < P::D)
        add_resident<R, P::NP>(r, res.col[b], sg);
      else
        fma_lds<R>(r, sg, Tl + (b + P::OFF) * P::RS);
      term_pair<R>(r, sb, up, (s & 1) != 0);
      __builtin_amdgcn_sched_barrier(0);
    });
    if (m + 1 < nblk) {
      const int b = LOGU + __builtin_ctz(m + 1);
      const uint64_t k = k0 + tb + U;
      const double sgb = ((k >> (b + 1)) & 1) ? -1.0 : 1.0;
      if constexpr (STAGE) {
        add_resident<R, P::NP>(r, xs, sgb);
        // the next block's boundary column (column 0, unused, after the last)
        stage_column_pair<N, ALGO>(xs, Tl, m + 2 < nblk ? LOGU + __builtin_ctz(m + 2) : -P::OFF);
      } else {
        fma_lds<R>(r, sgb, Tl + (b + P::OFF) * P::RS);
      }
      term_pair<R>(r, sb, up, false);
    }
    flush(acc, sb, plain, active);
  }
}

}  // namespace ph
