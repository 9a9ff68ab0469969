// Gradient of the permanent in one Gray-code sweep (gfx950).
//
// Differentiating the BB/FG formula, Eq. (S2), term by term:
//   M_ij = d Per / d a_ij = 2^-(n-1) sum_delta (prod_k delta_k) delta_j q_i(delta),
//   q_i  = prod_{k != i} r_k,   r_k = sum_j delta_j a_kj,
// and M_ij is the permanent of A without row i and column j.  The sweep walks
// delta in Gray order exactly like the forward kernels (sweep.hpp); what is
// new is (1) the leave-one-out products q_i and (2) collecting
// w_i(t) = s_t q_i(t) into all n columns without O(n^2) work per term.
//
// (1) A term is split over a group of H lanes (H = 4 or 8); lane `sigma` of
//     the group owns rows [sigma*M, sigma*M + M).  Each lane forms the suffix
//     products of its rows, the group exchanges partial products with DPP
//     lane permutes (quad xor 1, xor 2, then the half-row mirror for H = 8)
//     to get O = the product of the other lanes' rows, and a running prefix
//     started from s_t O yields s_t q_i for its rows, the last multiply fused
//     into the accumulation.  Splitting the rows keeps the per-lane state
//     (row sums, running sums, stored columns) in the register file.
//
// (2) Summation by parts.  In a chunk of L = 2^c terms with running sum
//     W(t) = sum_{tau <= t} w(tau),
//        sum_t delta_j(t) w(t) = delta_j(L-1) W(L-1) - 2 sum_{flips of j at t} delta_j(t) W(t-1),
//     so each step touches only the column whose delta flips.  The K columns
//     that flip most often (Gray bits 0..K-1, used by 1 - 2^-K of all steps)
//     are accumulated per lane in registers; a flip of any other column, and
//     the boundary term of every column at the chunk end, is summed over the
//     64/H groups of the wavefront (a reduce-scatter across lanes, in
//     registers) and added into the wavefront's n x ROWS
//     accumulator in global memory.  Every address of that accumulator is read
//     and written by one fixed lane only, so program order is the only
//     ordering needed.
//
// The loop takes the terms in blocks of 2^K: inside a block the steps flip
// Gray bits 0..K-1 in a fixed pattern, so the stored-column updates, the
// signs and the column addresses are compile-time constants (straight-line
// code, no branch); the step into a block flips bit K + ctz(block index), the
// same on every lane, and only that step branches (on the scalar bit index)
// between a register-held group sum and one added to memory.
//
// The permanent itself is the expansion of the same sweep along row 0:
// Eq. (S2) is linear in each row, so sum_delta (prod delta) prod_i r_i =
// sum_j a_0j Mhat_0j with Mhat the sweep's unscaled sums; the finalize forms
// it from the table's row 0 and M's row 0 in double-double.  All sums are in
// a fixed order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <utility>

#include "dd.hpp"
#include "permhip.h"
#include "ph_host.hpp"
#include "ph_internal.hpp"
#include "sweep.hpp"

namespace ph {

// lane permutes of a double: lane ^ 1, lane ^ 2 within each quad, and the
// mirror within each half row of 8 lanes (lane i <-> 7 - i)
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false),
                          __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double2 dpp_mov(double2 v) {
  return make_double2(dpp_mov<CTRL>(v.x), dpp_mov<CTRL>(v.y));
}
constexpr int DPP_QUAD_XOR1 = 0xB1, DPP_QUAD_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141;

// One halving step of a reduce-scatter across lane bit B, for a pair of
// values (x, y) held by every lane: the lanes on one side of bit B return
// x + (partner's x), the others y + (partner's y).
//  * B = 5, 4: v_permlane32_swap / v_permlane16_swap exchange the upper half
//    (odd rows) of one operand with the lower half (even rows) of the other,
//    so after the swap each lane holds its own value of the component its
//    side keeps and its partner's, whichever operand order the hardware
//    takes: the sum of the two results.
//  * B = 3, 2: two bank-masked DPP moves within each 16-lane row (a bank is
//    4 lanes; masked-off lanes keep the old value): the lanes with bit B
//    clear read x from lane + 2^B (row_ror 8 or 12), the others y from
//    lane - 2^B (row_ror 8 or 4).
template <int B>
__device__ __forceinline__ double pair_sum(double x, double y) {
  if constexpr (B >= 4) {
    const unsigned xl = (unsigned)__double2loint(x), xh = (unsigned)__double2hiint(x);
    const unsigned yl = (unsigned)__double2loint(y), yh = (unsigned)__double2hiint(y);
    if constexpr (B == 5) {
      const auto l = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
      const auto h = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
      return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
    } else {
      const auto l = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
      const auto h = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
      return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
    }
  } else {
    constexpr int UP = B == 3 ? 0x128 : 0x12C, DOWN = B == 3 ? 0x128 : 0x124;  // row_ror 8 / 12 / 4
    constexpr int CLEAR = B == 3 ? 0x3 : 0x5, SET = B == 3 ? 0xC : 0xA;         // banks by bit B
    const int xl = __double2loint(x), xh = __double2hiint(x);
    const int yl = __double2loint(y), yh = __double2hiint(y);
    // bit clear: partner's x (others keep y); bit set: partner's y (others keep x)
    const double a = __hiloint2double(__builtin_amdgcn_update_dpp(yh, xh, UP, 0xF, CLEAR, false),
                                      __builtin_amdgcn_update_dpp(yl, xl, UP, 0xF, CLEAR, false));
    const double b = __hiloint2double(__builtin_amdgcn_update_dpp(xh, yh, DOWN, 0xF, SET, false),
                                      __builtin_amdgcn_update_dpp(xl, yl, DOWN, 0xF, SET, false));
    return a + b;
  }
}

// Reduce-scatter of C values per lane over lane bits B, B-1, ..., BLAST:
// each step pairs value i with value i + ceil(C/2) (an unpaired middle value
// with zero) and halves the count, so that every (lane mod 2^BLAST, value)
// ends summed on exactly one lane; the other lanes end with 0.
template <int C, int B, int BLAST, int CMAX>
__device__ __forceinline__ double reduce_scatter(double (&v)[CMAX]) {
  constexpr int HALF = (C + 1) / 2;
  static_for<0, C / 2>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    v[i] = pair_sum<B>(v[i], v[i + HALF]);
  });
  if constexpr (C & 1) v[HALF - 1] = pair_sum<B>(v[HALF - 1], 0.0);
  if constexpr (B == BLAST) {
    static_assert(HALF == 1, "more values than the lane bits can spread");
    return v[0];
  } else {
    return reduce_scatter<HALF, B - 1, BLAST>(v);
  }
}

// Stored columns (K) and target wavefronts per SIMD per (rows per lane M,
// lanes per term H).
#ifndef PH_GRAD_K
#define PH_GRAD_K(M, H) ((H) == 8 ? 5 : ((M) == 1 ? 1 : ((M) <= 4 ? 2 : 5)))
#endif
#ifndef PH_GRAD_WAVES
#define PH_GRAD_WAVES(M, H) ((H) == 8 ? ((M) <= 2 ? 3 : 2) : ((M) <= 1 ? 4 : ((M) <= 3 ? 3 : 2)))
#endif
// which orders split a term over 4 lanes (the others over 8); the 4-lane
// layouts with 3 and 4 rows per lane are compiled only if some order uses them
#ifndef PH_GRAD_USE_H4
#define PH_GRAD_USE_H4(n) ((n) <= 8 || ((n) >= 17 && (n) <= 20))
#endif
#ifndef PH_GRAD_H4_M3
#define PH_GRAD_H4_M3 0
#endif
#ifndef PH_GRAD_H4_M4
#define PH_GRAD_H4_M4 0
#endif
// stored columns whose entries each lane also keeps in registers (the
// others are read from LDS when they flip)
#ifndef PH_GRAD_KR
#define PH_GRAD_KR(M, H) ((M) <= 2 ? 4 : ((M) == 3 ? 2 : 1))
#endif

template <int M, int H>
struct GradShape {
  static constexpr int K = PH_GRAD_K(M, H);
  static constexpr int ROWS = H * M;  // padded rows of the table
  static constexpr int NG = 64 / H;   // term groups per wavefront
  // Gray bits K..K+R-1 (the boundary columns flipped most often) collect
  // their group sums in registers of the owning lane
  static constexpr int R = 4;
  static constexpr int WAVES = PH_GRAD_WAVES(M, H);
  static constexpr int KR = PH_GRAD_KR(M, H) < K ? PH_GRAD_KR(M, H) : K;
};

struct GradArgs {
  const double2* tabs;  // per matrix: ncols columns x ROWS rows (zero padded)
  int n, c;
  int ncols;            // columns the sweep walks (n for a square matrix)
  int64_t nsuper;       // super-chunks per matrix (64/H chunks each)
  int s_per;            // units (slices) per matrix
  int64_t units;        // batch * s_per
  uint32_t* counter;
  double2* ghat;        // per (unit, wave): n x ROWS complex
};

template <int M, int H>
struct GradLane {
  double2 r[M];
  double2 W[M];
  double2 G[GradShape<M, H>::K][M];
  double2 colK[GradShape<M, H>::KR][M];  // the lane's rows of columns 1..KR
  double2 colv[M];                       // the next LDS-sourced step's column, read ahead
};

// Group sums: wt * W summed over the NG groups, for each lane position in the
// group and each of its rows, into an accumulator column of 2 ROWS doubles
// (row r's real part at 2r, imaginary at 2r + 1).  The 2M components of a
// lane (value j: row h M + j / 2 of lane position h, real part if j is even)
// are reduce-scattered over the lane bits above log2 H, so each entry ends on
// one lane, the one for which group_slot gives its index; the other lanes
// have slot -1.  wt may differ between groups (the chunk-end terms take each
// chunk's own signs), so it scales every lane's values before they are summed.
template <int H>
constexpr int log2_lanes() { return H == 4 ? 2 : 3; }
template <int M, int H>
__device__ __forceinline__ double group_sum(const double2 (&W)[M], double wt) {
  double v[2 * M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    v[2 * i] = wt * W[i].x;
    v[2 * i + 1] = wt * W[i].y;
  }
  return reduce_scatter<2 * M, 5, log2_lanes<H>()>(v);
}
// The slot of each lane, found by running the same exchanges on tags: value j
// set to j + 1 on every lane sums to NG (j + 1) on the lane that receives
// value j and to 0 elsewhere (all 64 lanes must be active).
template <int M, int H>
__device__ __forceinline__ int group_slot(int lane) {
  double v[2 * M];
#pragma unroll
  for (int j = 0; j < 2 * M; ++j) v[j] = (double)(j + 1);
  const double s = reduce_scatter<2 * M, 5, log2_lanes<H>()>(v);
  const int j = (int)(s / (64 / H)) - 1;
  // only an exact tag names a slot, so no lane can write outside its column
  const bool ok = j >= 0 && j < 2 * M && s == (double)((64 / H) * (j + 1));
  return ok ? 2 * M * (lane % H) + j : -1;
}

// Adds a group sum into the wavefront's accumulator column (global memory,
// owned entry by entry by the lanes that compute them; slot from group_slot).
template <int M, int H>
__device__ __forceinline__ void group_sum_add(const double2 (&W)[M], double wt, double* gcol, int slot) {
  const double s = group_sum<M, H>(W, wt);
  if (slot >= 0) gcol[slot] += s;
}

// Product of the rows owned by the other H - 1 lanes of the group, from each
// lane's product of its own rows; NEG returns its negative (the sign folds
// into the last multiply).
template <int H, bool NEG>
__device__ __forceinline__ double2 others_product(double2 own) {
  const double2 p1 = dpp_mov<DPP_QUAD_XOR1>(own);  // partner lane
  const double2 pair = cmul(own, p1);
  const double2 pair2 = dpp_mov<DPP_QUAD_XOR2>(pair);  // the other pair of the quad
  const double2 p1s = NEG ? make_double2(-p1.x, -p1.y) : p1;
  if constexpr (H == 4) {
    return cmul(p1s, pair2);
  } else {
    const double2 quad = cmul(pair, pair2);
    const double2 quad2 = dpp_mov<DPP_HALF_MIRROR>(quad);  // the other quad of the 8
    return cmul(cmul(p1s, pair2), quad2);
  }
}

// One term: W_i += st q_i for the lane's rows (st = the term's sign, NEG
// when it is negative; with ACT, st also carries the group's 0/1 activity
// `act`).  Suffix products of the own rows, the group exchange for O, then a
// running prefix t_i = st O prod_{k<i} r_k with q_i st = t_i suf_{i+1}, the
// last multiply fused into the W update.
template <int M, int H, bool NEG, bool ACT>
__device__ __forceinline__ void grad_term(GradLane<M, H>& L, double act) {
  double2 suf[M];
  suf[M - 1] = L.r[M - 1];
#pragma unroll
  for (int ii = M - 2; ii >= 0; --ii) suf[ii] = cmul(L.r[ii], suf[ii + 1]);
  double2 t = others_product<H, NEG>(suf[0]);
  if constexpr (ACT) t = make_double2(act * t.x, act * t.y);
#pragma unroll
  for (int ii = 0; ii < M; ++ii) {
    if (ii < M - 1) {
      const double2 s1 = suf[ii + 1];
      L.W[ii].x = fma(t.x, s1.x, L.W[ii].x);
      L.W[ii].x = fma(-t.y, s1.y, L.W[ii].x);
      L.W[ii].y = fma(t.x, s1.y, L.W[ii].y);
      L.W[ii].y = fma(t.y, s1.x, L.W[ii].y);
      t = cmul(t, L.r[ii]);
    } else {
      L.W[ii].x += t.x;
      L.W[ii].y += t.y;
    }
  }
}

// f(integral_constant<B>) for the one B in [B0, E) equal to b (b must be in
// range), as an if-else chain on the scalar b
template <int B0, int E, typename F>
__device__ __forceinline__ void select_case(int b, F&& f) {
  if constexpr (B0 + 1 >= E) {
    f(std::integral_constant<int, B0>{});
  } else {
    if (b == B0)
      f(std::integral_constant<int, B0>{});
    else
      select_case<B0 + 1, E>(b, f);
  }
}

// r += s * v (own rows, values already in registers)
template <int M, int H>
__device__ __forceinline__ void grad_apply(GradLane<M, H>& L, double s, const double2 (&v)[M]) {
#pragma unroll
  for (int ii = 0; ii < M; ++ii) {
    L.r[ii].x = fma(s, v[ii].x, L.r[ii].x);
    L.r[ii].y = fma(s, v[ii].y, L.r[ii].y);
  }
}

// r += s * column (own rows, from LDS)
template <int M, int H>
__device__ __forceinline__ void grad_update(GradLane<M, H>& L, double s, const double2* col) {
#pragma unroll
  for (int ii = 0; ii < M; ++ii) {
    const double2 v = col[ii];
    L.r[ii].x = fma(s, v.x, L.r[ii].x);
    L.r[ii].y = fma(s, v.y, L.r[ii].y);
  }
}

// G_b += w * W (summation by parts of a stored column)
template <int M, int H>
__device__ __forceinline__ void stored_add(double2 (&G)[M], double w, const double2 (&W)[M]) {
#pragma unroll
  for (int ii = 0; ii < M; ++ii) {
    G[ii].x = fma(w, W[ii].x, G[ii].x);
    G[ii].y = fma(w, W[ii].y, G[ii].y);
  }
}

// ACT: some term groups of the launch walk past the last chunk (orders with
// fewer chunks than groups in a super-chunk); they run a copy of the sweep
// with every term scaled by 0.  Without ACT every group is active and the
// terms' signs are compile-time constants.
template <int M, int H, bool ACT>
__global__ __launch_bounds__(256, (GradShape<M, H>::WAVES)) void k_grad(GradArgs a) {
  using GS = GradShape<M, H>;
  constexpr int K = GS::K, ROWS = GS::ROWS, NG = GS::NG;
  extern __shared__ double lds[];
  double2* tab = reinterpret_cast<double2*>(lds);  // ncols * ROWS complex
  __shared__ int64_t s_unit;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sig = lane % H, grp = lane / H;
  const int n = a.n, nc = a.ncols, c = a.c, nb = nc - 1;
  const int row0 = sig * M;
  const int gidx = group_slot<M, H>(lane);  // accumulator entry this lane owns, or -1
  const bool out_lane = gidx >= 0;
  for (;;) {
    if (threadIdx.x == 0) s_unit = (int64_t)atomicAdd(a.counter, 1u);
    __syncthreads();
    const int64_t u = s_unit;
    if (u >= a.units) break;
    const int64_t mat = u / a.s_per, sl = u % a.s_per;
    const double2* gtab = a.tabs + (size_t)mat * nc * ROWS;
    for (int e = threadIdx.x; e < nc * ROWS; e += blockDim.x) tab[e] = gtab[e];
    __syncthreads();
    const int64_t slot = u * 4 + wave;
    double* ghat = reinterpret_cast<double*>(a.ghat + (size_t)slot * nc * ROWS);
    // each lane zeroes the accumulator entries it will own
    if (out_lane)
      for (int j = 0; j < nc; ++j) ghat[j * 2 * ROWS + gidx] = 0.0;
    GradLane<M, H> L;
#pragma unroll
    for (int b = 0; b < K; ++b)
#pragma unroll
      for (int ii = 0; ii < M; ++ii) {
        L.G[b][ii] = make_double2(0.0, 0.0);
        if (b < GS::KR) L.colK[b < GS::KR ? b : 0][ii] = tab[(b + 1) * ROWS + row0 + ii];
      }
    double bacc[GS::R];
#pragma unroll
    for (int q = 0; q < GS::R; ++q) bacc[q] = 0.0;
    const int64_t sb0 = a.nsuper * sl / a.s_per, sb1 = a.nsuper * (sl + 1) / a.s_per;
    const uint64_t nchunks = (uint64_t)1 << (nb - c);
    for (int64_t sc = sb0 + wave; sc < sb1; sc += 4) {
      const uint64_t chunk = (uint64_t)sc * NG + grp;
      const uint64_t k0 = chunk << c;
      // groups past the last chunk (tiny n) walk a copy but add nothing
      const double act = (!ACT || chunk < nchunks) ? 1.0 : 0.0;
      // seed own rows: r_i = a_i0 + sum_{j>=1} delta_j a_ij (delta_j a_ij = (-delta_j/2) T[j])
      const uint64_t g0 = k0 ^ (k0 >> 1);
#pragma unroll
      for (int ii = 0; ii < M; ++ii) L.r[ii] = tab[row0 + ii];
#pragma unroll 1
      for (int j = 1; j < nc; ++j) grad_update<M, H>(L, ((g0 >> (j - 1)) & 1) ? 0.5 : -0.5, tab + j * ROWS + row0);
#pragma unroll
      for (int ii = 0; ii < M; ++ii) {
        if (row0 + ii >= n) L.r[ii] = make_double2(1.0, 0.0);  // padding rows
        L.W[ii] = make_double2(0.0, 0.0);
      }
      // The step to offset t flips Gray bit b = ctz(t); its new value is set
      // iff bit b+1 of k = k0 + t is clear (k0 is a multiple of 2^c, so below
      // bit c that is bit b+1 of t, and bit c is the chunk's parity).
      //
      // Terms in blocks of 2^K: inside a block the steps flip Gray bits
      // 0..K-1 in a fixed pattern, so every stored-column update, sign and
      // column address is a compile-time constant (the columns of bits below
      // KR from registers, the others from LDS); only the step into a block
      // flips a bit >= K, chosen at run time.
      constexpr int NBK = 1 << K;
      const uint32_t nblk = 1u << (c - K);
      // Steps whose column is not held in registers (Gray bits >= KR inside a
      // block, and every block's first step) take it from colv, read from
      // LDS one step ahead: during the term before, whose step flips a
      // register-held bit (bit 0 at every odd offset), so the read has a
      // whole term to arrive.  The reads are volatile and followed by a
      // scheduling barrier so that the compiler keeps them there instead of
      // next to their use.
      static_assert(GS::KR >= 1, "every other step must take its column from registers");
      auto prefetch = [&](int col) __attribute__((always_inline)) {
        typedef const volatile __attribute__((address_space(3))) double lds_double;
        lds_double* cp = (lds_double*)(tab + col * ROWS + row0);
#pragma unroll
        for (int ii = 0; ii < M; ++ii) L.colv[ii] = make_double2(cp[2 * ii], cp[2 * ii + 1]);
        // (and the scheduler may not move them down past this point)
        __builtin_amdgcn_sched_barrier(0);
      };
      for (uint32_t m = 0; m < nblk; ++m) {
        const uint32_t tb = m << K;
        if (m != 0) {
          // step into the block: bit b = K + ctz(m) of column b + 1;
          // summation by parts adds -2 delta(t) W(t-1), delta(t) = -sgu
          const int bq = __builtin_ctz(m);
          const int b = K + bq;
          const double sgu = (((k0 + tb) >> (b + 1)) & 1) ? -1.0 : 1.0;
          if (bq < GS::R) {
            const double qs = group_sum<M, H>(L.W, 2.0 * sgu);
            // (the marker after the update keeps the cases apart)
            select_case<0, GS::R>(bq, [&](auto qc) {
              constexpr int q = decltype(qc)::value;
              bacc[q] += qs;
              asm volatile("; boundary column %0" ::"n"(q));
            });
          } else {
            group_sum_add<M, H>(L.W, 2.0 * sgu, ghat + (size_t)(b + 1) * 2 * ROWS, gidx);
          }
          grad_apply<M, H>(L, sgu, L.colv);
        }
        // the new value of bit K-1 (step 2^(K-1) of the block) comes from bit
        // K of k
        const double sg_top = (((k0 + tb) >> K) & 1) ? -1.0 : 1.0;
        static_for<0, NBK>([&](auto sc) {
          constexpr int so = decltype(sc)::value;
          constexpr int bb = __builtin_ctz(so | NBK);
          if constexpr (so != 0) {
            const double sgu = bb + 1 < K ? (((so >> (bb + 1)) & 1) ? -1.0 : 1.0) : sg_top;
            stored_add<M, H>(L.G[bb], 2.0 * sgu, L.W);
            if constexpr (bb < GS::KR)
              grad_apply<M, H>(L, sgu, L.colK[bb]);
            else
              grad_apply<M, H>(L, sgu, L.colv);
          }
          // the next step's column, if it comes from LDS
          constexpr int bn = __builtin_ctz((so + 1) | NBK);
          if constexpr (so + 1 < NBK) {
            if constexpr (bn >= GS::KR) prefetch(bn + 1);
          } else {
            // the next block's first step (any column after the chunk's last block)
            prefetch(m + 1 < nblk ? K + __builtin_ctz(m + 1) + 1 : 1);
          }
          grad_term<M, H, (so & 1) != 0, ACT>(L, act);
        });
      }
      // boundary terms delta_j(last) W(last) for every column
      const uint64_t kl = k0 + ((uint64_t)1 << c) - 1;
      const uint64_t gl = kl ^ (kl >> 1);
      group_sum_add<M, H>(L.W, 1.0, ghat, gidx);  // column 0: delta_0 = +1
#pragma unroll 1
      for (int j = K + 1; j < nc; ++j)
        group_sum_add<M, H>(L.W, ((gl >> (j - 1)) & 1) ? -1.0 : 1.0, ghat + (size_t)j * 2 * ROWS, gidx);
#pragma unroll
      for (int b = 0; b < K; ++b) stored_add<M, H>(L.G[b], ((gl >> b) & 1) ? -1.0 : 1.0, L.W);
    }
    // register-held boundary columns and stored columns into the accumulator
    if (out_lane) {
#pragma unroll
      for (int q = 0; q < GS::R; ++q)
        if (K + q + 1 < nc) ghat[(size_t)(K + q + 1) * 2 * ROWS + gidx] += bacc[q];
    }
#pragma unroll
    for (int b = 0; b < K; ++b)
      if (b + 1 < nc) group_sum_add<M, H>(L.G[b], 1.0, ghat + (size_t)(b + 1) * 2 * ROWS, gidx);
    __syncthreads();
  }
}

// Table for the gradient sweep: T[0] = a_{.,0}, T[j] = -2 a_{.,j}, each
// column padded to ROWS rows with zeros.
__global__ void k_grad_prep(const double2* __restrict__ a, int n, int rows, double2* __restrict__ tabs) {
  const int64_t mat = blockIdx.x;
  const double2* am = a + mat * n * n;
  double2* t = tabs + mat * n * rows;
  for (int e = threadIdx.x; e < n * rows; e += blockDim.x) {
    const int j = e / rows, i = e % rows;
    double2 v = make_double2(0.0, 0.0);
    if (i < n) {
      v = am[(int64_t)i * n + j];
      if (j >= 1) v = make_double2(-2.0 * v.x, -2.0 * v.y);
    }
    t[e] = v;
  }
}

// acc += a * m, a complex binary64, m a double-double per component: the
// products of the high parts are split exactly (FMA), the rest added plainly.
__device__ __forceinline__ void dd_cmul_acc(dd2& acc, double2 a, const dd2& m) {
  double s, e;
  const double p1 = a.x * m.hr, p2 = a.y * m.hi, p3 = a.x * m.hi, p4 = a.y * m.hr;
  const double lo_r = fma(a.x, m.hr, -p1) - fma(a.y, m.hi, -p2) + (a.x * m.lr - a.y * m.li);
  const double lo_i = fma(a.x, m.hi, -p3) + fma(a.y, m.hr, -p4) + (a.x * m.li + a.y * m.lr);
  two_sum(acc.hr, p1, s, e);
  acc.hr = s;
  acc.lr += e;
  two_sum(acc.hr, -p2, s, e);
  acc.hr = s;
  acc.lr += e + lo_r;
  two_sum(acc.hi, p3, s, e);
  acc.hi = s;
  acc.li += e;
  two_sum(acc.hi, p4, s, e);
  acc.hi = s;
  acc.li += e + lo_i;
}

// Per matrix: M = 2^-(n-1) sum over the (unit, wave) accumulators in order
// (n x ncols, row-major), grad = g * conj(M).  The permanent is the
// expansion of the same sum along row 0: Eq. (S2)'s sum is linear in each
// row, so sum_delta (prod delta) prod_i r_i = sum_j a_0j sum_delta
// (prod delta) delta_j q_0 = sum_j a_0j Mhat_0j, Mhat the unscaled sums
// (a_00 = T[0]_0, a_0j = -T[j]_0 / 2 from the table), added in j order.
__global__ void k_grad_finalize(const double2* __restrict__ ghat, const double2* __restrict__ tabs, int n,
                                int ncols, int rows, int s_per, int plain, const double2* __restrict__ gout,
                                double2* __restrict__ pout, double2* __restrict__ grad) {
  __shared__ dd2 row0[NMAX_GRAD];
  __shared__ double2 a0s[NMAX_GRAD];  // row 0 of the matrix, for the Laplace expansion
  const int64_t mat = blockIdx.x;
  const int64_t slots = (int64_t)s_per * 4, first = mat * slots;
  const double2 g = gout ? gout[mat] : make_double2(1.0, 0.0);
  // entries e = i ncols + j are spread over the gridDim.y workgroups of the
  // matrix; the first holds every entry of row 0 (e < ncols <= blockDim.x)
  // and adds the Laplace expansion along it
  const bool first_wg = blockIdx.y == 0;
  if (pout && first_wg) {
    const double2* t = tabs + (size_t)mat * ncols * rows;
    for (int j = threadIdx.x; j < ncols; j += blockDim.x) {
      double2 a0 = t[(size_t)j * rows];
      if (j >= 1) a0 = make_double2(-0.5 * a0.x, -0.5 * a0.y);  // exact
      a0s[j] = a0;
    }
  }
  for (int e = blockIdx.y * blockDim.x + threadIdx.x; e < n * ncols; e += blockDim.x * gridDim.y) {
    const int i = e / ncols, j = e % ncols;
    dd2 s = {0.0, 0.0, 0.0, 0.0};
    // the loads of U slots are issued before the first add (one memory round
    // trip per group); the adds keep the slot order
    constexpr int U = 8;
    for (int64_t q0 = 0; q0 < slots; q0 += U) {
      double2 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (q0 + u < slots) v[u] = ghat[(first + q0 + u) * ncols * rows + (size_t)j * rows + i];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (q0 + u >= slots) break;
        if (plain) {
          s.hr += v[u].x;
          s.hi += v[u].y;
        } else {
          dd_accumulate(s, v[u].x, v[u].y);
        }
      }
    }
    if (i == 0) row0[j] = s;
    const double mr = ldexp(s.hr, -(n - 1)) + ldexp(s.lr, -(n - 1));
    const double mi = ldexp(s.hi, -(n - 1)) + ldexp(s.li, -(n - 1));
    // g * conj(M)
    grad[mat * n * ncols + e] = make_double2(g.x * mr + g.y * mi, g.y * mr - g.x * mi);
  }
  if (pout && first_wg) {
    __syncthreads();
    if (threadIdx.x == 0) {
      dd2 acc = {0.0, 0.0, 0.0, 0.0};
      for (int j = 0; j < ncols; ++j) {
        const double2 a0 = a0s[j];
        const dd2 m = row0[j];
        if (plain) {
          acc.hr += a0.x * m.hr - a0.y * m.hi;
          acc.hi += a0.x * m.hi + a0.y * m.hr;
        } else {
          dd_cmul_acc(acc, a0, m);
        }
      }
      pout[mat] = make_double2(ldexp(acc.hr, -(n - 1)) + ldexp(acc.lr, -(n - 1)),
                               ldexp(acc.hi, -(n - 1)) + ldexp(acc.li, -(n - 1)));
    }
  }
}

// n = 1: M_00 = Per(empty) = 1, so grad = g, perm = a_00.
__global__ void k_grad_n1(const double2* __restrict__ a, int64_t batch, const double2* __restrict__ gout,
                          double2* __restrict__ pout, double2* __restrict__ grad) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b < batch) {
    grad[b] = gout ? gout[b] : make_double2(1.0, 0.0);
    if (pout) pout[b] = a[b];
  }
}

__global__ void k_reset1(uint32_t* c) { *c = 0; }

// Layout of one gradient sweep: lanes per term, rows per lane, its kernels
// (every group active; some groups past the last chunk).
struct GradLayout {
  int H, M, K;
  const void* kern;
  const void* kern_act;
};

template <int M, int H>
static GradLayout layout() {
  return GradLayout{H, M, GradShape<M, H>::K, (const void*)&k_grad<M, H, false>, (const void*)&k_grad<M, H, true>};
}

static GradLayout grad_layout(int n) {
  if (!PH_GRAD_USE_H4(n)) {
    switch ((n + 7) / 8) {
      case 2: return layout<2, 8>();
      case 3: return layout<3, 8>();
      case 4: return layout<4, 8>();
    }
    return GradLayout{0, 0, 0, nullptr, nullptr};
  }
  switch ((n + 3) / 4) {
    case 1: return layout<1, 4>();
    case 2: return layout<2, 4>();
#if PH_GRAD_H4_M3
    case 3: return layout<3, 4>();
#endif
#if PH_GRAD_H4_M4
    case 4: return layout<4, 4>();
#endif
    case 5: return layout<5, 4>();
  }
  return GradLayout{0, 0, 0, nullptr, nullptr};
}

int grad_rows(int n) {
  const GradLayout lay = grad_layout(n);
  return lay.H * lay.M;
}

// Fewest columns a gradient sweep of n rows walks: its blocks take 2^K terms,
// K = the stored columns of n's layout, so ncols - 1 >= K.
int grad_min_cols(int n) { return grad_layout(n).K + 1; }

// Gradient sweeps over prebuilt tables: `batch` tables of ncols columns x
// grad_rows(n) rows (T[0] = column 0, T[j] = -2 column j, rows >= n zero),
// packed back to back.  grad (n x ncols per matrix) = g * conj(M), pout the
// 2^-(n-1)-scaled sums.  5 <= ncols <= n unless ncols == n.
int grad_sweep(const double2* tabs, int n, int ncols, int64_t batch, const double2* gout, double2* pout,
               double2* grad, const Opts& o, hipStream_t st, int cus) {
  if (batch == 0) return PH_OK;
  const GradLayout lay = grad_layout(n);
  if (!lay.kern) return fail(PH_ERANGE, "no gradient kernel for n=%d", n);
  const int K = lay.K, rows = lay.H * lay.M, ng = 64 / lay.H, nb = ncols - 1;
  if (nb < K) return fail(PH_EINVAL, "gradient sweep over %d columns of %d rows", ncols, n);
  // chunk length: at most 2^12 terms with 4 lanes per term and 2^10 with 8,
  // and at least one chunk for each group of the four wavefronts of a unit
  // (4 * ng chunks) where the sweep is long enough.  Each chunk ends with group
  // sums over every column, which longer chunks amortise (n = 20: 5.46 ms per
  // 1024 matrices against 5.93 ms with 2^10).  The rounding of the running sums
  // grows with the chunk length: with 8 lanes per term 2^12 raised the Laplace
  // identity's error at n = 22 from 1.8e-12 to 1.4e-11, so those keep 2^10
  const int need = 2 + (ng == 8 ? 3 : 4);
  int c = o.chunk_log2 > 0 ? o.chunk_log2 : std::min(lay.H == 4 ? 12 : 10, nb - need);
  c = std::max(K, std::min(c, nb));  // a chunk holds whole blocks of 2^K terms
  const uint64_t nchunks = (uint64_t)1 << (nb - c);
  const int64_t nsuper = (int64_t)((nchunks + ng - 1) / ng);
  // a super-chunk holds ng chunks: groups past the last chunk need the kernel
  // that scales their terms by 0
  const void* kern = nchunks % ng == 0 ? lay.kern : lay.kern_act;
  const size_t lds = (size_t)ncols * rows * sizeof(double2);
  int per_cu = 0;
  int rc = resident_per_cu(kern, lds, &per_cu);
  if (rc) return rc;
  per_cu = std::max(1, per_cu);
  if (o.waves > 0) per_cu = std::min(per_cu, o.waves);
  const int64_t blocks_full = (int64_t)cus * per_cu;
  // slices per matrix: about four units per resident workgroup, at least one
  // super-chunk per wavefront of a unit
  int64_t s_per = std::max<int64_t>(1, (4 * blocks_full + batch - 1) / batch);
  s_per = std::min<int64_t>(s_per, std::max<int64_t>(1, nsuper / 4));
  const int64_t units = batch * s_per;
  const size_t ghat_elems = (size_t)units * 4 * ncols * rows;
  const size_t off_c = (((ghat_elems * sizeof(double2)) + 255) & ~(size_t)255);
  void* ws = nullptr;
  if ((rc = workspace(st, off_c + 256, &ws))) return rc;
  char* base = static_cast<char*>(ws);
  GradArgs ga;
  ga.tabs = tabs;
  ga.n = n;
  ga.ncols = ncols;
  ga.c = c;
  ga.nsuper = nsuper;
  ga.s_per = (int)s_per;
  ga.units = units;
  ga.counter = reinterpret_cast<uint32_t*>(base + off_c);
  ga.ghat = reinterpret_cast<double2*>(base);
  hipLaunchKernelGGL(k_reset1, dim3(1), dim3(1), 0, st, ga.counter);
  const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(blocks_full, units));
  void* args[] = {&ga};
  hipError_t e = hipLaunchKernel(kern, dim3((unsigned)grid), dim3(256), args, lds, st);
  if (e != hipSuccess) return hip_fail(e, "grad sweep launch");
  // one workgroup per 256 entries of a matrix's n x ncols gradient
  const unsigned fin_y = (unsigned)((n * ncols + 255) / 256);
  hipLaunchKernelGGL(k_grad_finalize, dim3((unsigned)batch, fin_y), dim3(256), 0, st, ga.ghat, tabs, n, ncols, rows,
                     (int)s_per, o.plain ? 1 : 0, gout, pout, grad);
  e = hipGetLastError();
  return e == hipSuccess ? PH_OK : hip_fail(e, "grad launch");
}

// Enqueue the gradient of `batch` n x n matrices (device pointers).
int perm_grad_launch(const double2* A, int n, int64_t batch, const double2* gout, double2* pout, double2* grad,
                     const Opts& o, hipStream_t st, int cus) {
  if (batch == 0) return PH_OK;
  if (n == 1) {
    hipLaunchKernelGGL(k_grad_n1, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, st, A, batch, gout, pout,
                       grad);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? PH_OK : hip_fail(e, "grad launch");
  }
  const int rows = grad_rows(n);
  if (rows <= 0) return fail(PH_ERANGE, "no gradient kernel for n=%d", n);
  // the tables in a workspace slot of their own: the sweep may grow WS_SWEEP
  void* tw = nullptr;
  int rc = workspace_slot(st, (size_t)batch * n * rows * sizeof(double2), WS_GRAD_TABLES, &tw);
  if (rc) return rc;
  double2* tabs = static_cast<double2*>(tw);
  hipLaunchKernelGGL(k_grad_prep, dim3((unsigned)batch), dim3(256), 0, st, A, n, rows, tabs);
  return grad_sweep(tabs, n, n, batch, gout, pout, grad, o, st, cus);
}

}  // namespace ph

using namespace ph;

extern "C" int ph_perm_grad(const ph_c128* A, int32_t n, int64_t batch, const ph_c128* grad_out, ph_c128* perm_out,
                            ph_c128* grad_A, const ph_opts* opt, void* stream) {
  PH_TRACE("ph_perm_grad");
  Opts o;
  int rc = read_opts(opt, &o);
  if (rc) return rc;
  if (o.algo != PH_GLYNN) return fail(PH_EINVAL, "ph_perm_grad supports PH_GLYNN only");
  if (n < 1) return fail(PH_EINVAL, "n=%d < 1", n);
  if (n > PH_NMAX_GRAD) return fail(PH_ERANGE, "n=%d > %d", n, PH_NMAX_GRAD);
  if (batch < 0) return fail(PH_EINVAL, "batch=%lld < 0", (long long)batch);
  if (batch > 0 && (!A || !grad_A)) return fail(PH_EINVAL, "A or grad_A is NULL");
  const int cus = num_cus();
  if (cus <= 0) return PH_EUNSUPPORTED;
  return perm_grad_launch(reinterpret_cast<const double2*>(A), n, batch, reinterpret_cast<const double2*>(grad_out),
                          reinterpret_cast<double2*>(perm_out), reinterpret_cast<double2*>(grad_A), o,
                          (hipStream_t)stream, cus);
}
