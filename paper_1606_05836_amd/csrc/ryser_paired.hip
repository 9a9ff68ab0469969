// Ryser's formula with the complement pairing of Supplementary Algorithm S3
// (gfx950): one lane, or from n = 19 a pair of lanes, per chunk of the
// pairing loop.
//
// Eq. (S1) sums over all 2^n column subsets S.  Algorithm S3 runs its loop
// over the subsets S of the first n - 1 columns only and takes with each the
// term of its complement S_C among all n columns, so every subset is summed
// once and every iteration does the same work.  Here the loop index k in
// [0, 2^(n-1)) is walked in reflected Gray order (S = the set bits of
// k XOR (k >> 1)): each lane takes a chunk of 2^c consecutive indices, seeds
// its row sums r_i(S) at the chunk start and updates them by one column per
// step.  The complement's row sums are T_i - r_i(S), T_i the full row sums
// (computed once per workgroup, in column order), and the pair contributes
//     (-1)^|S| [ prod_i r_i(S) + (-1)^n prod_i (T_i - r_i(S)) ],
// where (-1)^|S| = (-1)^k.  The chunk sums go through the per-wave partials
// and the fixed-order finalize of the one-matrix sweeps, which apply the
// formula's (-1)^n.
//
// Up to n = 18 one lane takes a loop index, with the row totals read from
// LDS at every term.  From n = 19 the rows of both sums would not fit one
// lane at two waves per SIMD, so lanes l and l + 32 share the index as in the
// two-lane forward sweep: each holds R = ceil(n/2) rows of r_i(S) and of T_i
// (in registers), forms its half of both products, and the upper lane's two
// halves reach the lower lane through v_permlane32_swap.  For odd n the upper
// lane's last row is padding with r = 1 and T = 2, so both of its factors are 1.
// It walks its chunks as the two-lane forward sweep does: blocks of 16 steps
// whose columns, directions and term signs are compile-time constants, the
// four lowest update columns resident across each 16-lane DPP row, the
// block-boundary column from LDS; its chunks are therefore at least 16 indices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>

#include "dd.hpp"
#include "permhip.h"
#include "ph_host.hpp"
#include "ph_internal.hpp"
#include "sweep.hpp"
#include "sweep_pair.hpp"

namespace ph {

constexpr int PAIRED_NMAX = 32;
constexpr int PAIRED_TWO_LANE_NMIN = 19;

template <int N>
__global__ __launch_bounds__(256) void k_ryser_paired(const double2* __restrict__ a, int64_t lda, int c,
                                                      uint64_t nchunks, double4* __restrict__ partials, int plain) {
  extern __shared__ double2 lds_paired[];
  double2* col = lds_paired;          // column j of A at col + j * N
  double2* tot = lds_paired + N * N;  // row totals T_i
  for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
    const int i = e / N, j = e % N;
    col[j * N + i] = a[(int64_t)i * lda + j];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    double2 s = make_double2(0.0, 0.0);
    for (int j = 0; j < N; ++j) {
      s.x += col[j * N + i].x;
      s.y += col[j * N + i].y;
    }
    tot[i] = s;
  }
  __syncthreads();
  const double sgn_c = (N & 1) ? -1.0 : 1.0;  // (-1)^|S_C| = (-1)^n (-1)^|S|
  const uint64_t lanes = (uint64_t)gridDim.x * blockDim.x;
  const uint32_t len = 1u << c;
  dd2 acc = {0.0, 0.0, 0.0, 0.0};
  for (uint64_t ch = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; ch < nchunks; ch += lanes) {
    const uint64_t k0 = ch << c;
    uint64_t g = k0 ^ (k0 >> 1);
    double2 r[N];
#pragma unroll
    for (int i = 0; i < N; ++i) r[i] = make_double2(0.0, 0.0);
#pragma unroll 1
    for (int j = 0; j < N - 1; ++j) {
      if ((g >> j) & 1) {
        const double2* cj = col + j * N;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          r[i].x += cj[i].x;
          r[i].y += cj[i].y;
        }
      }
    }
    double2 sb = make_double2(0.0, 0.0);
    for (uint32_t t = 0; t < len; ++t) {
      if (t != 0) {
        // the step into index k0 + t flips bit b = ctz(t) of the Gray word
        // (k0 is a multiple of the chunk length): column b joins S or leaves it
        const int b = __builtin_ctz(t);
        g ^= (uint64_t)1 << b;
        const double w = ((g >> b) & 1) ? 1.0 : -1.0;
        const double2* cb = col + b * N;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          r[i].x = fma(w, cb[i].x, r[i].x);
          r[i].y = fma(w, cb[i].y, r[i].y);
        }
      }
      double2 p = r[0];
      double2 q = make_double2(tot[0].x - r[0].x, tot[0].y - r[0].y);
#pragma unroll
      for (int i = 1; i < N; ++i) {
        p = cmul(p, r[i]);
        q = cmul(q, make_double2(tot[i].x - r[i].x, tot[i].y - r[i].y));
      }
      const double s = ((k0 + t) & 1) ? -1.0 : 1.0;  // (-1)^|S|
      sb.x = fma(s, fma(sgn_c, q.x, p.x), sb.x);
      sb.y = fma(s, fma(sgn_c, q.y, p.y), sb.y);
      if (((t + 1) & 15) == 0 || t + 1 == len) flush(acc, sb, plain != 0, true);
    }
  }
  acc = wave_reduce(acc, plain != 0);
  const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if ((threadIdx.x & 63) == 0) partials[wave] = make_double4(acc.hr, acc.lr, acc.hi, acc.li);
}

// One loop index over a pair of lanes: sb += (-1)^|S| [prod_i r_i + (-1)^n
// prod_i (T_i - r_i)], each lane multiplying its own rows (two chains per
// product), the upper lane's two halves received through v_permlane32_swap
// (up_p and up_q enter with the previous index's, dead by then).
template <int R>
__device__ __forceinline__ void term_paired(const double2 (&r)[R], const double2 (&tr)[R], double2& sb,
                                            double2& up_p, double2& up_q, bool neg, double sgn_c) {
  static_assert(R >= 2, "two chains");
  double2 p0 = r[0], p1 = r[1];
  double2 q0 = make_double2(tr[0].x - r[0].x, tr[0].y - r[0].y);
  double2 q1 = make_double2(tr[1].x - r[1].x, tr[1].y - r[1].y);
#pragma unroll
  for (int i = 2; i < R; ++i) {
    const double2 d = make_double2(tr[i].x - r[i].x, tr[i].y - r[i].y);
    if (i & 1) {
      p1 = cmul(p1, r[i]);
      q1 = cmul(q1, d);
    } else {
      p0 = cmul(p0, r[i]);
      q0 = cmul(q0, d);
    }
  }
  double2 p = cmul(p0, p1), q = cmul(q0, q1);
  from_upper(p.x, up_p.x);
  from_upper(p.y, up_p.y);
  from_upper(q.x, up_q.x);
  from_upper(q.y, up_q.y);
  const double2 pp = cmul(p, up_p), qq = cmul(q, up_q);
  const double s = neg ? -1.0 : 1.0;
  sb.x = fma(s, fma(sgn_c, qq.x, pp.x), sb.x);
  sb.y = fma(s, fma(sgn_c, qq.y, pp.y), sb.y);
}

// Two lanes per loop index (n >= PAIRED_TWO_LANE_NMIN), the walk of the
// two-lane forward sweep: the column table in LDS with stride 2R (rows
// padded with zeros), four update columns resident over each 16-lane DPP row,
// chunks of 2^c indices (c >= 4) in blocks of 16 whose steps, signs and term
// signs are compile-time constants, the block-boundary column from LDS.
template <int N>
__global__ __launch_bounds__(256) void k_ryser_paired_2l(const double2* __restrict__ a, int64_t lda, int c,
                                                         uint64_t nchunks, double4* __restrict__ partials,
                                                         int plain) {
  using P = PairShape<N, ALGO_RYSER>;
  constexpr int R = P::R, RS = P::RS, LOGU = P::LOGU, U = 1 << LOGU;
  static_assert(LOGU == 4 && P::OFF == 0, "Gray bit b is column b");
  extern __shared__ double2 lds_paired[];
  double2* tot = lds_paired + N * RS;  // row totals T_i; 2 on a padding row
  stage_table_pair<N, ALGO_RYSER>(lds_paired, a, lda);
  for (int i = threadIdx.x; i < RS; i += blockDim.x) {
    double2 t = make_double2(i < N ? 0.0 : 2.0, 0.0);
    if (i < N) {
      for (int j = 0; j < N; ++j) {
        t.x += lds_paired[j * RS + i].x;
        t.y += lds_paired[j * RS + i].y;
      }
    }
    tot[i] = t;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const bool upper = lane >= 32;
  const double2* Tl = lds_paired + (upper ? R : 0);  // this lane's half of each column
  double2 tr[R];                                      // this lane's row totals
#pragma unroll
  for (int i = 0; i < R; ++i) tr[i] = tot[(upper ? R : 0) + i];
  ResidentPair<N, ALGO_RYSER> res;
  res.load(Tl);
  const double sgn_c = (N & 1) ? -1.0 : 1.0;
  // lanes l and l + 32 of a wavefront form one pair and take the same chunks
  const uint64_t pairs = (uint64_t)gridDim.x * (blockDim.x >> 1);
  const uint64_t pid = (uint64_t)blockIdx.x * (blockDim.x >> 1) + (threadIdx.x >> 6) * 32 + (lane & 31);
  const uint32_t nblk = 1u << (c - LOGU);
  const double one = 1.0, mone = -1.0;
  // n >= 23 (two waves per SIMD already): each block boundary's column comes
  // from a staged buffer refilled after the previous boundary (column 0,
  // unused, when no boundary is left); below, the extra registers would cost
  // a wave per SIMD and the boundary reads its column from LDS at the step
  constexpr bool STG = N >= 23;
  double xs[P::NP];
  dd2 acc = {0.0, 0.0, 0.0, 0.0};
  for (uint64_t ch = pid; ch < nchunks; ch += pairs) {
    const uint64_t k0 = ch << c;
    double2 r[R];
    seed_pair<N, ALGO_RYSER>(r, k0, Tl, upper);
    if constexpr (STG) stage_column_pair<N, ALGO_RYSER>(xs, Tl, nblk > 1 ? LOGU : 0);
    double2 sb = make_double2(0.0, 0.0), up_p = make_double2(0.0, 0.0), up_q = make_double2(0.0, 0.0);
    term_paired<R>(r, tr, sb, up_p, up_q, false, sgn_c);  // index k0 (even)
    for (uint32_t m = 0; m < nblk; ++m) {
      const uint32_t tb = m << LOGU;
      static_for<1, U>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        constexpr int b = __builtin_ctz(s);
        // column b joins S (+) iff bit b + 1 of the new index is clear
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
          fma_lds<R>(r, sg, Tl + b * RS);
        term_paired<R>(r, tr, sb, up_p, up_q, (s & 1) != 0, sgn_c);
        __builtin_amdgcn_sched_barrier(0);
      });
      if (m + 1 < nblk) {
        // block boundary: index k0 + tb + U flips bit LOGU + ctz(m + 1)
        const int b = LOGU + __builtin_ctz(m + 1);
        const uint64_t k = k0 + tb + U;
        const double sgb = ((k >> (b + 1)) & 1) ? -1.0 : 1.0;
        if constexpr (STG) {
          add_resident<R, P::NP>(r, xs, sgb);
          stage_column_pair<N, ALGO_RYSER>(xs, Tl, m + 2 < nblk ? LOGU + __builtin_ctz(m + 2) : 0);
        } else {
          fma_lds<R>(r, sgb, Tl + b * RS);
        }
        term_paired<R>(r, tr, sb, up_p, up_q, false, sgn_c);
      }
      flush(acc, sb, plain != 0, !upper);
    }
  }
  acc = wave_reduce(acc, plain != 0);
  const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (lane == 0) partials[wave] = make_double4(acc.hr, acc.lr, acc.hi, acc.li);
}

template <int N>
static const void* paired_kernel() {
  if constexpr (N < PAIRED_TWO_LANE_NMIN) return (const void*)&k_ryser_paired<N>;
  else return (const void*)&k_ryser_paired_2l<N>;
}

template <int... Is>
static const void* paired_lookup(int n, std::integer_sequence<int, Is...>) {
  const void* out = nullptr;
  ((n == Is + 1 ? (out = paired_kernel<Is + 1>(), 0) : 0), ...);
  return out;
}

static int perm_ryser_paired(const double2* A, int n, int64_t lda, double2* out, const Opts& o, hipStream_t st,
                             int cus) {
  hipError_t e;
  const int plain = o.plain ? 1 : 0;
  if (n == 0) {
    launch_finalize_single(nullptr, 0, 0, ALGO_RYSER, plain, out, st);
    e = hipGetLastError();
    return e == hipSuccess ? PH_OK : hip_fail(e, "finalize launch");
  }
  const void* kern = paired_lookup(n, std::make_integer_sequence<int, PAIRED_NMAX>{});
  if (!kern) return fail(PH_ERANGE, "no paired Ryser kernel for n=%d", n);
  // loop indices [0, 2^(n-1)) in chunks of 2^c: at least 2^17 chunks where
  // the range allows, at most 2^10 indices per chunk
  const int nb = n - 1;
  const bool two_lane = n >= PAIRED_TWO_LANE_NMIN;
  int c = o.chunk_log2 > 0 ? o.chunk_log2 : std::min(10, nb - 17);
  // the two-lane walk takes its steps in blocks of 16
  c = std::max(two_lane ? 4 : 0, std::min(c, nb));
  const uint64_t nchunks = (uint64_t)1 << (nb - c);
  const uint64_t per_block = two_lane ? 128 : 256;  // chunks a workgroup takes at a time
  const uint64_t blocks =
      std::max<uint64_t>(1, std::min<uint64_t>((nchunks + per_block - 1) / per_block, (uint64_t)cus * 2));
  const uint64_t nwaves = blocks * 4;
  void* ws = nullptr;
  int rc = workspace(st, nwaves * sizeof(double4), &ws);
  if (rc) return rc;
  double4* pw = static_cast<double4*>(ws);
  const int rs = two_lane ? 2 * ((n + 1) / 2) : n;  // rows per stored column
  const size_t lds = (size_t)(n * rs + rs) * sizeof(double2);
  const double2* a = A;
  int64_t ld = lda;
  uint64_t nch = nchunks;
  int cc = c, pl = plain;
  void* args[] = {&a, &ld, &cc, &nch, &pw, &pl};
  e = hipLaunchKernel(kern, dim3((unsigned)blocks), dim3(256), args, lds, st);
  if (e != hipSuccess) return hip_fail(e, "paired Ryser launch");
  launch_finalize_single(pw, (int64_t)nwaves, n, ALGO_RYSER, plain, out, st);
  e = hipGetLastError();
  return e == hipSuccess ? PH_OK : hip_fail(e, "finalize launch");
}

}  // namespace ph

using namespace ph;

extern "C" int ph_perm_ryser_paired(const ph_c128* A, int32_t n, int64_t lda, ph_c128* out, const ph_opts* opt,
                                    void* stream) {
  PH_TRACE("ph_perm_ryser_paired");
  Opts o;
  int rc = read_opts(opt, &o);
  if (rc) return rc;
  if (n < 0) return fail(PH_EINVAL, "n=%d < 0", n);
  if (n > PAIRED_NMAX) return fail(PH_ERANGE, "n=%d > %d (the paired walk keeps n row sums per lane)", n, PAIRED_NMAX);
  if (!out) return fail(PH_EINVAL, "out is NULL");
  if (n > 0 && !A) return fail(PH_EINVAL, "A is NULL");
  if (n > 0 && lda < n) return fail(PH_EINVAL, "lda=%lld < n=%d", (long long)lda, n);
  return perm_ryser_paired(reinterpret_cast<const double2*>(A), n, lda, reinterpret_cast<double2*>(out), o,
                           (hipStream_t)stream, num_cus());
}
