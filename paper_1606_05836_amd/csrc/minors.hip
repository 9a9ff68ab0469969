// Minors along one row: for an (N) x (N+1) matrix B, the N+1 permanents
//   P_l = Per(B without column l),  l = 0..N,
// i.e. the derivatives of Per([B; x]) with respect to the entries of a last
// row x.  Differentiating Eq. (S2) of that (N+1) x (N+1) matrix in x_l gives
//   P_l = 2^-N sum_delta (prod_j delta_j) delta_l prod_{i<N} r_i(delta),
// r_i = sum_j delta_j b_ij, delta_0 = +1: the forward sweep of B's N rows over
// its N + 1 columns, with each term s Q (sign times product) also added,
// signed by delta_l, into one sum per column.  The sampler needs exactly
// these (the weights of every candidate mode follow by expanding along x).
//
// Per lane, chunk [k0, k0 + 2^C) with C = 10, blocks of 16 terms:
//   columns of Gray bits 0..3 flip inside a block: one plain accumulator each,
//     the sign of every step known at compile time (bit 3 also depends on the
//     block index);
//   columns of bits 4..9 are constant inside a block: per block, the block's
//     sum signed by delta;
//   column 0 and the columns of bits >= 10 are constant over the chunk: the
//     chunk sum, signed by delta of the chunk's Gray word.
// At the chunk's end each column's contribution is summed over the
// wavefront (butterfly, fixed order) and lane l adds column l's total into
// its double-double accumulator.  Waves of a block are then summed in order
// per column, and a finalize kernel sums the blocks of each matrix in order.
#include <hip/hip_runtime.h>

#include <utility>

#include "dd.hpp"
#include "permhip.h"
#include "ph_host.hpp"
#include "ph_internal.hpp"
#include "sweep.hpp"

namespace ph {

constexpr int MINORS_C = 10;           // log2 chunk length
constexpr int MINORS_NMIN = 12;        // rows (the kernel needs N >= MINORS_C)
constexpr int MINORS_NMAX = PH_NMAX_GRAD - 1;

template <int N>
__device__ __forceinline__ double2 row_product(const double2 (&r)[N]) {
  double2 ch[4] = {r[0], r[1], r[2], r[3]};
#pragma unroll
  for (int i = 4; i < N; ++i) ch[i % 4] = cmul(ch[i % 4], r[i]);
  return cmul(cmul(ch[0], ch[1]), cmul(ch[2], ch[3]));
}

__device__ __forceinline__ double2 shfl_xor2(double2 v, int m) {
  return make_double2(__shfl_xor(v.x, m, 64), __shfl_xor(v.y, m, 64));
}

// Sum of v over the 64 lanes of the wavefront (same order on every lane).
__device__ __forceinline__ double2 wave_sum2(double2 v) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    const double2 o = shfl_xor2(v, m);
    v.x += o.x;
    v.y += o.y;
  }
  return v;
}

// tabs: batch of N x (N+1) BB/FG tables (T[0] = b_.0, T[j] = -2 b_.j,
// column-major, column stride N), table b at tabs + b * N * (N + 1).
// Block g works on matrix g / bpm; partials[g * (N + 1) + l] receives its
// unscaled double-double sum for column l.
template <int N>
__global__ __launch_bounds__(256) void k_minors(const double2* __restrict__ tabs, int bpm, uint64_t nchunks,
                                                double4* __restrict__ partials) {
  using S = Shape<N, ALGO_GLYNN>;
  // STG (N = 14..30): bits 0..2 resident, bit 3 and the block boundaries read
  // a staged column (stage_column) refilled after each use; the other orders
  // keep bits 0..3 resident and read the boundary column from LDS at the step
  // (the staged column would cost N = 12, 13 a wave per SIMD and spill at 31)
  constexpr bool STG = N >= 14 && N <= 30;
  constexpr int NC = N + 1, C = MINORS_C, DR = STG ? S::D - 1 : S::D;
  static_assert(S::LOGU == 4 && N >= C, "block and chunk sizes");
  __shared__ double2 T[N * NC];
  __shared__ dd2 wsum[4][NC];
  const int mat = blockIdx.x / bpm, blk = blockIdx.x % bpm;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double2* tab = tabs + (int64_t)mat * N * NC;
  for (int e = threadIdx.x; e < N * NC; e += blockDim.x) T[e] = tab[e];
  __syncthreads();
  Resident<N, ALGO_GLYNN, DR> res;
  res.load(T);
  const uint64_t nsuper = (nchunks + 63) >> 6;
  const uint64_t gw = (uint64_t)blk * 4 + w, nw = (uint64_t)bpm * 4;
  const uint64_t s0 = nsuper * gw / nw, s1 = nsuper * (gw + 1) / nw;
  dd2 own = {0.0, 0.0, 0.0, 0.0};  // column `lane`
  const double one = 1.0, mone = -1.0;
  for (uint64_t sc = s0; sc < s1; ++sc) {
    const uint64_t chunk = (sc << 6) + lane;
    const bool active = chunk < nchunks;
    const uint64_t k0 = chunk << C;
    double2 r[N];
    seed<N, ALGO_GLYNN>(r, k0, T, NC);
    double2 low[4], blkc[C - 4], V = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < 4; ++q) low[q] = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < C - 4; ++q) blkc[q] = make_double2(0.0, 0.0);
    constexpr uint32_t NBLK = 1u << (C - 4);
    double xs[S::NP];
    if constexpr (STG) stage_column<N, ALGO_GLYNN>(xs, T, 3);  // block 0's bit-3 step
    for (uint32_t m = 0; m < NBLK; ++m) {
      // delta of Gray bit 3 inside block m: bit 3 of t ^ bit 0 of m
      const double d3 = (m & 1) ? mone : one;
      double2 bs = make_double2(0.0, 0.0);
      static_for<0, 16>([&](auto sc2) {
        constexpr int s = decltype(sc2)::value;
        if constexpr (s > 0) {
          constexpr int b = __builtin_ctz(s);
          double sg;
          if constexpr (b + 1 < 4) sg = (((s >> (b + 1)) & 1) == 0) ? one : mone;
          else sg = (m & 1) ? mone : one;  // bit 4 of t = bit 0 of m
          static_assert(b < DR || b == 3, "bits above DR other than 3 are block boundaries");
          if constexpr (b < DR) {
            add_resident<N, S::NP>(r, res.col[b], sg);
          } else if constexpr (!STG) {
            fma_lds<N>(r, sg, T + (b + 1) * N);
          } else {
            add_resident<N, S::NP>(r, xs, sg);
            // the next block's boundary column (column 0, unused, after the last)
            stage_column<N, ALGO_GLYNN>(xs, T, m + 1 < NBLK ? 4 + __builtin_ctz(m + 1) : -1);
          }
        } else {
          if (m > 0) {
            // block boundary: t = 16 m flips Gray bit 4 + ctz(m)
            const int b = 4 + __builtin_ctz(m);
            const uint64_t k = k0 + ((uint64_t)m << 4);
            const double sgb = ((k >> (b + 1)) & 1) ? -1.0 : 1.0;
            if constexpr (STG) {
              add_resident<N, S::NP>(r, xs, sgb);
              stage_column<N, ALGO_GLYNN>(xs, T, 3);  // this block's bit-3 step
            } else {
              fma_lds<N>(r, sgb, T + (b + 1) * N);
            }
          }
        }
        double2 v = row_product<N>(r);
        if constexpr (s & 1) {
          v.x = -v.x;
          v.y = -v.y;
        }
        bs.x += v.x;
        bs.y += v.y;
        // Gray bits 0..2 of t: bit q of s ^ bit q+1 of s (set: delta = -1)
        static_for<0, 3>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          if constexpr ((((s >> q) ^ (s >> (q + 1))) & 1) != 0) {
            low[q].x -= v.x;
            low[q].y -= v.y;
          } else {
            low[q].x += v.x;
            low[q].y += v.y;
          }
        });
        constexpr double s3 = ((s >> 3) & 1) ? -1.0 : 1.0;
        low[3].x = fma(s3 * d3, v.x, low[3].x);
        low[3].y = fma(s3 * d3, v.y, low[3].y);
        __builtin_amdgcn_sched_barrier(0);
      });
      // bits 4..C-1 of the Gray word are constant in the block
      const uint64_t k = k0 + ((uint64_t)m << 4);
      const uint64_t g = k ^ (k >> 1);
#pragma unroll
      for (int q = 0; q < C - 4; ++q) {
        const double d = ((g >> (q + 4)) & 1) ? -1.0 : 1.0;
        blkc[q].x = fma(d, bs.x, blkc[q].x);
        blkc[q].y = fma(d, bs.y, blkc[q].y);
      }
      V.x += bs.x;
      V.y += bs.y;
    }
    // chunk contributions per column, summed over the wavefront
    const uint64_t g0 = k0 ^ (k0 >> 1);
#pragma unroll
    for (int l = 0; l < NC; ++l) {
      double2 x;
      if (l == 0) x = V;
      else if (l <= 4) x = low[l - 1];
      else if (l <= C) x = blkc[l - 5];
      else {
        const double d = ((g0 >> (l - 1)) & 1) ? -1.0 : 1.0;
        x = make_double2(d * V.x, d * V.y);
      }
      if (!active) x = make_double2(0.0, 0.0);
      x = wave_sum2(x);
      if (lane == l) dd_accumulate(own, x.x, x.y);
    }
  }
  if (lane < NC) wsum[w][lane] = own;
  __syncthreads();
  if (threadIdx.x < NC) {
    dd2 t = wsum[0][threadIdx.x];
    for (int q = 1; q < 4; ++q) t = dd_add(t, wsum[q][threadIdx.x]);
    partials[(int64_t)blockIdx.x * NC + threadIdx.x] = make_double4(t.hr, t.lr, t.hi, t.li);
  }
}

// out[mat * (N+1) + l] = 2^-N * sum over the matrix's bpm blocks (in order).
__global__ void k_minors_finalize(const double4* __restrict__ partials, int n_rows, int bpm,
                                  double2* __restrict__ out) {
  const int mat = blockIdx.x, l = threadIdx.x, nc = n_rows + 1;
  if (l >= nc) return;
  dd2 t = {0.0, 0.0, 0.0, 0.0};
  // the loads of U partials are issued before the first add (one memory
  // round trip per group); the adds keep the block order
  constexpr int U = 8;
  for (int b0 = 0; b0 < bpm; b0 += U) {
    double4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (b0 + u < bpm) v[u] = partials[((int64_t)mat * bpm + b0 + u) * nc + l];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (b0 + u >= bpm) break;
      t = dd_add(t, dd2{v[u].x, v[u].y, v[u].z, v[u].w});
    }
  }
  out[(int64_t)mat * nc + l] =
      make_double2(ldexp(t.hr, -n_rows) + ldexp(t.lr, -n_rows), ldexp(t.hi, -n_rows) + ldexp(t.li, -n_rows));
}

template <int... Is>
static const void* minors_lookup(int n, std::integer_sequence<int, Is...>) {
  const void* out = nullptr;
  ((n == MINORS_NMIN + Is ? (out = (const void*)&k_minors<MINORS_NMIN + Is>, 0) : 0), ...);
  return out;
}

// Minors along the last row for `batch` tables of n_rows x (n_rows + 1)
// (MINORS_NMIN <= n_rows <= MINORS_NMAX); out: batch x (n_rows + 1) complex.
int row_minors_launch(const double2* tabs, int n_rows, int64_t batch, double2* out, hipStream_t st, int cus) {
  const void* kern =
      minors_lookup(n_rows, std::make_integer_sequence<int, MINORS_NMAX - MINORS_NMIN + 1>{});
  if (!kern) return fail(PH_ERANGE, "row minors: %d rows", n_rows);
  const uint64_t nchunks = (uint64_t)1 << (n_rows - MINORS_C);
  const uint64_t nsuper = (nchunks + 63) / 64;
  // about 8 blocks per compute unit in all, at most one super-chunk-group per wave
  int64_t bpm = std::max<int64_t>(1, (8LL * cus + batch - 1) / std::max<int64_t>(batch, 1));
  bpm = std::min<int64_t>(bpm, std::max<int64_t>(1, (int64_t)((nsuper + 3) / 4)));
  const int nc = n_rows + 1;
  void* ws = nullptr;
  int rc = workspace_slot(st, (size_t)batch * bpm * nc * sizeof(double4), WS_MINORS, &ws);
  if (rc) return rc;
  double4* parts = static_cast<double4*>(ws);
  int b = (int)bpm;
  uint64_t nch = nchunks;
  void* args[] = {(void*)&tabs, &b, &nch, &parts};
  hipError_t e = hipLaunchKernel(kern, dim3((unsigned)(batch * bpm)), dim3(256), args, 0, st);
  if (e != hipSuccess) return hip_fail(e, "row minors launch");
  hipLaunchKernelGGL(k_minors_finalize, dim3((unsigned)batch), dim3(64), 0, st, parts, n_rows, b, out);
  e = hipGetLastError();
  return e == hipSuccess ? PH_OK : hip_fail(e, "row minors finalize");
}

// Row-major n x (n+1) matrices -> BB/FG tables (column-major, stride n).
__global__ void k_minors_prep(const double2* __restrict__ b, int n, double2* __restrict__ tabs) {
  const int64_t mat = blockIdx.x;
  const int nc = n + 1;
  const double2* src = b + mat * n * nc;
  double2* out = tabs + mat * n * nc;
  for (int e = threadIdx.x; e < n * nc; e += blockDim.x) {
    const int j = e / n, i = e % n;
    double2 v = src[i * nc + j];
    if (j > 0) v = make_double2(-2.0 * v.x, -2.0 * v.y);
    out[e] = v;
  }
}

// Row-major n x (n+1) matrices -> (n+1) x (n+1) matrices with a zero last row.
__global__ void k_minors_square(const double2* __restrict__ b, int n, double2* __restrict__ sq) {
  const int64_t mat = blockIdx.x;
  const int nc = n + 1;
  for (int e = threadIdx.x; e < nc * nc; e += blockDim.x) {
    const int i = e / nc;
    sq[mat * nc * nc + e] = i < n ? b[mat * n * nc + e] : make_double2(0.0, 0.0);
  }
}

// minors[mat][l] = conj(grad[mat][n][l]) (the gradient sweep writes conj(minor)).
__global__ void k_minors_from_grad(const double2* __restrict__ grad, int n, int64_t batch,
                                   double2* __restrict__ out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int nc = n + 1;
  if (e < batch * nc) {
    const int64_t mat = e / nc;
    const int l = (int)(e % nc);
    const double2 g = grad[mat * nc * nc + (int64_t)n * nc + l];
    out[e] = make_double2(g.x, -g.y);
  }
}

__global__ void k_fill_one(double2* __restrict__ out, int64_t count) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < count) out[e] = make_double2(1.0, 0.0);
}

}  // namespace ph

using namespace ph;

extern "C" int ph_perm_row_minors(const ph_c128* B, int32_t n, int64_t batch, ph_c128* minors, const ph_opts* opt,
                                  void* stream) {
  PH_TRACE("ph_perm_row_minors");
  Opts o;
  int rc = read_opts(opt, &o);
  if (rc) return rc;
  if (o.algo != PH_GLYNN) return fail(PH_EINVAL, "ph_perm_row_minors supports PH_GLYNN only");
  if (n < 0) return fail(PH_EINVAL, "n=%d < 0", n);
  if (n > PH_NMAX_GRAD - 1) return fail(PH_ERANGE, "n=%d > %d", n, PH_NMAX_GRAD - 1);
  if (batch < 0) return fail(PH_EINVAL, "batch=%lld < 0", (long long)batch);
  if (batch == 0) return PH_OK;
  if (!minors || (n > 0 && !B)) return fail(PH_EINVAL, "B or minors is NULL");
  const int cus = num_cus();
  if (cus <= 0) return PH_EUNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  double2* out = reinterpret_cast<double2*>(minors);
  const double2* b = reinterpret_cast<const double2*>(B);
  const int nc = n + 1;
  if (n == 0) {
    hipLaunchKernelGGL(k_fill_one, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, st, out, batch);
  } else if (n >= MINORS_NMIN) {
    void* ws = nullptr;
    if ((rc = workspace_slot(st, (size_t)batch * n * nc * sizeof(double2), WS_MINORS_TABLES, &ws))) return rc;
    double2* tabs = static_cast<double2*>(ws);
    hipLaunchKernelGGL(k_minors_prep, dim3((unsigned)batch), dim3(256), 0, st, b, n, tabs);
    if ((rc = row_minors_launch(tabs, n, batch, out, st, cus))) return rc;
  } else {
    void* ws = nullptr;
    const size_t sq = (size_t)batch * nc * nc * sizeof(double2);
    if ((rc = workspace_slot(st, 2 * sq, WS_MINORS_TABLES, &ws))) return rc;
    double2* sqm = static_cast<double2*>(ws);
    double2* grad = reinterpret_cast<double2*>(static_cast<char*>(ws) + sq);
    hipLaunchKernelGGL(k_minors_square, dim3((unsigned)batch), dim3(256), 0, st, b, n, sqm);
    if ((rc = perm_grad_launch(sqm, nc, batch, nullptr, nullptr, grad, o, st, cus))) return rc;
    const int64_t tot = batch * nc;
    hipLaunchKernelGGL(k_minors_from_grad, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, grad, n, batch,
                       out);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? PH_OK : hip_fail(e, "row minors");
}
