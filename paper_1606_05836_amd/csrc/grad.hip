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
// (1) A term is split over a quad of four lanes; lane `sigma` of the quad
//     owns rows [sigma*M, sigma*M + M).  Each lane forms suffix products of
//     its rows, the quad exchanges the partial products with DPP quad
//     permutes (P_other = product of the other three lanes' rows), and a
//     prefix pass started from P_other yields q_i for its rows.  Splitting
//     the rows keeps the per-lane state (row sums, suffix products, running
//     sums, stored columns) in the register file.
//
// (2) Summation by parts.  In a chunk of L = 2^c terms with running sum
//     W(t) = sum_{tau <= t} w(tau),
//        sum_t delta_j(t) w(t) = delta_j(L-1) W(L-1) - 2 sum_{flips of j at t} delta_j(t) W(t-1),
//     so each step touches only the column whose delta flips.  The K columns
//     that flip most often (Gray bits 0..K-1, used by 1 - 2^-K of all steps)
//     are accumulated per lane in registers; a flip of any other column, and
//     the boundary term of every column at the chunk end, is summed over the
//     16 quads of the wavefront through LDS (each lane adds 16 values for one
//     output) and added into the wavefront's n x n accumulator in global
//     memory.  Every address of that accumulator is read and written by one
//     fixed lane only, so program order is the only ordering needed.
//
// The forward permanent comes out of the same sweep (prod of all rows).
// All sums are in a fixed order, so results are bitwise reproducible.
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

// quad permutes of a double: lane ^ 1 and lane ^ 2 within each quad
__device__ __forceinline__ double quad_xor1(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false),
                          __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double quad_xor2(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false),
                          __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false));
}
__device__ __forceinline__ double2 quad_xor1(double2 v) { return make_double2(quad_xor1(v.x), quad_xor1(v.y)); }
__device__ __forceinline__ double2 quad_xor2(double2 v) { return make_double2(quad_xor2(v.x), quad_xor2(v.y)); }

// registers: stored columns per M (rows per lane)
#ifndef PH_GRAD_K
#define PH_GRAD_K(M) ((M) == 1 ? 1 : ((M) <= 5 ? 2 : 1))
#endif
#ifndef PH_GRAD_WAVES
#define PH_GRAD_WAVES(M) ((M) <= 1 ? 4 : ((M) <= 3 ? 3 : 2))
#endif

template <int M>
struct GradShape {
  static constexpr int K = PH_GRAD_K(M);
  static constexpr int U = 1 << K;
  static constexpr int ROWS = 4 * M;  // padded rows of the table
  // Gray bits K..K+R-1 (the columns flipped at block boundaries most often)
  // collect their quad sums in registers of the owning lane
  static constexpr int R = 4;
  // target wavefronts per SIMD (register budget 512 / WAVES per lane)
  static constexpr int WAVES = PH_GRAD_WAVES(M);
};

struct GradArgs {
  const double2* tabs;  // per matrix: n columns x ROWS rows (zero padded)
  int n, c;
  int64_t nsuper;       // super-chunks per matrix (16 chunks each)
  int s_per;            // units (slices) per matrix
  int64_t units;        // batch * s_per
  uint32_t* counter;
  double2* ghat;        // per (unit, wave): n x ROWS complex
  double4* fparts;      // per (unit, wave): forward partial (dd)
  int plain;
};

template <int M>
struct GradLane {
  double2 r[M];
  double2 W[M];
  double2 G[GradShape<M>::K][M];
  double2 colK[GradShape<M>::K][M];  // the lane's rows of columns 1..K
};

// LDS sum of wt * W over the 16 quads of the wavefront.  Lane o < 8M gets
// output o -- row o / 2 of the quad's 4M rows, real part if o is even --
// the other lanes get 0.  Staging: lane l writes its M complex values at
// complex offset l * SS with SS = M rounded up to odd, so the 16-byte
// writes of eight consecutive lanes cover all 32 banks once and the reads
// (consecutive lanes, consecutive addresses) are conflict-free.
template <int M>
struct Stage {
  static constexpr int SS = M | 1;  // complex entries per lane
};

template <int M>
__device__ __forceinline__ double quad_sum(const double2 (&W)[M], double wt, double* stage) {
  constexpr int SS = Stage<M>::SS;
  const int lane = threadIdx.x & 63;
  double2* st2 = reinterpret_cast<double2*>(stage);
#pragma unroll
  for (int ii = 0; ii < M; ++ii) st2[lane * SS + ii] = make_double2(wt * W[ii].x, wt * W[ii].y);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  double s = 0.0;
  if (lane < 8 * M) {
    const int sig = lane / (2 * M), d = lane % (2 * M);
    const double* base = stage + 2 * sig * SS + d;
#pragma unroll
    for (int g = 0; g < 16; ++g) s += base[2 * 4 * SS * g];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  return s;
}

// Adds a quad sum into the wavefront's accumulator column (global memory,
// owned entry by entry by the lanes that compute them).
template <int M>
__device__ __forceinline__ void quad_sum_add(const double2 (&W)[M], double wt, double* stage, double* gcol) {
  const double s = quad_sum<M>(W, wt, stage);
  const int lane = threadIdx.x & 63;
  if (lane < 8 * M) gcol[lane] += s;
}

// One term: leave-one-out products of the quad's rows, W += st q, and the
// full product into sb (st = the term's sign).  The suffix products and the
// prefix products of the lane's own rows are two independent chains; the
// quad exchange then gives O = product of the other lanes' rows and
// q_i = (O pre_i) suf_{i+1}, the last multiply fused into the W update.
template <int M>
__device__ __forceinline__ void grad_term(GradLane<M>& L, double st, double2& sb) {
  double2 suf[M], pre[M];
  suf[M - 1] = L.r[M - 1];
#pragma unroll
  for (int ii = M - 2; ii >= 0; --ii) suf[ii] = cmul(L.r[ii], suf[ii + 1]);
  if constexpr (M > 1) {
    pre[1] = L.r[0];
#pragma unroll
    for (int ii = 2; ii < M; ++ii) pre[ii] = cmul(pre[ii - 1], L.r[ii - 1]);
  }
  const double2 p1 = quad_xor1(suf[0]);
  const double2 pair = cmul(suf[0], p1);
  const double2 pair2 = quad_xor2(pair);
  const double2 o = cmul(p1, pair2);  // product of the other three lanes' rows
  const double2 os = make_double2(st * o.x, st * o.y);
#pragma unroll
  for (int ii = 0; ii < M; ++ii) {
    const double2 t = ii == 0 ? os : cmul(os, pre[ii]);  // st * O * prefix
    if (ii < M - 1) {
      const double2 s1 = suf[ii + 1];
      L.W[ii].x = fma(t.x, s1.x, L.W[ii].x);
      L.W[ii].x = fma(-t.y, s1.y, L.W[ii].x);
      L.W[ii].y = fma(t.x, s1.y, L.W[ii].y);
      L.W[ii].y = fma(t.y, s1.x, L.W[ii].y);
    } else {
      L.W[ii].x += t.x;
      L.W[ii].y += t.y;
    }
  }
  // full product st * O * P_own
  sb.x = fma(os.x, suf[0].x, sb.x);
  sb.x = fma(-os.y, suf[0].y, sb.x);
  sb.y = fma(os.x, suf[0].y, sb.y);
  sb.y = fma(os.y, suf[0].x, sb.y);
}

// r += s * v (own rows, values already loaded)
template <int M>
__device__ __forceinline__ void grad_apply(GradLane<M>& L, double s, const double2 (&v)[M]) {
#pragma unroll
  for (int ii = 0; ii < M; ++ii) {
    L.r[ii].x = fma(s, v[ii].x, L.r[ii].x);
    L.r[ii].y = fma(s, v[ii].y, L.r[ii].y);
  }
}

template <int M>
__device__ __forceinline__ void grad_load(double2 (&v)[M], const double2* col) {
#pragma unroll
  for (int ii = 0; ii < M; ++ii) v[ii] = col[ii];
}

// r += s * column (own rows, from LDS)
template <int M>
__device__ __forceinline__ void grad_update(GradLane<M>& L, double s, const double2* col) {
#pragma unroll
  for (int ii = 0; ii < M; ++ii) {
    const double2 v = col[ii];
    L.r[ii].x = fma(s, v.x, L.r[ii].x);
    L.r[ii].y = fma(s, v.y, L.r[ii].y);
  }
}

template <int M>
__global__ __launch_bounds__(256, GradShape<M>::WAVES) void k_grad(GradArgs a) {
  using GS = GradShape<M>;
  constexpr int K = GS::K, U = GS::U, ROWS = GS::ROWS;
  extern __shared__ double lds[];
  double2* tab = reinterpret_cast<double2*>(lds);               // n * ROWS complex
  double* stage_all = lds + 2 * (size_t)a.n * ROWS;               // 4 waves * 64 * SS complex
  __shared__ int64_t s_unit;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sig = lane & 3, grp = lane >> 2;
  double* stage = stage_all + wave * 2 * 64 * Stage<M>::SS;
  const int n = a.n, c = a.c, nb = n - 1;
  const int row0 = sig * M;
  for (;;) {
    if (threadIdx.x == 0) s_unit = (int64_t)atomicAdd(a.counter, 1u);
    __syncthreads();
    const int64_t u = s_unit;
    if (u >= a.units) break;
    const int64_t mat = u / a.s_per, sl = u % a.s_per;
    const double2* gtab = a.tabs + (size_t)mat * n * ROWS;
    for (int e = threadIdx.x; e < n * ROWS; e += blockDim.x) tab[e] = gtab[e];
    __syncthreads();
    const int64_t slot = u * 4 + wave;
    double* ghat = reinterpret_cast<double*>(a.ghat + (size_t)slot * n * ROWS);
    // each lane zeroes the accumulator entries it will own
    if (lane < 8 * M)
      for (int j = 0; j < n; ++j) ghat[j * 2 * ROWS + lane] = 0.0;
    GradLane<M> L;
#pragma unroll
    for (int b = 0; b < K; ++b)
#pragma unroll
      for (int ii = 0; ii < M; ++ii) {
        L.G[b][ii] = make_double2(0.0, 0.0);
        L.colK[b][ii] = tab[(b + 1) * ROWS + row0 + ii];
      }
    dd2 acc = {0.0, 0.0, 0.0, 0.0};
    double bacc[GS::R];
#pragma unroll
    for (int q = 0; q < GS::R; ++q) bacc[q] = 0.0;
    const int64_t sb0 = a.nsuper * sl / a.s_per, sb1 = a.nsuper * (sl + 1) / a.s_per;
    const uint64_t nchunks = (uint64_t)1 << (nb - c);
    for (int64_t sc = sb0 + wave; sc < sb1; sc += 4) {
      const uint64_t chunk = ((uint64_t)sc << 4) + grp;
      const uint64_t k0 = chunk << c;
      // quads past the last chunk (tiny n) walk a copy but add nothing
      const double act = chunk < nchunks ? 1.0 : 0.0;
      // seed own rows: r_i = a_i0 + sum_{j>=1} delta_j a_ij (delta_j a_ij = (-delta_j/2) T[j])
      const uint64_t g0 = k0 ^ (k0 >> 1);
#pragma unroll
      for (int ii = 0; ii < M; ++ii) L.r[ii] = tab[row0 + ii];
#pragma unroll 1
      for (int j = 1; j < n; ++j) grad_update<M>(L, ((g0 >> (j - 1)) & 1) ? 0.5 : -0.5, tab + j * ROWS + row0);
#pragma unroll
      for (int ii = 0; ii < M; ++ii) {
        if (row0 + ii >= n) L.r[ii] = make_double2(1.0, 0.0);  // padding rows
        L.W[ii] = make_double2(0.0, 0.0);
      }
      double2 sb = make_double2(0.0, 0.0);
      grad_term<M>(L, act, sb);  // offset 0 (k0 even)
      const uint32_t nblk = 1u << (c - K);
      for (uint32_t m = 0; m < nblk; ++m) {
        const uint32_t tb = m << K;
        static_for<1, U>([&](auto scst) {
          constexpr int s = decltype(scst)::value;
          constexpr int b = __builtin_ctz(s);
          // "set" <=> the new Gray bit is 1 <=> delta_{b+1} becomes -1
          double sgu;
          if constexpr (b + 1 < K) {
            sgu = (((s >> (b + 1)) & 1) == 0) ? 1.0 : -1.0;
          } else {
            const uint64_t k = k0 + tb + s;
            sgu = ((k >> (b + 1)) & 1) ? -1.0 : 1.0;
          }
          // summation by parts with W through t-1: -2 delta_new W = 2 sgu W
#pragma unroll
          for (int ii = 0; ii < M; ++ii) {
            L.G[b][ii].x = fma(2.0 * sgu, L.W[ii].x, L.G[b][ii].x);
            L.G[b][ii].y = fma(2.0 * sgu, L.W[ii].y, L.G[b][ii].y);
          }
          grad_apply<M>(L, sgu, L.colK[b]);
          grad_term<M>(L, (s & 1) ? -act : act, sb);
          __builtin_amdgcn_sched_barrier(0);
        });
        if (m + 1 < nblk) {
          const int b = K + __builtin_ctz(m + 1);
          const uint64_t k = k0 + tb + U;
          const double sgu = ((k >> (b + 1)) & 1) ? -1.0 : 1.0;
          if (b < K + GS::R) {
            const double qs = quad_sum<M>(L.W, 2.0 * sgu, stage);
#pragma unroll
            for (int q = 0; q < GS::R; ++q)
              if (b == K + q) bacc[q] += qs;
          } else {
            quad_sum_add<M>(L.W, 2.0 * sgu, stage, ghat + (size_t)(b + 1) * 2 * ROWS);
          }
          grad_update<M>(L, sgu, tab + (b + 1) * ROWS + row0);
          grad_term<M>(L, act, sb);
        }
        flush(acc, sb, a.plain != 0, sig == 0);
      }
      // boundary terms delta_j(last) W(last) for every column
      const uint64_t kl = k0 + ((uint64_t)1 << c) - 1;
      const uint64_t gl = kl ^ (kl >> 1);
      quad_sum_add<M>(L.W, 1.0, stage, ghat);  // column 0: delta_0 = +1
#pragma unroll 1
      for (int j = K + 1; j < n; ++j)
        quad_sum_add<M>(L.W, ((gl >> (j - 1)) & 1) ? -1.0 : 1.0, stage, ghat + (size_t)j * 2 * ROWS);
#pragma unroll
      for (int b = 0; b < K; ++b) {
        const double dl = ((gl >> b) & 1) ? -1.0 : 1.0;
#pragma unroll
        for (int ii = 0; ii < M; ++ii) {
          L.G[b][ii].x = fma(dl, L.W[ii].x, L.G[b][ii].x);
          L.G[b][ii].y = fma(dl, L.W[ii].y, L.G[b][ii].y);
        }
      }
    }
    // register-held boundary columns and stored columns into the accumulator
    if (lane < 8 * M) {
#pragma unroll
      for (int q = 0; q < GS::R; ++q)
        if (K + q + 1 < n) ghat[(size_t)(K + q + 1) * 2 * ROWS + lane] += bacc[q];
    }
#pragma unroll
    for (int b = 0; b < K; ++b)
      if (b + 1 < n) quad_sum_add<M>(L.G[b], 1.0, stage, ghat + (size_t)(b + 1) * 2 * ROWS);
    if (sig != 0) acc = dd2{0.0, 0.0, 0.0, 0.0};
    acc = wave_reduce(acc, a.plain != 0);
    if (lane == 0) a.fparts[slot] = make_double4(acc.hr, acc.lr, acc.hi, acc.li);
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

// Per matrix: M = 2^-(n-1) sum over the (unit, wave) accumulators in order,
// grad = g * conj(M), perm = 2^-(n-1) sum of forward partials.
__global__ void k_grad_finalize(const double2* __restrict__ ghat, const double4* __restrict__ fparts, int n, int rows,
                                int s_per, int plain, const double2* __restrict__ gout, double2* __restrict__ pout,
                                double2* __restrict__ grad) {
  const int64_t mat = blockIdx.x;
  const int64_t slots = (int64_t)s_per * 4, first = mat * slots;
  const double2 g = gout ? gout[mat] : make_double2(1.0, 0.0);
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    dd2 s = {0.0, 0.0, 0.0, 0.0};
    for (int64_t q = 0; q < slots; ++q) {
      const double2 v = ghat[(first + q) * n * rows + (size_t)j * rows + i];
      if (plain) {
        s.hr += v.x;
        s.hi += v.y;
      } else {
        dd_accumulate(s, v.x, v.y);
      }
    }
    const double mr = ldexp(s.hr, -(n - 1)) + ldexp(s.lr, -(n - 1));
    const double mi = ldexp(s.hi, -(n - 1)) + ldexp(s.li, -(n - 1));
    // g * conj(M)
    grad[mat * n * n + e] = make_double2(g.x * mr + g.y * mi, g.y * mr - g.x * mi);
  }
  if (pout && threadIdx.x == 0) {
    dd2 s = {0.0, 0.0, 0.0, 0.0};
    for (int64_t q = 0; q < slots; ++q) {
      const double4 v = fparts[first + q];
      if (plain) {
        s.hr += v.x;
        s.hi += v.z;
      } else {
        s = dd_add(s, dd2{v.x, v.y, v.z, v.w});
      }
    }
    pout[mat] = make_double2(ldexp(s.hr, -(n - 1)) + ldexp(s.lr, -(n - 1)),
                             ldexp(s.hi, -(n - 1)) + ldexp(s.li, -(n - 1)));
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

template <int M>
static const void* grad_kernel() {
  return (const void*)&k_grad<M>;
}

static const void* grad_kernel_for(int m) {
  switch (m) {
    case 1: return grad_kernel<1>();
    case 2: return grad_kernel<2>();
    case 3: return grad_kernel<3>();
    case 4: return grad_kernel<4>();
    case 5: return grad_kernel<5>();
    case 6: return grad_kernel<6>();
    case 7: return grad_kernel<7>();
    case 8: return grad_kernel<8>();
  }
  return nullptr;
}

static int grad_K(int m) { return PH_GRAD_K(m); }

// Enqueue the gradient of `batch` n x n matrices (device pointers).
int perm_grad_launch(const double2* A, int n, int64_t batch, const double2* gout, double2* pout, double2* grad,
                     const Opts& o, hipStream_t st, int cus) {
  if (batch == 0) return PH_OK;
  hipError_t e;
  if (n == 1) {
    hipLaunchKernelGGL(k_grad_n1, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, st, A, batch, gout, pout,
                       grad);
    e = hipGetLastError();
    return e == hipSuccess ? PH_OK : hip_fail(e, "grad launch");
  }
  const int M = (n + 3) / 4, K = grad_K(M), rows = 4 * M, nb = n - 1;
  int c = o.chunk_log2 > 0 ? o.chunk_log2 : std::min(10, nb - 4);
  c = std::max(K, std::min(c, nb));
  const int64_t nsuper = (int64_t)((((uint64_t)1 << (nb - c)) + 15) / 16);
  const void* kern = grad_kernel_for(M);
  const size_t lds = (size_t)n * rows * sizeof(double2) + 4 * 64 * (size_t)(M | 1) * sizeof(double2);
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, lds);
  if (e != hipSuccess) return hip_fail(e, "occupancy");
  per_cu = std::max(1, per_cu);
  if (o.waves > 0) per_cu = std::min(per_cu, o.waves);
  const int64_t blocks_full = (int64_t)cus * per_cu;
  // slices per matrix: about four units per resident workgroup, at least one
  // super-chunk per wavefront of a unit
  int64_t s_per = std::max<int64_t>(1, (4 * blocks_full + batch - 1) / batch);
  s_per = std::min<int64_t>(s_per, std::max<int64_t>(1, nsuper / 4));
  const int64_t units = batch * s_per;
  const size_t tab_elems = (size_t)batch * n * rows;
  const size_t ghat_elems = (size_t)units * 4 * n * rows;
  const size_t off_g = ((tab_elems * sizeof(double2)) + 255) & ~(size_t)255;
  const size_t off_f = off_g + (((ghat_elems * sizeof(double2)) + 255) & ~(size_t)255);
  const size_t off_c = off_f + (((size_t)units * 4 * sizeof(double4) + 255) & ~(size_t)255);
  void* ws = nullptr;
  int rc = workspace(st, off_c + 256, &ws);
  if (rc) return rc;
  char* base = static_cast<char*>(ws);
  GradArgs ga;
  ga.tabs = reinterpret_cast<double2*>(base);
  ga.n = n;
  ga.c = c;
  ga.nsuper = nsuper;
  ga.s_per = (int)s_per;
  ga.units = units;
  ga.counter = reinterpret_cast<uint32_t*>(base + off_c);
  ga.ghat = reinterpret_cast<double2*>(base + off_g);
  ga.fparts = reinterpret_cast<double4*>(base + off_f);
  ga.plain = o.plain ? 1 : 0;
  hipLaunchKernelGGL(k_reset1, dim3(1), dim3(1), 0, st, ga.counter);
  hipLaunchKernelGGL(k_grad_prep, dim3((unsigned)batch), dim3(256), 0, st, A, n, rows,
                     const_cast<double2*>(ga.tabs));
  const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(blocks_full, units));
  void* args[] = {&ga};
  e = hipLaunchKernel(kern, dim3((unsigned)grid), dim3(256), args, lds, st);
  if (e != hipSuccess) return hip_fail(e, "grad sweep launch");
  hipLaunchKernelGGL(k_grad_finalize, dim3((unsigned)batch), dim3(256), 0, st, ga.ghat, ga.fparts, n, rows,
                     (int)s_per, ga.plain, gout, pout, grad);
  e = hipGetLastError();
  return e == hipSuccess ? PH_OK : hip_fail(e, "grad launch");
}

}  // namespace ph

using namespace ph;

extern "C" int ph_perm_grad(const ph_c128* A, int32_t n, int64_t batch, const ph_c128* grad_out, ph_c128* perm_out,
                            ph_c128* grad_A, const ph_opts* opt, void* stream) {
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
