// Table builder (staging of A) and final reduction kernels.
#include "dd.hpp"
#include "ph_internal.hpp"
#include "sweep.hpp"

namespace ph {

// Staging for the batched sweeps: the n-column table (table_entry in
// sweep.hpp) of each matrix, stored column-major in the plan's table memory.
__device__ __forceinline__ void prep_one(const double2* __restrict__ a, int64_t lda, int n, int algo,
                                         double2* __restrict__ tab, int e) {
  const int i = e / n, j = e % n;  // row-major read
  tab[(size_t)j * n + i] = table_entry(a, lda, algo, i, j);
}

__global__ void k_prep_batched(const MatDesc* __restrict__ mats, const double2* __restrict__ a_base, int algo) {
  const MatDesc m = mats[blockIdx.x];
  for (int e = threadIdx.x; e < m.n * m.n; e += blockDim.x) prep_one(a_base + m.a_off, m.lda, m.n, algo, m.tab, e);
}

__global__ void k_reset(uint32_t* __restrict__ counters, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) counters[i] = 0;
}

// Fixed-order reduction of partials [begin, end) by one block of 64, 128 or
// 256 threads: thread t sums a contiguous slice in index order, each wavefront
// adds its lanes' sums in a fixed butterfly (no barrier), and the wavefront
// totals are added in wavefront order, so the result depends only on the
// partials and the block size.  The total is returned to every thread.
__device__ dd2 reduce_range(const double4* __restrict__ p, int64_t begin, int64_t end, int plain) {
  __shared__ dd2 wsum[4];
  const int t = threadIdx.x, nt = blockDim.x;
  const int64_t cnt = end - begin;
  const int64_t b0 = begin + cnt * t / nt, b1 = begin + cnt * (t + 1) / nt;
  dd2 acc = {0.0, 0.0, 0.0, 0.0};
  // the loads of a group of U partials are all issued before the first add
  // (one memory round trip per group, not per partial); the adds keep the
  // order q = b0, b0 + 1, ...
  constexpr int U = 4;
  for (int64_t q0 = b0; q0 < b1; q0 += U) {
    double4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (q0 + u < b1) v[u] = p[q0 + u];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (q0 + u >= b1) break;
      if (plain) {
        acc.hr += v[u].x;
        acc.hi += v[u].z;
      } else {
        acc = dd_add(acc, dd2{v[u].x, v[u].y, v[u].z, v[u].w});
      }
    }
  }
  acc = wave_reduce(acc, plain != 0);
  if ((t & 63) == 0) wsum[t >> 6] = acc;  // lane 0's total
  __syncthreads();
  dd2 s = wsum[0];
  for (int w = 1; w < (nt >> 6); ++w) {
    if (plain) {
      s.hr += wsum[w].hr;
      s.hi += wsum[w].hi;
    } else {
      s = dd_add(s, wsum[w]);
    }
  }
  return s;
}

// The reduced sum, then the formula's scale: 2^-(n-1) (BB/FG, exact on both
// halves of the double-double) or (-1)^n (Ryser), and a single rounding to
// complex128.
__device__ void finalize_range(const double4* __restrict__ p, int64_t begin, int64_t end, int n, int algo,
                               int plain, double2* __restrict__ out) {
  const dd2 s = reduce_range(p, begin, end, plain);
  if (threadIdx.x == 0) {
    double2 r;
    if (n == 0) {
      r = make_double2(1.0, 0.0);  // permanent of the empty matrix
    } else if (algo == ALGO_GLYNN) {
      r.x = ldexp(s.hr, -(n - 1)) + ldexp(s.lr, -(n - 1));
      r.y = ldexp(s.hi, -(n - 1)) + ldexp(s.li, -(n - 1));
    } else {
      const double sg = (n & 1) ? -1.0 : 1.0;
      r.x = sg * (s.hr + s.lr);
      r.y = sg * (s.hi + s.li);
    }
    *out = r;
  }
}

__global__ void k_finalize_single(const double4* __restrict__ p, int64_t nparts, int n, int algo, int plain,
                                  double2* __restrict__ out) {
  finalize_range(p, 0, nparts, n, algo, plain, out);
}

// One unscaled double-double {re_hi, re_lo, im_hi, im_lo} from the per-wave
// partials of a share of the Gray-code range.
__global__ void k_reduce_partials(const double4* __restrict__ p, int64_t nparts, int plain,
                                  double4* __restrict__ out) {
  const dd2 s = reduce_range(p, 0, nparts, plain);
  if (threadIdx.x == 0) *out = make_double4(s.hr, s.lr, s.hi, s.li);
}

__global__ void k_finalize_batched(const MatDesc* __restrict__ mats, const double4* __restrict__ p, int algo,
                                   int plain, double2* __restrict__ out) {
  const MatDesc m = mats[blockIdx.x];
  finalize_range(p, m.part_begin, m.part_end, m.n, algo, plain, out + m.out_index);
}

void launch_finalize_single(const double4* partials, int64_t nparts, int n, int algo, int plain, double2* out,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_finalize_single, dim3(1), dim3(256), 0, st, partials, nparts, n, algo, plain, out);
}

void launch_reduce_partials(const double4* partials, int64_t nparts, int plain, double4* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, st, partials, nparts, plain, out);
}

// Deterministic bounded values for timing runs (no meaning beyond that).
__global__ void k_fill_synthetic(double2* a, int64_t count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) {
    const uint64_t h = (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
    a[i] = make_double2((double)((h >> 11) & 1023) / 2048.0 - 0.25, (double)((h >> 31) & 1023) / 2048.0 - 0.25);
  }
}

void launch_fill_synthetic(double2* a, int64_t count, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fill_synthetic, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, a, count);
}

const void* prep_batched_kernel() { return (const void*)&k_prep_batched; }
const void* finalize_batched_kernel() { return (const void*)&k_finalize_batched; }
const void* reset_kernel() { return (const void*)&k_reset; }

const void* batched_kernel(int bucket, int algo) {
  switch (bucket) {
    case 0: return ph_batched_kernel_1_16(algo);
    case 1: return ph_batched_kernel_17_24(algo);
    case 2: return ph_batched_kernel_25_32(algo);
    case 3: return ph_batched_kernel_33_40(algo);
    case 4: return ph_batched_kernel_41_44(algo);
    case 5: return ph_batched_kernel_45_52(algo);
  }
  return nullptr;
}

const void* single_kernel(int n, int algo) {
  if (n >= 1 && n <= 16) return ph_single_kernel_1_16(n, algo);
  if (n <= 24) return ph_single_kernel_17_24(n, algo);
  if (n <= 32) return ph_single_kernel_25_32(n, algo);
  if (n <= 40) return ph_single_kernel_33_40(n, algo);
  if (n <= 44) return ph_single_kernel_41_44(n, algo);
  if (n <= 52) return ph_single_kernel_45_52(n, algo);
  return nullptr;
}

}  // namespace ph
