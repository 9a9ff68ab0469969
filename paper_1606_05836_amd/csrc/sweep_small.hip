// Two lanes per term for the small orders of one-matrix calls
// (SMALL_PAIR_NMIN..SMALL_PAIR_NMAX), whose whole sweep takes microseconds.
//
// At the shortest chunk (16 terms) these orders have too few chunks to give
// every SIMD a wavefront with one lane per term (n = 20: 2^15 chunks, 512
// wavefronts for 1024 SIMDs), and each lane's seed and sweep are a serial
// chain of a few thousand instructions.  Splitting each term's rows over two
// lanes, as the two-lane walk of the largest orders does (sweep_pair.hpp),
// doubles the wavefronts and halves each lane's chain.  The launch and its
// partials are those of k_sweep_single: super-chunks of 32 chunks, one
// partial per wavefront, the same finalize.
#include <utility>

#include "ph_internal.hpp"
#include "sweep.hpp"
#include "sweep_pair.hpp"

namespace ph {

template <int N, int ALGO>
__global__ __launch_bounds__(256) void k_sweep_pair_small(const double2* __restrict__ a, int64_t lda, int c,
                                                          uint64_t chunk0, uint64_t nchunks,
                                                          double4* __restrict__ partials, int plain) {
  static_assert(Shape<N, ALGO>::LOGU == 4, "chunks of at least 16 terms");
  const int lane = threadIdx.x & 63;
  const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const uint32_t nwaves = gridDim.x * (blockDim.x >> 6);
  extern __shared__ double2 lds_tab[];
  dd2 acc = {0.0, 0.0, 0.0, 0.0};
  const bool upper = lane >= 32;
  const uint64_t nsuper = (nchunks + 31) >> 5;
  const uint64_t s0 = nsuper * wave / nwaves;
  const uint64_t s1 = nsuper * (wave + 1) / nwaves;
  stage_table_pair<N, ALGO>(lds_tab, a, lda);
  const double2* Tl = lds_tab + (upper ? PairShape<N, ALGO>::R : 0);
  ResidentPair<N, ALGO> res;
  res.load(Tl);
  for (uint64_t s = s0; s < s1; ++s) {
    const uint64_t chunk = (s << 5) + (lane & 31);
    sweep_chunk_pair<N, ALGO>((chunk0 + chunk) << c, c, res, Tl, upper, acc, plain != 0, chunk < nchunks && !upper);
  }
  acc = wave_reduce(acc, plain != 0);
  if (lane == 0) partials[wave] = make_double4(acc.hr, acc.lr, acc.hi, acc.li);
}

template <int N>
static const void* pick(int algo) {
  return algo == ALGO_GLYNN ? (const void*)&k_sweep_pair_small<N, ALGO_GLYNN>
                            : (const void*)&k_sweep_pair_small<N, ALGO_RYSER>;
}

template <int... Is>
static const void* lookup(int n, int algo, std::integer_sequence<int, Is...>) {
  const void* out = nullptr;
  ((n == SMALL_PAIR_NMIN + Is ? (out = pick<SMALL_PAIR_NMIN + Is>(algo), 0) : 0), ...);
  return out;
}

const void* small_pair_kernel(int n, int algo) {
  return lookup(n, algo, std::make_integer_sequence<int, SMALL_PAIR_NMAX - SMALL_PAIR_NMIN + 1>{});
}

}  // namespace ph
