// Single-matrix sweep kernels, one instance per (n, algorithm).
//
// This file is compiled once per size range (-DPH_NLO=.. -DPH_NHI=..) so that
// the instances build in parallel; each compilation exports one lookup
// function ph_single_kernel_<lo>_<hi>(n, algo) returning the kernel handle.
//
// Work split: the launch covers the C chunks [chunk0, chunk0 + C) of length
// 2^c (all 2^nb / 2^c of them for a whole permanent, a contiguous share of
// them for one part of a sharded sum).  They are grouped in "super-chunks" of
// 64 consecutive chunks (one per lane of a wavefront; 32 for n >= PAIR_NMIN,
// where two lanes share a chunk, see sweep_pair.hpp).  Wave w of the grid
// takes the contiguous super-chunk range [S w / W, S (w+1) / W),
// S = ceil(C / 64), keeps a double-double (or plain) accumulator per lane
// across all of it, and writes one partial per wave -- the per-process
// contiguous ranges and final reduce of the parallel listings, mapped to
// wavefronts.
#include "sweep.hpp"
#include "sweep_pair.hpp"
#include "ph_internal.hpp"

#ifndef PH_NLO
#error "define PH_NLO and PH_NHI"
#endif

namespace ph {

template <int N, int ALGO>
__global__ __launch_bounds__(256) void k_sweep_single(const double2* __restrict__ a, int64_t lda, int c, uint64_t chunk0,
                                                      uint64_t nchunks, double4* __restrict__ partials, int plain) {
  const int lane = threadIdx.x & 63;
  const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const uint32_t nwaves = gridDim.x * (blockDim.x >> 6);
  extern __shared__ double2 lds_tab[];
  dd2 acc = {0.0, 0.0, 0.0, 0.0};
  if constexpr (N >= PAIR_NMIN) {
    // two lanes per chunk: super-chunks of 32 chunks
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
      sweep_chunk_pair<N, ALGO, true>((chunk0 + chunk) << c, c, res, Tl, upper, acc, plain != 0,
                                      chunk < nchunks && !upper);
    }
  } else {
    const uint64_t nsuper = (nchunks + 63) >> 6;
    const uint64_t s0 = nsuper * wave / nwaves;
    const uint64_t s1 = nsuper * (wave + 1) / nwaves;
    stage_table<N, ALGO>(lds_tab, a, lda);
    // The steps whose update column is not resident read a staged column
    // instead of one LDS entry per row at the step.  n = 24..32 (two waves
    // per SIMD already) stage the block boundaries in spare registers;
    // n = 33..44 keep one resident column fewer and its registers hold the
    // staged one (n = 40 2.0%, n = 42 and 44 6.3-6.6% faster); n = 45..48
    // keep none, every step reading the staged column (5-7% faster than two
    // lanes per term).  n <= 23 would lose a wave per SIMD to the extra
    // registers.
    constexpr int DF = Shape<N, ALGO>::D;
    constexpr bool STG = N >= 24 && (DF >= 1 || N > DPP_NMAX);
    Resident<N, ALGO, (STG && N >= 33) ? DF - 1 : DF> res;
    res.load(lds_tab);
    for (uint64_t s = s0; s < s1; ++s) {
      const uint64_t chunk = (s << 6) + lane;
      sweep_chunk<N, ALGO, decltype(res)::D, STG>((chunk0 + chunk) << c, c, res, lds_tab, acc, plain != 0,
                                                   chunk < nchunks);
    }
  }
  acc = wave_reduce(acc, plain != 0);
  if (lane == 0) partials[wave] = make_double4(acc.hr, acc.lr, acc.hi, acc.li);
}

template <int N>
static const void* pick(int algo) {
  return algo == ALGO_GLYNN ? (const void*)&k_sweep_single<N, ALGO_GLYNN>
                            : (const void*)&k_sweep_single<N, ALGO_RYSER>;
}

template <int... Is>
static const void* lookup(int n, int algo, std::integer_sequence<int, Is...>) {
  const void* out = nullptr;
  ((n == PH_NLO + Is ? (out = pick<PH_NLO + Is>(algo), 0) : 0), ...);
  return out;
}

}  // namespace ph

#define PH_CAT2(a, b, c) a##b##_##c
#define PH_CAT(a, b, c) PH_CAT2(a, b, c)

const void* PH_CAT(ph_single_kernel_, PH_NLO, PH_NHI)(int n, int algo) {
  return ph::lookup(n, algo, std::make_integer_sequence<int, PH_NHI - PH_NLO + 1>{});
}
