// Batched permanents: one persistent kernel per size bucket [PH_NLO, PH_NHI].
//
// The plan (host) sorts matrices by n, largest first, and cuts each matrix's
// Gray range into work items of up to four super-chunks (64 chunks each, one
// chunk per lane).  A workgroup of four wavefronts claims items with an
// integer atomic counter, stages the item's matrix table into LDS, and each
// wavefront sweeps one super-chunk of it with the same code as the
// single-matrix kernel (sweep.hpp), selected by n through a switch over the
// bucket's compile-time sizes.  Every (item, wavefront) pair owns one partial
// slot, so the fixed-order finalize makes the result independent of which
// workgroup ran which item.
//
// Compiled once per bucket (-DPH_NLO, -DPH_NHI); exports
// ph_batched_kernel_<lo>_<hi>(algo).
#include "ph_internal.hpp"
#include "sweep.hpp"

#ifndef PH_NLO
#error "define PH_NLO and PH_NHI"
#endif

namespace ph {

constexpr int BATCHED_DPP_NMAX = 40;

template <int N, int ALGO>
__device__ __forceinline__ void run_item(const double2* lds, int c, int ncols, const WorkItem& w, int64_t slot,
                                         double4* __restrict__ partials, int plain) {
  using S = Shape<N, ALGO>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nb = ALGO == ALGO_GLYNN ? ncols - 1 : ncols;
  const uint64_t nchunks = (uint64_t)1 << (nb - c);
  // the item loop keeps extra state live: above n = 32 at most 3 resident
  // columns, above n = BATCHED_DPP_NMAX every column comes from LDS
  constexpr int DR = N > BATCHED_DPP_NMAX ? 0 : (N > 32 && S::D > 3 ? 3 : S::D);
  // n = 17..32: the block boundaries read a staged column (above n = 32 the
  // staged column does not fit next to the item loop's state)
  constexpr bool STG = N >= 17 && N <= 32;
  Resident<N, ALGO, DR> res;
  res.load(lds);
  dd2 acc = {0.0, 0.0, 0.0, 0.0};
  for (int r = wave; r < w.rounds; r += 4) {
    const uint64_t chunk = ((uint64_t)(w.super0 + r) << 6) + lane;
    sweep_chunk<N, ALGO, DR, STG>(chunk << c, c, res, lds, acc, plain != 0, chunk < nchunks, ncols);
  }
  acc = wave_reduce(acc, plain != 0);
  if (lane == 0) partials[slot * 4 + wave] = make_double4(acc.hr, acc.lr, acc.hi, acc.li);
}

template <int NLO, int ALGO, int... Is>
__device__ __forceinline__ void dispatch(int n, const double2* lds, int c, int ncols, const WorkItem& w, int64_t slot,
                                         double4* partials, int plain, std::integer_sequence<int, Is...>) {
  ((n == NLO + Is ? (run_item<NLO + Is, ALGO>(lds, c, ncols, w, slot, partials, plain), 0) : 0), ...);
}

// Templated on the bucket bounds so that each compilation defines distinct
// symbols.
template <int NLO, int NHI, int ALGO>
__global__ __launch_bounds__(256) void k_sweep_batched(const MatDesc* __restrict__ mats,
                                                       const WorkItem* __restrict__ items, int64_t item_begin,
                                                       int64_t item_end, uint32_t* __restrict__ counter,
                                                       double4* __restrict__ partials, int plain) {
  extern __shared__ double2 lds_tab[];
  __shared__ int64_t s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = item_begin + (int64_t)atomicAdd(counter, 1u);
    __syncthreads();
    const int64_t it = s_item;
    if (it >= item_end) break;
    const WorkItem w = items[it];
    const MatDesc m = mats[w.mat];
    for (int e = threadIdx.x; e < m.n * m.ncols; e += blockDim.x) lds_tab[e] = m.tab[e];
    __syncthreads();
    dispatch<NLO, ALGO>(m.n, lds_tab, m.c, m.ncols, w, it, partials, plain,
                        std::make_integer_sequence<int, NHI - NLO + 1>{});
    __syncthreads();  // LDS and s_item are reused by the next item
  }
}

}  // namespace ph

#define PH_CAT2(a, b, c) a##b##_##c
#define PH_CAT(a, b, c) PH_CAT2(a, b, c)

const void* PH_CAT(ph_batched_kernel_, PH_NLO, PH_NHI)(int algo) {
  return algo == ph::ALGO_GLYNN ? (const void*)&ph::k_sweep_batched<PH_NLO, PH_NHI, ph::ALGO_GLYNN>
                                : (const void*)&ph::k_sweep_batched<PH_NLO, PH_NHI, ph::ALGO_RYSER>;
}
