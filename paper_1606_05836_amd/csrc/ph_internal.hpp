// Internal declarations shared by the host library and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ph {

constexpr int NMAX = 52;       // largest n of the forward sweeps
constexpr int NMAX_GRAD = 32;  // largest n of the backward sweep

// Complex entries of the per-matrix table (n columns of n entries; a table
// with ncols < n columns uses the first ncols * n of them).
inline size_t table_elems(int n) { return (size_t)n * n; }
// The one-matrix sweep takes two lanes per term from n = PAIR_NMIN on: below,
// the n row sums fit one lane's registers next to the update columns (at
// n = 45..48 a single staged column, every step reading it; sweep_single.hip),
// and one lane per term issues fewer instructions (no cross-lane product).
constexpr int PAIR_NMIN = 49;

// Small one-matrix sweeps take two lanes per term although one lane would
// fit: with at most 2^15 chunks, one lane per chunk leaves SIMDs without a
// wavefront, and two lanes halve each lane's serial chain (sweep_small.hip).
// With more chunks one lane per term fills the chip and is faster.
constexpr int SMALL_PAIR_NMIN = 12, SMALL_PAIR_NMAX = 21;
constexpr uint64_t SMALL_PAIR_MAX_CHUNKS = (uint64_t)1 << 15;
inline bool small_pair(int n, uint64_t nchunks) {
  return n >= SMALL_PAIR_NMIN && n <= SMALL_PAIR_NMAX && nchunks <= SMALL_PAIR_MAX_CHUNKS;
}

// LDS table of the one-matrix sweep: n columns of n rows, or of 2 ceil(n/2)
// rows when two lanes share a term
inline size_t single_lds_bytes(int n, bool pair) {
  return (size_t)n * (pair ? 2 * ((n + 1) / 2) : n) * 16;
}

// Per-matrix descriptor used by the batched kernels (device memory).
struct MatDesc {
  int64_t a_off;       // offset of the input (row-major, contiguous) in the packed batch
  int64_t lda;         // row stride of the input (elements)
  double2* tab;        // table (table_elems(n) complex entries)
  int32_t n;           // order (rows)
  int32_t c;           // log2 chunk length
  int32_t ncols;       // columns the sweep walks (n, or fewer for a caller-built table)
  int32_t reserved;
  int64_t part_begin;  // first partial slot of this matrix
  int64_t part_end;    // one past the last
  int64_t out_index;   // position of the result in the caller's output
};

// One wavefront's work item in a batched launch: super-chunks
// [super0, super0 + rounds) of matrix `mat` (64 chunks per super-chunk).
struct WorkItem {
  int32_t mat;
  int32_t rounds;
  int64_t super0;
};

// size-range kernel lookups (sweep_single.hip compiled once per range)
const void* single_kernel(int n, int algo);
const void* small_pair_kernel(int n, int algo);  // SMALL_PAIR_NMIN <= n <= SMALL_PAIR_NMAX
// batched persistent kernels (sweep_batched.hip), one per size bucket
constexpr int NBUCKETS = 6;
constexpr int BUCKET_LO[NBUCKETS] = {1, 17, 25, 33, 41, 45};
constexpr int BUCKET_HI[NBUCKETS] = {16, 24, 32, 40, 44, 52};
inline int bucket_of(int n) {
  for (int b = 0; b < NBUCKETS; ++b)
    if (n >= BUCKET_LO[b] && n <= BUCKET_HI[b]) return b;
  return -1;
}
const void* batched_kernel(int bucket, int algo);

const void* prep_batched_kernel();      // k_prep_batched(mats, a_base, algo)
const void* finalize_batched_kernel();  // k_finalize_batched(mats, partials, algo, plain, out)
const void* reset_kernel();             // k_reset(counters, count)
void launch_fill_synthetic(double2* a, int64_t count, hipStream_t st);
void launch_finalize_single(const double4* partials, int64_t nparts, int n, int algo, int plain, double2* out,
                            hipStream_t st);
void launch_reduce_partials(const double4* partials, int64_t nparts, int plain, double4* out, hipStream_t st);

}  // namespace ph

#define PH_DECLARE_RANGE(lo, hi) const void* ph_single_kernel_##lo##_##hi(int n, int algo);
PH_DECLARE_RANGE(1, 16)
PH_DECLARE_RANGE(17, 24)
PH_DECLARE_RANGE(25, 32)
PH_DECLARE_RANGE(33, 40)
PH_DECLARE_RANGE(41, 44)
PH_DECLARE_RANGE(45, 52)
#undef PH_DECLARE_RANGE
#define PH_DECLARE_BUCKET(lo, hi) const void* ph_batched_kernel_##lo##_##hi(int algo);
PH_DECLARE_BUCKET(1, 16)
PH_DECLARE_BUCKET(17, 24)
PH_DECLARE_BUCKET(25, 32)
PH_DECLARE_BUCKET(33, 40)
PH_DECLARE_BUCKET(41, 44)
PH_DECLARE_BUCKET(45, 52)
#undef PH_DECLARE_BUCKET
