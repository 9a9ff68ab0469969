// Internal declarations shared by the host library and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ph {

constexpr int NMAX = 52;       // largest n of the forward sweeps
constexpr int NMAX_GRAD = 32;  // largest n of the backward sweep

// Complex entries of the per-matrix table (n columns of n entries).
inline size_t table_elems(int n) { return (size_t)n * n; }

// Per-matrix descriptor used by the batched kernels (device memory).
struct MatDesc {
  const double2* a;    // input, row-major
  int64_t lda;         // row stride of a (elements)
  double2* tab;        // table (table_elems(n) complex entries)
  int32_t n;           // order
  int32_t c;           // log2 chunk length
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
// batched persistent kernels (sweep_batched.hip), by size bucket
const void* batched_kernel(int bucket, int algo);
int batched_bucket(int n);       // bucket index of an order n
int batched_bucket_count();
int batched_bucket_nmax(int bucket);

void launch_prep(const double2* a, int64_t lda, int n, int algo, double2* tab, hipStream_t st);
void launch_prep_batched(const MatDesc* mats, int nmat, int nmax, int algo, hipStream_t st);
void launch_finalize_single(const double4* partials, int64_t nparts, int n, int algo, int plain, double2* out,
                            hipStream_t st);
void launch_finalize_batched(const MatDesc* mats, int nmat, const double4* partials, int algo, int plain,
                             double2* out, hipStream_t st);

}  // namespace ph

#define PH_DECLARE_RANGE(lo, hi) const void* ph_single_kernel_##lo##_##hi(int n, int algo);
PH_DECLARE_RANGE(1, 16)
PH_DECLARE_RANGE(17, 24)
PH_DECLARE_RANGE(25, 32)
PH_DECLARE_RANGE(33, 40)
PH_DECLARE_RANGE(41, 46)
PH_DECLARE_RANGE(47, 52)
#undef PH_DECLARE_RANGE
