// Host-only helpers shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "permhip.h"

namespace ph {

struct Opts {
  int algo = 0;        // PH_GLYNN / PH_RYSER
  bool plain = false;  // plain binary64 outer sum instead of double-double
  int chunk_log2 = 0;  // 0 = library choice
  int waves = 0;       // waves per SIMD, 0 = occupancy limit
};

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int read_opts(const ph_opts* o, Opts* r);
int workspace(hipStream_t st, size_t bytes, void** out);
int workspace_slot(hipStream_t st, size_t bytes, int slot, void** out);
int num_cus();
int gray_bits(int n, int algo);
int min_chunk_log2(int nb);
int pick_chunk_log2(int n, int algo, int requested);
int perm_single(const double2* A, int n, int64_t lda, double2* out, const Opts& o, hipStream_t st, int cus);

}  // namespace ph
