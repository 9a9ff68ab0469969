// Host-only helpers shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <vector>

#include "permhip.h"

namespace ph {

struct Opts {
  int algo = 0;        // PH_GLYNN / PH_RYSER
  bool plain = false;  // plain binary64 outer sum instead of double-double
  int chunk_log2 = 0;  // 0 = library choice
  int waves = 0;       // waves per SIMD, 0 = occupancy limit
  bool ungrouped = false;  // boson probabilities: no multiplicity grouping
  bool unsorted = false;   // boson samples: placement order
  bool du_full = false;    // boson gradient: m x m dU, photons folded onto U's columns
};

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int read_opts(const ph_opts* o, Opts* r);
int workspace(hipStream_t st, size_t bytes, void** out);
// Workspace slots: each call keeps its buffers in its own slot, so that a
// call composed of others (the boson layer over the gradient sweep, the
// sampler over the row minors) never has a buffer it still needs grown
// (reallocated) under it.
enum WsSlot {
  WS_SWEEP = 0,          // partial sums of the one-matrix and gradient sweeps
  WS_BOSON = 1,          // ungrouped boson layer
  WS_BOSON_GROUPED = 2,  // multiplicity-grouped boson layer
  WS_GRAD_TABLES = 3,    // gradient-sweep tables
  WS_SAMPLER = 4,        // sampler state
  WS_MINORS = 5,         // row-minor partial sums
  WS_MINORS_TABLES = 6,  // row-minor tables
  WS_BOSON_FOLD = 7      // per-photon boson gradient before the fold onto U's columns
};
// fresh (nullable) tells whether the buffer was (re)allocated by this call
int workspace_slot(hipStream_t st, size_t bytes, int slot, void** out, bool* fresh = nullptr);
int num_cus();
// resident 256-thread workgroups per CU of kern with lds bytes of dynamic LDS
int resident_per_cu(const void* kern, size_t lds, int* per_cu);
int gray_bits(int n, int algo);
int min_chunk_log2(int nb);
int pick_chunk_log2(int n, int algo, int requested);
int perm_single(const double2* A, int n, int64_t lda, double2* out, const Opts& o, hipStream_t st, int cus);

// One-matrix sweep launches (permhip.cpp).
struct SweepGeom {
  const void* kern = nullptr;
  size_t lds = 0;
  uint64_t blocks = 0;  // workgroups of 256 threads; 4 partials each
};
int single_geometry(int n, const Opts& o, int cus, uint64_t nchunks, SweepGeom* g);
int launch_single(const SweepGeom& g, const double2* A, int64_t lda, int c, uint64_t chunk0, uint64_t nchunks,
                  int plain, double4* parts, hipStream_t st);

// rocTX range for the lifetime of the object when PERMHIP_ROCTX=1 (trace.cpp).
struct TraceRange {
  explicit TraceRange(const char* name);
  ~TraceRange();
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
  bool on = false;
};
#define PH_TRACE(name) ::ph::TraceRange ph_trace_range_(name)

// Host arrays copied to device memory in one transfer through a per-stream
// pinned staging buffer (boson.hip): piece q lands at dst + the sum of the
// previous pieces' sizes, each rounded up to 256 bytes.  Returns before the
// copy completes; the host arrays may be reused at once.
struct Piece {
  const void* src;
  size_t bytes;
};
int upload(hipStream_t st, void* dst, const Piece* pc, int npc);

// Gradient sweep of `batch` contiguous n x n matrices (grad.hip).
int perm_grad_launch(const double2* A, int n, int64_t batch, const double2* gout, double2* pout, double2* grad,
                     const Opts& o, hipStream_t st, int cus);

// Batched sweep over caller-built tables (plan.cpp).
struct PlanImpl;
double2* plan_table(PlanImpl* p, int64_t b);
double2* plan_tables_base(PlanImpl* p);
const std::vector<int64_t>& plan_table_offsets(PlanImpl* p);
int plan_exec(PlanImpl* p, const double2* a, double2* out, hipStream_t st);
int plan_ext_run(const int32_t* n_host, const int32_t* ncols_host, int64_t batch, const Opts& o, hipStream_t st,
                 const std::function<int(PlanImpl*)>& fill, double2* out);

}  // namespace ph
