// Host side of the C ABI declared in include/permhip.h: argument checks,
// workspace, launch geometry, dispatch to the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "permhip.h"
#include "ph_host.hpp"
#include "ph_internal.hpp"

namespace ph {

// ------------------------------------------------------------------ errors

static thread_local std::string t_err = "no error";

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(PH_EHIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

// ------------------------------------------------------------------ devices

struct DevInfo {
  int cus = 0;
  std::string arch;
};

static std::mutex g_mu;
static std::map<int, DevInfo> g_dev;

int device_info(int* dev_out, DevInfo* info) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_dev.find(dev);
  if (it == g_dev.end()) {
    hipDeviceProp_t p;
    e = hipGetDeviceProperties(&p, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    DevInfo d;
    d.cus = p.multiProcessorCount;
    d.arch = p.gcnArchName;
    if (d.arch.rfind("gfx950", 0) != 0)
      return fail(PH_EUNSUPPORTED, "device %d is %s; this library is built for gfx950", dev, d.arch.c_str());
    it = g_dev.emplace(dev, d).first;
  }
  *dev_out = dev;
  *info = it->second;
  return PH_OK;
}

int num_cus() {
  int dev;
  DevInfo d;
  if (device_info(&dev, &d) != PH_OK) return 0;
  return d.cus;
}

// --------------------------------------------------------------- workspace

struct Buf {
  void* p = nullptr;
  size_t cap = 0;
};
static std::map<std::tuple<int, hipStream_t, int>, Buf> g_ws;

// Library-owned scratch for one (device, stream, slot); grown on demand.
// Work on one stream is ordered, so reuse across calls on that stream is
// safe.  The slots (WsSlot, ph_host.hpp) separate the callers' buffers.
int workspace_slot(hipStream_t st, size_t bytes, int slot, void** out, bool* fresh) {
  if (fresh) *fresh = false;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_mu);
  Buf& b = g_ws[{dev, st, slot}];
  if (b.cap < bytes) {
    if (b.p) {
      // the old buffer may still be in use by queued work on this stream
      e = hipStreamSynchronize(st);
      if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
      (void)hipFree(b.p);  // nothing queued uses it any more
      b.p = nullptr;
      b.cap = 0;
    }
    size_t cap = std::max(bytes, (size_t)1 << 20);
    e = hipMalloc(&b.p, cap);
    if (e != hipSuccess) return fail(PH_ENOMEM, "hipMalloc(%zu): %s", cap, hipGetErrorString(e));
    b.cap = cap;
    if (fresh) *fresh = true;
  }
  *out = b.p;
  return PH_OK;
}

int workspace(hipStream_t st, size_t bytes, void** out) { return workspace_slot(st, bytes, WS_SWEEP, out); }

// Workgroups of 256 threads with `lds` bytes of dynamic LDS that fit on one
// CU, asked of the runtime once per (kernel, LDS size) and kept: the answer
// follows from the kernel's registers and LDS on the one architecture the
// library runs on, and the query costs a small call more host time than the
// rest of its launch preparation.
int resident_per_cu(const void* kern, size_t lds, int* per_cu) {
  static std::mutex mu;
  static std::map<std::pair<const void*, size_t>, int> known;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = known.find({kern, lds});
    if (it != known.end()) {
      *per_cu = it->second;
      return PH_OK;
    }
  }
  int v = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, kern, 256, lds);
  if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
  std::lock_guard<std::mutex> lk(mu);
  known[{kern, lds}] = v;
  *per_cu = v;
  return PH_OK;
}

// ------------------------------------------------------------------ options

int read_opts(const ph_opts* o, Opts* r) {
  Opts d;
  if (!o) {
    // defaults; PERMHIP_ACCUM=plain|dd overrides the accumulation
    const char* acc = getenv("PERMHIP_ACCUM");
    if (acc && *acc) {
      if (!strcmp(acc, "plain")) d.plain = true;
      else if (strcmp(acc, "dd")) return fail(PH_EINVAL, "PERMHIP_ACCUM=%s (plain or dd)", acc);
    }
  }
  if (o) {
    if (o->algo != PH_GLYNN && o->algo != PH_RYSER) return fail(PH_EINVAL, "opts.algo=%d", o->algo);
    if (o->accum != PH_ACC_DD && o->accum != PH_ACC_PLAIN) return fail(PH_EINVAL, "opts.accum=%d", o->accum);
    if (o->chunk_log2 < 0) return fail(PH_EINVAL, "opts.chunk_log2=%d < 0", o->chunk_log2);
    if (o->waves < 0 || o->waves > 8) return fail(PH_EINVAL, "opts.waves=%d", o->waves);
    if ((o->flags & ~(PH_FLAG_UNGROUPED | PH_FLAG_UNSORTED | PH_FLAG_DU_FULL)) != 0)
      return fail(PH_EINVAL, "opts.flags=%u", o->flags);
    d.ungrouped = (o->flags & PH_FLAG_UNGROUPED) != 0;
    d.unsorted = (o->flags & PH_FLAG_UNSORTED) != 0;
    d.du_full = (o->flags & PH_FLAG_DU_FULL) != 0;
    d.algo = o->algo;
    d.plain = o->accum == PH_ACC_PLAIN;
    // longer chunks are clamped: the sweeps count steps inside a chunk in
    // 32-bit integers, and the row-sum drift grows with the chunk length
    d.chunk_log2 = std::min<int32_t>(o->chunk_log2, PH_CHUNK_LOG2_MAX);
    d.waves = o->waves;
  }
  *r = d;
  return PH_OK;
}

int gray_bits(int n, int algo) { return algo == PH_GLYNN ? n - 1 : n; }

int min_chunk_log2(int nb) { return nb >= 4 ? 4 : (nb >= 1 ? 1 : 0); }

// Chunk length: long enough to amortise the O(n^2) seed over the O(n) steps,
// short enough to leave work for every lane and to bound row-sum drift.  At
// most 2^12 terms, and at least 2^17 chunks where the range allows: one per
// lane of two 256-thread workgroups on each of 256 CUs, so that mid-size
// orders fill the chip instead of a few CUs.
int pick_chunk_log2(int n, int algo, int requested) {
  const int nb = gray_bits(n, algo);
  const int lo = min_chunk_log2(nb);
  int c = requested > 0 ? requested : std::min(12, nb - 17);
  return std::max(lo, std::min(c, nb));
}

}  // namespace ph

using namespace ph;

// ======================================================================= ABI

extern "C" const char* ph_last_error(void) { return t_err.c_str(); }

extern "C" int ph_version(void) { return 10000; }

extern "C" int ph_perm(const ph_c128* A, int32_t n, int64_t lda, ph_c128* out, const ph_opts* opt, void* stream) {
  PH_TRACE("ph_perm");
  Opts o;
  int rc = read_opts(opt, &o);
  if (rc) return rc;
  if (n < 0) return fail(PH_EINVAL, "n=%d < 0", n);
  if (n > PH_NMAX) return fail(PH_ERANGE, "n=%d > %d", n, PH_NMAX);
  if (!out) return fail(PH_EINVAL, "out is NULL");
  if (n > 0 && !A) return fail(PH_EINVAL, "A is NULL");
  if (n > 0 && lda < n) return fail(PH_EINVAL, "lda=%lld < n=%d", (long long)lda, n);
  int dev;
  DevInfo di;
  if ((rc = device_info(&dev, &di))) return rc;
  return perm_single(reinterpret_cast<const double2*>(A), n, lda, reinterpret_cast<double2*>(out), o,
                     (hipStream_t)stream, di.cus);
}

namespace ph {

// Launch shape of the one-matrix sweep over `nchunks` chunks: 256-thread
// workgroups, as many as can be resident (or as waves per SIMD asks), at most
// one per four super-chunks.
int single_geometry(int n, const Opts& o, int cus, uint64_t nchunks, SweepGeom* g) {
  // super-chunks of 64 chunks (one lane per term), or of 32 for the small
  // sweeps that take two lanes per term
  const bool pair = small_pair(n, nchunks);
  const uint64_t nsuper = pair ? (nchunks + 31) / 32 : (nchunks + 63) / 64;
  g->kern = pair ? small_pair_kernel(n, o.algo) : single_kernel(n, o.algo);
  if (!g->kern) return fail(PH_ERANGE, "no kernel for n=%d", n);
  g->lds = single_lds_bytes(n, pair || n >= PAIR_NMIN);
  int per_cu = 0;
  int rc = resident_per_cu(g->kern, g->lds, &per_cu);
  if (rc) return rc;
  if (per_cu < 1) return fail(PH_EHIP, "kernel for n=%d cannot be resident", n);
  if (o.waves > 0) per_cu = std::min(per_cu, o.waves);
  uint64_t blocks = (uint64_t)cus * per_cu;
  blocks = std::min<uint64_t>(blocks, (nsuper + 3) / 4);
  g->blocks = std::max<uint64_t>(blocks, 1);
  return PH_OK;
}

// Enqueue the sweep of the chunks [chunk0, chunk0 + nchunks) of length 2^c
// of one matrix: every workgroup builds the table from A in its LDS and each
// wave writes one partial to parts (4 * blocks of them).
int launch_single(const SweepGeom& g, const double2* A, int64_t lda, int c, uint64_t chunk0, uint64_t nchunks,
                  int plain, double4* parts, hipStream_t st) {
  const double2* a = A;
  int64_t ld = lda;
  int cc = c;
  uint64_t ch0 = chunk0, nch = nchunks;
  int pl = plain;
  void* args[] = {&a, &ld, &cc, &ch0, &nch, &parts, &pl};
  const hipError_t e = hipLaunchKernel(g.kern, dim3((unsigned)g.blocks), dim3(256), args, g.lds, st);
  return e == hipSuccess ? PH_OK : hip_fail(e, "sweep launch");
}

int perm_single(const double2* A, int n, int64_t lda, double2* out, const Opts& o, hipStream_t st, int cus) {
  hipError_t e;
  if (n == 0) {
    launch_finalize_single(nullptr, 0, 0, o.algo, o.plain, out, st);
    e = hipGetLastError();
    return e == hipSuccess ? PH_OK : hip_fail(e, "finalize launch");
  }
  const int nb = gray_bits(n, o.algo);
  const int c = pick_chunk_log2(n, o.algo, o.chunk_log2);
  const uint64_t nchunks = (uint64_t)1 << (nb - c);
  SweepGeom g;
  int rc = single_geometry(n, o, cus, nchunks, &g);
  if (rc) return rc;
  void* ws = nullptr;
  if ((rc = workspace(st, g.blocks * 4 * sizeof(double4), &ws))) return rc;
  double4* parts = static_cast<double4*>(ws);
  if ((rc = launch_single(g, A, lda, c, 0, nchunks, o.plain ? 1 : 0, parts, st))) return rc;
  launch_finalize_single(parts, (int64_t)g.blocks * 4, n, o.algo, o.plain, out, st);
  e = hipGetLastError();
  return e == hipSuccess ? PH_OK : hip_fail(e, "finalize launch");
}

}  // namespace ph

extern "C" int ph_perm_chunk_log2(int32_t n, const ph_opts* opt, int32_t* out) {
  Opts o;
  int rc = read_opts(opt, &o);
  if (rc) return rc;
  if (n < 1) return fail(PH_EINVAL, "n=%d < 1", n);
  if (n > PH_NMAX) return fail(PH_ERANGE, "n=%d > %d", n, PH_NMAX);
  if (!out) return fail(PH_EINVAL, "out is NULL");
  *out = pick_chunk_log2(n, o.algo, o.chunk_log2);
  return PH_OK;
}

extern "C" int ph_perm_partial(const ph_c128* A, int32_t n, int64_t lda, uint64_t k_begin, uint64_t k_end,
                               double* partial, const ph_opts* opt, void* stream) {
  PH_TRACE("ph_perm_partial");
  Opts o;
  int rc = read_opts(opt, &o);
  if (rc) return rc;
  if (n < 1) return fail(PH_EINVAL, "n=%d < 1", n);
  if (n > PH_NMAX) return fail(PH_ERANGE, "n=%d > %d", n, PH_NMAX);
  if (!partial) return fail(PH_EINVAL, "partial is NULL");
  if (!A) return fail(PH_EINVAL, "A is NULL");
  if (lda < n) return fail(PH_EINVAL, "lda=%lld < n=%d", (long long)lda, n);
  const int nb = gray_bits(n, o.algo);
  const int c = pick_chunk_log2(n, o.algo, o.chunk_log2);
  const uint64_t total = (uint64_t)1 << nb, mask = ((uint64_t)1 << c) - 1;
  if (k_begin > k_end || k_end > total)
    return fail(PH_EINVAL, "term range [%llu, %llu) outside [0, 2^%d)", (unsigned long long)k_begin,
                (unsigned long long)k_end, nb);
  if ((k_begin & mask) || (k_end & mask))
    return fail(PH_EINVAL, "term range [%llu, %llu) not aligned to the chunk length 2^%d",
                (unsigned long long)k_begin, (unsigned long long)k_end, c);
  int dev;
  DevInfo di;
  if ((rc = device_info(&dev, &di))) return rc;
  hipStream_t st = (hipStream_t)stream;
  double4* out = reinterpret_cast<double4*>(partial);
  double4* parts = nullptr;
  int64_t nparts = 0;
  if (k_end > k_begin) {
    const uint64_t nchunks = (k_end - k_begin) >> c;
    SweepGeom g;
    if ((rc = single_geometry(n, o, di.cus, nchunks, &g))) return rc;
    void* ws = nullptr;
    if ((rc = workspace(st, g.blocks * 4 * sizeof(double4), &ws))) return rc;
    parts = static_cast<double4*>(ws);
    nparts = (int64_t)g.blocks * 4;
    rc = launch_single(g, reinterpret_cast<const double2*>(A), lda, c, k_begin >> c, nchunks, o.plain ? 1 : 0, parts,
                       st);
    if (rc) return rc;
  }
  launch_reduce_partials(parts, nparts, o.plain ? 1 : 0, out, st);  // zero for an empty range
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? PH_OK : hip_fail(e, "kernel launch");
}

extern "C" int ph_perm_combine(const double* partials, int64_t count, int32_t n, ph_c128* out, const ph_opts* opt,
                               void* stream) {
  PH_TRACE("ph_perm_combine");
  Opts o;
  int rc = read_opts(opt, &o);
  if (rc) return rc;
  if (n < 1) return fail(PH_EINVAL, "n=%d < 1", n);
  if (n > PH_NMAX) return fail(PH_ERANGE, "n=%d > %d", n, PH_NMAX);
  if (count < 0) return fail(PH_EINVAL, "count=%lld < 0", (long long)count);
  if (count > 0 && !partials) return fail(PH_EINVAL, "partials is NULL");
  if (!out) return fail(PH_EINVAL, "out is NULL");
  int dev;
  DevInfo di;
  if ((rc = device_info(&dev, &di))) return rc;
  launch_finalize_single(reinterpret_cast<const double4*>(partials), count, n, o.algo, o.plain,
                         reinterpret_cast<double2*>(out), (hipStream_t)stream);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? PH_OK : hip_fail(e, "kernel launch");
}
