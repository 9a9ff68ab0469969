// ph_perm_noalloc: the one-matrix permanent of ph_perm without any device
// allocation, for callers that cannot allocate (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// ph_perm keeps its per-wave partial sums in library workspace grown with
// hipMalloc.  Here they live in one file-scope device array, `scratch`, of a
// fixed size (room for SCRATCH_PARTIALS of them).  Each device has its own
// copy at its own address; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (the array's name is a host-side
// stand-in in host code), looked up once per device on the first call there.
// The kernels and the launch shape are ph_perm's (the sweep writes every
// partial before the finalize reads it, so nothing needs clearing), and the
// result has the same bits.  Every call on a device shares that device's
// array: calls that overlap on one device (two streams at once) race.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "permhip.h"
#include "ph_host.hpp"
#include "ph_internal.hpp"

namespace ph {

// 4 wavefronts x 8 resident workgroups x 256 CUs: every launch shape of the
// one-matrix sweep on an MI355X.
constexpr uint64_t SCRATCH_PARTIALS = 8192;

static __device__ __align__(256) double4 scratch[SCRATCH_PARTIALS];

static std::mutex g_scratch_mu;
static std::map<int, double4*> g_scratch;  // device -> device address of its scratch

// The device address of this device's scratch (looked up on the first call
// on the device, with that device current).
static int scratch_on(int dev, double4** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(dev);
  if (it == g_scratch.end()) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(PH_EHIP, "hipGetSymbolAddress(scratch) gave NULL");
    it = g_scratch.emplace(dev, static_cast<double4*>(p)).first;
  }
  *out = it->second;
  return PH_OK;
}

}  // namespace ph

using namespace ph;

extern "C" int ph_perm_noalloc(const ph_c128* A, int32_t n, int64_t lda, ph_c128* out, const ph_opts* opt,
                               void* stream) {
  PH_TRACE("ph_perm_noalloc");
  Opts o;
  int rc = read_opts(opt, &o);
  if (rc) return rc;
  if (n < 0) return fail(PH_EINVAL, "n=%d < 0", n);
  if (n > PH_NMAX) return fail(PH_ERANGE, "n=%d > %d", n, PH_NMAX);
  if (!out) return fail(PH_EINVAL, "out is NULL");
  if (n > 0 && !A) return fail(PH_EINVAL, "A is NULL");
  if (n > 0 && lda < n) return fail(PH_EINVAL, "lda=%lld < n=%d", (long long)lda, n);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  const int cus = num_cus();
  if (cus <= 0) return PH_EUNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  double2* res = reinterpret_cast<double2*>(out);
  if (n == 0) {
    launch_finalize_single(nullptr, 0, 0, o.algo, o.plain, res, st);
    e = hipGetLastError();
    return e == hipSuccess ? PH_OK : hip_fail(e, "finalize launch");
  }
  const int nb = gray_bits(n, o.algo);
  const int c = pick_chunk_log2(n, o.algo, o.chunk_log2);
  const uint64_t nchunks = (uint64_t)1 << (nb - c);
  SweepGeom g;
  if ((rc = single_geometry(n, o, cus, nchunks, &g))) return rc;
  const uint64_t nparts = g.blocks * 4;
  if (nparts > SCRATCH_PARTIALS)
    return fail(PH_ERANGE, "ph_perm_noalloc: %llu partial sums needed, the static scratch holds %llu",
                (unsigned long long)nparts, (unsigned long long)SCRATCH_PARTIALS);
  double4* parts = nullptr;
  if ((rc = scratch_on(dev, &parts))) return rc;
  if ((rc = launch_single(g, reinterpret_cast<const double2*>(A), lda, c, 0, nchunks, o.plain ? 1 : 0, parts, st)))
    return rc;
  launch_finalize_single(parts, (int64_t)nparts, n, o.algo, o.plain, res, st);
  e = hipGetLastError();
  return e == hipSuccess ? PH_OK : hip_fail(e, "finalize launch");
}
