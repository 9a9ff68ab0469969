// Boson-sampling output probabilities (main text, Eq. (1)) and their
// gradient with respect to the input columns of the unitary.
//
//   Pr[S -> T] = |Per(U_{S,T})|^2 / (prod_i s_i! prod_j t_j!)
//
// U_{S,T} takes rows = the output modes of T (a mode holding t photons
// repeated t times) and columns = the input modes of S (likewise), U indexed
// [output mode, input mode].  The kernels here gather every pattern's
// submatrix into a packed batch, normalise the permanents, and scatter the
// per-pattern gradients back onto the columns of U in a fixed order.  The
// permanents and their gradients come from the batched forward plans and
// the gradient sweep.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "permhip.h"
#include "ph_host.hpp"
#include "ph_internal.hpp"

namespace ph {

int perm_grad_launch(const double2* A, int n, int64_t batch, const double2* gout, double2* pout, double2* grad,
                     const Opts& o, hipStream_t st, int cus);

// a[p][i][k] = U[T_p[i], S[k]]
__global__ void k_boson_gather(const double2* __restrict__ u, int64_t ldu, const int32_t* __restrict__ in_modes,
                               const int32_t* __restrict__ pats, int n, double2* __restrict__ a) {
  const int64_t p = blockIdx.x;
  const int32_t* t = pats + p * n;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, k = e % n;
    a[p * n * n + e] = u[(int64_t)t[i] * ldu + in_modes[k]];
  }
}

// prod over modes of (photons in the mode)! for a list of n modes: the
// running count of each mode at its i-th occurrence multiplies to t!.
__device__ double occupation_factorials(const int32_t* modes, int n) {
  double f = 1.0;
  for (int i = 0; i < n; ++i) {
    int c = 0;
    for (int j = 0; j <= i; ++j) c += modes[j] == modes[i];
    f *= (double)c;
  }
  return f;
}

// probs[p] = |perm_p|^2 / (prod s! prod t!); optionally the upstream
// gradient of L = sum w_p Pr_p with respect to perm_p (PyTorch convention):
// g_p = 2 w_p perm_p / D_p.
__global__ void k_boson_normalize(const double2* __restrict__ perms, const int32_t* __restrict__ in_modes,
                                  const int32_t* __restrict__ pats, int n, int64_t npat,
                                  const double* __restrict__ weights, double* __restrict__ probs,
                                  double2* __restrict__ gperm) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= npat) return;
  const double d = occupation_factorials(in_modes, n) * occupation_factorials(pats + p * n, n);
  const double2 v = perms[p];
  if (probs) probs[p] = (v.x * v.x + v.y * v.y) / d;
  if (gperm) {
    const double w = weights ? weights[p] : 1.0;
    gperm[p] = make_double2(2.0 * w * v.x / d, 2.0 * w * v.y / d);
  }
}

// dU[r][k] = sum over (p, i) with T_p[i] = r, in the order of the list, of
// g_p * conj(M_p)[i][k]; rows of U that no pattern uses get 0.
// rowstart/rowlist: CSR over output modes of the (p * n + i) entries.
__global__ void k_boson_scatter(const double2* __restrict__ gA, const double2* __restrict__ gperm, int n,
                                const int64_t* __restrict__ rowstart, const int64_t* __restrict__ rowlist, int m,
                                double2* __restrict__ du, int64_t lddu) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * n) return;
  const int r = (int)(e / n), k = (int)(e % n);
  double sr = 0.0, si = 0.0;
  for (int64_t q = rowstart[r]; q < rowstart[r + 1]; ++q) {
    const int64_t pi = rowlist[q];  // p * n + i
    const int64_t p = pi / n;
    const double2 c = gA[pi * n + k];  // conj(M_p)[i][k]
    const double2 g = gperm[p];
    sr += g.x * c.x - g.y * c.y;
    si += g.x * c.y + g.y * c.x;
  }
  du[(int64_t)r * lddu + k] = make_double2(sr, si);
}

static int check_boson_args(const ph_c128* U, int32_t m, int64_t ldu, const int32_t* in_modes, int32_t n,
                            const int32_t* patterns, int64_t npat, int nmax) {
  if (m < 1) return fail(PH_EINVAL, "m=%d < 1", m);
  if (n < 0) return fail(PH_EINVAL, "n=%d < 0", n);
  if (n > nmax) return fail(PH_ERANGE, "n=%d > %d", n, nmax);
  if (ldu < m) return fail(PH_EINVAL, "ldu=%lld < m=%d", (long long)ldu, m);
  if (npat < 0) return fail(PH_EINVAL, "n_patterns < 0");
  if (npat > ((int64_t)1 << 30)) return fail(PH_ERANGE, "n_patterns=%lld > 2^30", (long long)npat);
  if (!U) return fail(PH_EINVAL, "U is NULL");
  if (n > 0 && (!in_modes || (npat > 0 && !patterns))) return fail(PH_EINVAL, "modes are NULL");
  for (int k = 0; k < n; ++k)
    if (in_modes[k] < 0 || in_modes[k] >= m) return fail(PH_EINVAL, "in_modes[%d]=%d out of [0,%d)", k, in_modes[k], m);
  for (int64_t q = 0; q < npat * n; ++q)
    if (patterns[q] < 0 || patterns[q] >= m)
      return fail(PH_EINVAL, "patterns[%lld]=%d out of [0,%d)", (long long)q, patterns[q], m);
  return PH_OK;
}

static size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// Pinned host staging for the host-side mode lists and the scatter index, one
// per (device, stream): the call copies the caller's arrays here and uploads
// from here, so it returns without waiting for the upload.  The event marks
// when the previous upload from this buffer has been consumed.
struct Staging {
  void* host = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
};
static std::mutex g_stage_mu;
static std::map<std::pair<int, hipStream_t>, Staging> g_stage;

// Copy `bytes` from the host pieces into device memory `dst` on `st`.
struct Piece {
  const void* src;
  size_t bytes;
};
static int upload(hipStream_t st, void* dst, const Piece* pc, int npc) {
  size_t bytes = 0;
  for (int q = 0; q < npc; ++q) bytes += up256(pc[q].bytes);
  if (bytes == 0) return PH_OK;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_stage_mu);
  Staging& s = g_stage[{dev, st}];
  if (s.pending) {
    e = hipEventSynchronize(s.ev);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    s.pending = false;
  }
  if (!s.ev) {
    e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
  }
  if (s.cap < bytes) {
    if (s.host) hipHostFree(s.host);
    s.host = nullptr;
    s.cap = 0;
    const size_t cap = std::max(bytes, (size_t)1 << 16);
    e = hipHostMalloc(&s.host, cap, hipHostMallocDefault);
    if (e != hipSuccess) return fail(PH_ENOMEM, "hipHostMalloc(%zu): %s", cap, hipGetErrorString(e));
    s.cap = cap;
  }
  char* h = static_cast<char*>(s.host);
  size_t off = 0;
  for (int q = 0; q < npc; ++q) {
    if (pc[q].bytes) std::memcpy(h + off, pc[q].src, pc[q].bytes);
    off += up256(pc[q].bytes);
  }
  e = hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "mode upload");
  e = hipEventRecord(s.ev, st);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  s.pending = true;
  return PH_OK;
}

// Device buffers of one boson call, in workspace slot 1 of the stream (the
// permanent kernels own slot 0).  Layout: in_modes | patterns | [rowstart |
// rowlist] | gathered batch | perms | [gA | gperm].
struct BosonBufs {
  int32_t* d_in;
  int32_t* d_pat;
  int64_t* d_start;
  int64_t* d_list;
  double2* a;
  double2* perms;
  double2* gA;
  double2* gperm;
};

static int boson_setup(hipStream_t st, const ph_c128* U, int32_t m, int64_t ldu, const int32_t* in_modes, int n,
                       const int32_t* patterns, int64_t npat, bool grad, BosonBufs* b) {
  std::vector<int64_t> start, list;
  if (grad) {
    // CSR of the (pattern, position) entries p * n + i by output mode, in
    // increasing order within each mode
    start.assign(m + 1, 0);
    list.resize(npat * n);
    for (int64_t q = 0; q < npat * n; ++q) start[patterns[q] + 1]++;
    for (int r = 0; r < m; ++r) start[r + 1] += start[r];
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t q = 0; q < npat * n; ++q) list[fill[patterns[q]]++] = q;
  }
  const Piece pc[4] = {{in_modes, n * sizeof(int32_t)},
                       {patterns, (size_t)(npat * n) * sizeof(int32_t)},
                       {start.data(), start.size() * sizeof(int64_t)},
                       {list.data(), list.size() * sizeof(int64_t)}};
  size_t off[9];
  off[0] = 0;
  for (int q = 0; q < 4; ++q) off[q + 1] = off[q] + up256(pc[q].bytes);
  off[5] = off[4] + up256((size_t)(npat * n * n) * sizeof(double2));
  off[6] = off[5] + up256((size_t)npat * sizeof(double2));
  off[7] = off[6] + (grad ? up256((size_t)(npat * n * n) * sizeof(double2)) : 0);
  off[8] = off[7] + (grad ? up256((size_t)npat * sizeof(double2)) : 0);
  void* ws = nullptr;
  int rc = workspace_slot(st, std::max<size_t>(off[8], 256), 1, &ws);
  if (rc) return rc;
  char* q = static_cast<char*>(ws);
  b->d_in = reinterpret_cast<int32_t*>(q + off[0]);
  b->d_pat = reinterpret_cast<int32_t*>(q + off[1]);
  b->d_start = reinterpret_cast<int64_t*>(q + off[2]);
  b->d_list = reinterpret_cast<int64_t*>(q + off[3]);
  b->a = reinterpret_cast<double2*>(q + off[4]);
  b->perms = reinterpret_cast<double2*>(q + off[5]);
  b->gA = reinterpret_cast<double2*>(q + off[6]);
  b->gperm = reinterpret_cast<double2*>(q + off[7]);
  if ((rc = upload(st, q, pc, 4))) return rc;
  if (npat > 0 && n > 0)
    hipLaunchKernelGGL(k_boson_gather, dim3((unsigned)npat), dim3(256), 0, st, reinterpret_cast<const double2*>(U),
                       ldu, b->d_in, b->d_pat, n, b->a);
  return PH_OK;
}

}  // namespace ph

using namespace ph;

extern "C" int ph_boson_probs(const ph_c128* U, int32_t m, int64_t ldu, const int32_t* in_modes, int32_t n,
                              const int32_t* patterns, int64_t n_patterns, double* probs, const ph_opts* opt,
                              void* stream) {
  Opts o;
  int rc = read_opts(opt, &o);
  if (rc) return rc;
  if ((rc = check_boson_args(U, m, ldu, in_modes, n, patterns, n_patterns, PH_NMAX))) return rc;
  if (n_patterns > 0 && !probs) return fail(PH_EINVAL, "probs is NULL");
  if (n_patterns == 0) return PH_OK;
  if (num_cus() <= 0) return PH_EUNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  BosonBufs b;
  if ((rc = boson_setup(st, U, m, ldu, in_modes, n, patterns, n_patterns, false, &b))) return rc;
  std::vector<int32_t> ns(n_patterns, n);
  rc = ph_perm_batched(reinterpret_cast<const ph_c128*>(b.a), nullptr, ns.data(), n_patterns,
                       reinterpret_cast<ph_c128*>(b.perms), opt, stream);
  if (rc) return rc;
  hipLaunchKernelGGL(k_boson_normalize, dim3((unsigned)((n_patterns + 255) / 256)), dim3(256), 0, st, b.perms,
                     b.d_in, b.d_pat, n, n_patterns, (const double*)nullptr, probs, (double2*)nullptr);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? PH_OK : hip_fail(e, "boson launch");
}

extern "C" int ph_boson_probs_grad(const ph_c128* U, int32_t m, int64_t ldu, const int32_t* in_modes, int32_t n,
                                   const int32_t* patterns, int64_t n_patterns, const double* weights, double* probs,
                                   ph_c128* dU, int64_t lddu, const ph_opts* opt, void* stream) {
  Opts o;
  int rc = read_opts(opt, &o);
  if (rc) return rc;
  if (o.algo != PH_GLYNN) return fail(PH_EINVAL, "the gradient supports PH_GLYNN only");
  if ((rc = check_boson_args(U, m, ldu, in_modes, n, patterns, n_patterns, PH_NMAX_GRAD))) return rc;
  if (n < 1) return fail(PH_EINVAL, "n=%d < 1", n);
  if (!dU) return fail(PH_EINVAL, "dU is NULL");
  if (lddu < n) return fail(PH_EINVAL, "lddu=%lld < n=%d", (long long)lddu, n);
  const int cus = num_cus();
  if (cus <= 0) return PH_EUNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  BosonBufs b;
  if ((rc = boson_setup(st, U, m, ldu, in_modes, n, patterns, n_patterns, true, &b))) return rc;
  if (n_patterns > 0) {
    // permanents and conj(M) of every pattern in one gradient sweep
    rc = perm_grad_launch(b.a, n, n_patterns, nullptr, b.perms, b.gA, o, st, cus);
    if (rc) return rc;
    hipLaunchKernelGGL(k_boson_normalize, dim3((unsigned)((n_patterns + 255) / 256)), dim3(256), 0, st, b.perms,
                       b.d_in, b.d_pat, n, n_patterns, weights, probs, b.gperm);
  }
  const int64_t tot = (int64_t)m * n;
  hipLaunchKernelGGL(k_boson_scatter, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, b.gA, b.gperm, n,
                     b.d_start, b.d_list, m, reinterpret_cast<double2*>(dU), lddu);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? PH_OK : hip_fail(e, "boson grad launch");
}
