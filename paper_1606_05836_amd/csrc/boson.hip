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

#include "dd.hpp"
#include "permhip.h"
#include "ph_host.hpp"
#include "ph_internal.hpp"
#include "sweep.hpp"

namespace ph {

int perm_grad_launch(const double2* A, int n, int64_t batch, const double2* gout, double2* pout, double2* grad,
                     const Opts& o, hipStream_t st, int cus);
int grad_rows(int n);
int grad_min_cols(int n);
int grad_sweep(const double2* tabs, int n, int ncols, int64_t batch, const double2* gout, double2* pout,
               double2* grad, const Opts& o, hipStream_t st, int cus);

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

// Input modes by value (n <= PH_NMAX_GRAD), for the fold below.
struct InModes {
  int32_t v[PH_NMAX_GRAD];
};

// dU[r][j] = sum over the photons k with in_modes[k] == j, in increasing k,
// of dUn[r][k] (the per-photon columns); columns no photon uses get 0.  Every
// entry of the m x m output is written.
__global__ void k_boson_fold_photons(const double2* __restrict__ dun, int n, InModes in, int m,
                                     double2* __restrict__ du, int64_t lddu) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)m * m) return;
  const int r = (int)(t / m), j = (int)(t % m);
  double sr = 0.0, si = 0.0;
  for (int k = 0; k < n; ++k) {
    if (in.v[k] == j) {
      const double2 x = dun[(int64_t)r * n + k];
      sr += x.x;
      si += x.y;
    }
  }
  du[(int64_t)r * lddu + j] = make_double2(sr, si);
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

// Copy the host pieces into device memory at base + off[q] (piece q), one
// transfer of off[npc] bytes on `st` through the pinned staging buffer.
static int upload_at(hipStream_t st, void* base, const size_t* off, const Piece* pc, int npc) {
  const size_t bytes = off[npc];
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
    if (s.host) (void)hipHostFree(s.host);  // the old staging buffer's last upload has completed
    s.host = nullptr;
    s.cap = 0;
    const size_t cap = std::max(bytes, (size_t)1 << 16);
    e = hipHostMalloc(&s.host, cap, hipHostMallocDefault);
    if (e != hipSuccess) return fail(PH_ENOMEM, "hipHostMalloc(%zu): %s", cap, hipGetErrorString(e));
    s.cap = cap;
  }
  char* h = static_cast<char*>(s.host);
  for (int q = 0; q < npc; ++q)
    if (pc[q].bytes) std::memcpy(h + off[q], pc[q].src, pc[q].bytes);
  e = hipMemcpyAsync(base, h, bytes, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "mode upload");
  e = hipEventRecord(s.ev, st);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  s.pending = true;
  return PH_OK;
}

// Pieces packed back to back at 256-byte boundaries.
int upload(hipStream_t st, void* dst, const Piece* pc, int npc) {
  std::vector<size_t> off(npc + 1, 0);
  for (int q = 0; q < npc; ++q) off[q + 1] = off[q] + up256(pc[q].bytes);
  return upload_at(st, dst, off.data(), pc, npc);
}

// Device buffers of one boson call, in workspace slot 1 of the stream (the
// permanent kernels own WS_SWEEP).  Layout: in_modes | patterns | [rowstart |
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
  int rc = workspace_slot(st, std::max<size_t>(off[8], 256), WS_BOSON, &ws);
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


// ------------------------------------------------ multiplicity-grouped sweeps
//
// Per(U_{S,T}) = Per(B) with B = U_{S,T}^T (rows: input photons, columns:
// output photons).  The columns of B that belong to one output mode l are
// equal (mu_l copies).  In Eq. (S2) the signs of those copies enter the row
// sums as (mu_l - 2 k_l) b_l and the sign product as (-1)^{k_l}, with k_l
// their number of -1 entries, C(mu_l, k_l) ways each.  With the sign of one
// single-photon mode l0 fixed:
//   Per = 2^-(n-1) sum_{k over collided modes} w(k) G(k),
//   w(k) = prod_l C(mu_l, k_l) (-1)^{k_l},
//   G(k) = BB/FG sum over the single-photon modes of the n x n1 table whose
//          first column is b_l0 + sum_l (mu_l - 2 k_l) b_l.
// Each (pattern, k) is one sweep of 2^(n1-1) terms of the batched kernels.

// Sweep tables: column 0 = U[mode0, S_i] + sum_c coef_c U[coll_c, S_i],
// column j >= 1 = -2 U[mode_j, S_i]; column-major, n rows per column.
__global__ void k_boson_vtab(const double2* __restrict__ u, int64_t ldu, const int32_t* __restrict__ in_modes, int n,
                             const int32_t* __restrict__ vcol, const int32_t* __restrict__ vncols,
                             const int32_t* __restrict__ vcoef, const int32_t* __restrict__ vncoef,
                             const int32_t* __restrict__ colmodes, const int32_t* __restrict__ collmodes,
                             const double* __restrict__ coefs, const int64_t* __restrict__ tab_off,
                             double2* __restrict__ tabs) {
  const int64_t v = blockIdx.x;
  const int ncols = vncols[v];
  const int32_t* cm = colmodes + vcol[v];
  const int c0 = vcoef[v], nc = vncoef[v];
  double2* t = tabs + tab_off[v];
  for (int e = threadIdx.x; e < n * ncols; e += blockDim.x) {
    const int j = e / n, i = e % n;
    const int64_t s = in_modes[i];
    double2 val = u[(int64_t)cm[j] * ldu + s];
    if (j == 0) {
      for (int q = 0; q < nc; ++q) {
        const double w = coefs[c0 + q];
        const double2 b = u[(int64_t)collmodes[c0 + q] * ldu + s];
        val.x = fma(w, b.x, val.x);
        val.y = fma(w, b.y, val.y);
      }
    } else {
      val = make_double2(-2.0 * val.x, -2.0 * val.y);
    }
    t[(int64_t)j * n + i] = val;
  }
}

// perms[p] = sum over the pattern's sweeps of w_v * vout[vpos[v]] (vpos
// NULL: vout in sweep order), one wavefront per pattern: lane t sums a
// contiguous slice of the sweeps in order, then the lanes meet in a fixed
// butterfly, so the result depends only on the inputs.
__global__ __launch_bounds__(64) void k_boson_combine(const double2* __restrict__ vout,
                                                      const int32_t* __restrict__ vpos, const double* __restrict__ w,
                                                      const int32_t* __restrict__ pv, int64_t npat, int plain,
                                                      double2* __restrict__ perms) {
  const int64_t p = blockIdx.x;
  if (p >= npat) return;
  const int t = threadIdx.x;
  const int64_t v0 = pv[p], cnt = pv[p + 1] - v0;
  const int64_t b0 = v0 + cnt * t / 64, b1 = v0 + cnt * (t + 1) / 64;
  dd2 s = {0.0, 0.0, 0.0, 0.0};
  for (int64_t v = b0; v < b1; ++v) {
    const double2 x = vout[vpos ? vpos[v] : v];
    if (plain) {
      s.hr = fma(w[v], x.x, s.hr);
      s.hi = fma(w[v], x.y, s.hi);
    } else {
      // w is a small integer: w * x is one rounding, accumulated compensated
      dd_accumulate(s, w[v] * x.x, w[v] * x.y);
    }
  }
  s = wave_reduce(s, plain != 0);
  if (t == 0) perms[p] = make_double2(s.hr + s.lr, s.hi + s.li);
}

// Host description of the sweeps of a call.
struct Sweeps {
  std::vector<int32_t> vcol, vncols, vcoef, vncoef;  // per sweep
  std::vector<double> w;                            // per sweep
  std::vector<int32_t> colmodes, collmodes;
  std::vector<double> coefs;
  std::vector<int32_t> pv;  // per pattern: first sweep (npat + 1 entries)
};

// Limits: single-photon modes a grouped pattern needs (the sweep kernels walk
// at least 4 Gray bits), sweeps per pattern, sweeps per call.
constexpr int GROUP_MIN_SINGLES = 5;
constexpr int64_t GROUP_MAX_PER_PATTERN = 4096;
constexpr int64_t GROUP_MAX_SWEEPS = (int64_t)1 << 18;

// min_singles: the fewest single-photon modes (columns of a grouped sweep)
// a pattern needs to be grouped.
static void plan_sweeps(const int32_t* patterns, int n, int64_t npat, bool ungrouped, int min_singles, Sweeps* sw) {
  sw->pv.assign(npat + 1, 0);
  int64_t budget = GROUP_MAX_SWEEPS;
  std::vector<std::pair<int32_t, int>> cls;  // (mode, photons), first-appearance order
  for (int64_t p = 0; p < npat; ++p) {
    const int32_t* t = patterns + p * n;
    sw->pv[p] = (int32_t)sw->w.size();
    cls.clear();
    for (int i = 0; i < n; ++i) {
      bool found = false;
      for (auto& c : cls)
        if (c.first == t[i]) {
          ++c.second;
          found = true;
          break;
        }
      if (!found) cls.emplace_back(t[i], 1);
    }
    int singles = 0;
    int64_t combos = 1;
    for (auto& c : cls) {
      if (c.second == 1) ++singles;
      else combos *= c.second + 1;
      if (combos > GROUP_MAX_PER_PATTERN) break;
    }
    const bool group = !ungrouped && singles >= min_singles && combos > 1 &&
                       combos <= GROUP_MAX_PER_PATTERN && combos <= budget;
    if (!group) {
      // one sweep over all n columns (repeats included), weight 1
      sw->vcol.push_back((int32_t)sw->colmodes.size());
      sw->colmodes.insert(sw->colmodes.end(), t, t + n);
      sw->vncols.push_back(n);
      sw->vcoef.push_back((int32_t)sw->coefs.size());
      sw->vncoef.push_back(0);
      sw->w.push_back(1.0);
      continue;
    }
    budget -= combos;
    const int32_t col_off = (int32_t)sw->colmodes.size();
    for (auto& c : cls)
      if (c.second == 1) sw->colmodes.push_back(c.first);
    std::vector<std::pair<int32_t, int>> coll;
    for (auto& c : cls)
      if (c.second > 1) coll.push_back(c);
    // signed binomials (-1)^k C(mu, k) of each collided mode
    const size_t nl = coll.size();
    std::vector<std::vector<double>> sbin(nl);
    for (size_t l = 0; l < nl; ++l) {
      const int mu = coll[l].second;
      for (int kk = 0; kk <= mu; ++kk) {
        double binom = 1.0;
        for (int z = 0; z < kk; ++z) binom = binom * (mu - z) / (z + 1);
        sbin[l].push_back((kk & 1) ? -binom : binom);
      }
    }
    // k in mixed radix, first collided mode fastest, stepped like an odometer
    std::vector<int> k(nl, 0);
    for (int64_t q = 0; q < combos; ++q) {
      double w = 1.0;
      sw->vcoef.push_back((int32_t)sw->coefs.size());
      sw->vncoef.push_back((int32_t)nl);
      for (size_t l = 0; l < nl; ++l) {
        w *= sbin[l][k[l]];
        sw->collmodes.push_back(coll[l].first);
        sw->coefs.push_back((double)(coll[l].second - 2 * k[l]));
      }
      sw->vcol.push_back(col_off);
      sw->vncols.push_back(singles);
      sw->w.push_back(w);
      for (size_t l = 0; l < nl; ++l) {
        if (++k[l] <= coll[l].second) break;
        k[l] = 0;
      }
    }
  }
  sw->pv[npat] = (int32_t)sw->w.size();
}

// Eq. (1) probabilities of all patterns through the grouped sweeps: one
// staged upload of the mode lists and sweep descriptions, the sweep tables,
// one batched plan replay, the weighted combination and the normalisation.
static int boson_probs_grouped(hipStream_t st, const ph_c128* U, int64_t ldu, const int32_t* in_modes, int n,
                               const int32_t* patterns, int64_t npat, const Opts& o, double* probs) {
  Sweeps sw;
  plan_sweeps(patterns, n, npat, o.ungrouped, GROUP_MIN_SINGLES, &sw);
  const int64_t V = (int64_t)sw.w.size();
  std::vector<int32_t> ns(V, n);
  // device layout in workspace slot WS_BOSON_GROUPED (the first NP_UP entries are uploaded)
  enum { P_IN, P_VCOL, P_VNCOLS, P_VCOEF, P_VNCOEF, P_COLM, P_COLLM, P_PV, P_PAT, P_COEFS, P_W, P_TABOFF, NP_UP,
         B_VOUT = NP_UP, B_PERMS, NB_ALL };
  auto one = [](size_t x) { return std::max<size_t>(x, 1); };
  size_t sz[NB_ALL];
  sz[P_IN] = one(n) * 4;
  sz[P_VCOL] = sz[P_VNCOLS] = sz[P_VCOEF] = sz[P_VNCOEF] = one(V) * 4;
  sz[P_COLM] = one(sw.colmodes.size()) * 4;
  sz[P_COLLM] = one(sw.collmodes.size()) * 4;
  sz[P_PV] = one(npat + 1) * 4;
  sz[P_PAT] = one(npat * n) * 4;
  sz[P_COEFS] = one(sw.coefs.size()) * 8;
  sz[P_W] = sz[P_TABOFF] = one(V) * 8;
  sz[B_VOUT] = one(V) * 16;
  sz[B_PERMS] = one(npat) * 16;
  size_t off[NB_ALL + 1];
  off[0] = 0;
  for (int q = 0; q < NB_ALL; ++q) off[q + 1] = off[q] + up256(sz[q]);
  void* ws = nullptr;
  int rc = workspace_slot(st, off[NB_ALL], WS_BOSON_GROUPED, &ws);
  if (rc) return rc;
  char* d = static_cast<char*>(ws);
  auto I32 = [&](int q) { return reinterpret_cast<int32_t*>(d + off[q]); };
  auto F64 = [&](int q) { return reinterpret_cast<double*>(d + off[q]); };
  auto C128 = [&](int q) { return reinterpret_cast<double2*>(d + off[q]); };
  auto fill = [&](PlanImpl* p) -> int {
    const std::vector<int64_t>& toff = plan_table_offsets(p);
    const Piece pc[NP_UP] = {{in_modes, (size_t)n * 4},
                             {sw.vcol.data(), (size_t)V * 4},
                             {sw.vncols.data(), (size_t)V * 4},
                             {sw.vcoef.data(), (size_t)V * 4},
                             {sw.vncoef.data(), (size_t)V * 4},
                             {sw.colmodes.data(), sw.colmodes.size() * 4},
                             {sw.collmodes.data(), sw.collmodes.size() * 4},
                             {sw.pv.data(), (size_t)(npat + 1) * 4},
                             {patterns, (size_t)(npat * n) * 4},
                             {sw.coefs.data(), sw.coefs.size() * 8},
                             {sw.w.data(), (size_t)V * 8},
                             {toff.data(), (size_t)V * 8}};
    int r = upload_at(st, d, off, pc, NP_UP);
    if (r) return r;
    hipLaunchKernelGGL(k_boson_vtab, dim3((unsigned)V), dim3(256), 0, st, reinterpret_cast<const double2*>(U), ldu,
                       I32(P_IN), n, I32(P_VCOL), I32(P_VNCOLS), I32(P_VCOEF), I32(P_VNCOEF), I32(P_COLM),
                       I32(P_COLLM), F64(P_COEFS), reinterpret_cast<int64_t*>(d + off[P_TABOFF]),
                       plan_tables_base(p));
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? PH_OK : hip_fail(e, "boson table launch");
  };
  Opts og = o;
  og.algo = PH_GLYNN;
  rc = plan_ext_run(ns.data(), sw.vncols.data(), V, og, st, fill, C128(B_VOUT));
  if (rc) return rc;
  const unsigned pb = (unsigned)((npat + 255) / 256);
  hipLaunchKernelGGL(k_boson_combine, dim3((unsigned)npat), dim3(64), 0, st, C128(B_VOUT), (const int32_t*)nullptr,
                     F64(P_W), I32(P_PV), npat, o.plain ? 1 : 0, C128(B_PERMS));
  hipLaunchKernelGGL(k_boson_normalize, dim3(pb), dim3(256), 0, st, C128(B_PERMS), I32(P_IN), I32(P_PAT), n, npat,
                     (const double*)nullptr, probs, (double2*)nullptr);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PH_OK : hip_fail(e, "boson launch");
}

// ------------------------------------------- gradient of the grouped sweeps
//
// The gradient sweep over sweep v's n x n1 table gives conj(dF_v / dC_v) with
// F_v = 2^-(n-1) G_v and C_v its columns.  Column 0 is b_l0 + sum_c coef_c b_c
// and column j >= 1 is b_(mode j), so for output mode x of pattern p
//   conj(dPer_p / db_x) = sum_v w_v [ sum_{j: mode j = x} conj(dF_v/dC_v[:, j])
//                                     + sum_{c: coll c = x} coef_c conj(dF_v/dC_v[:, 0]) ],
// a list of (entry of conj(dF), coefficient) per (pattern, mode) summed in a
// fixed order; dU[x][k] = sum over patterns holding x of g_p conj(dPer_p/db_x[k]).

// Gradient tables of one group of sweeps with equal column counts: like
// k_boson_vtab, rows padded to `rows` with zeros, T[j * rows + i].
__global__ void k_boson_gtab(const double2* __restrict__ u, int64_t ldu, const int32_t* __restrict__ in_modes, int n,
                             int rows, const int32_t* __restrict__ vlist, const int32_t* __restrict__ vcol, int ncols,
                             const int32_t* __restrict__ vcoef, const int32_t* __restrict__ vncoef,
                             const int32_t* __restrict__ colmodes, const int32_t* __restrict__ collmodes,
                             const double* __restrict__ coefs, double2* __restrict__ tabs) {
  const int64_t b = blockIdx.x;
  const int32_t v = vlist[b];
  const int32_t* cm = colmodes + vcol[v];
  const int c0 = vcoef[v], nc = vncoef[v];
  double2* t = tabs + b * ncols * rows;
  for (int e = threadIdx.x; e < ncols * rows; e += blockDim.x) {
    const int j = e / rows, i = e % rows;
    double2 val = make_double2(0.0, 0.0);
    if (i < n) {
      const int64_t s = in_modes[i];
      val = u[(int64_t)cm[j] * ldu + s];
      if (j == 0) {
        for (int q = 0; q < nc; ++q) {
          const double w = coefs[c0 + q];
          const double2 bq = u[(int64_t)collmodes[c0 + q] * ldu + s];
          val.x = fma(w, bq.x, val.x);
          val.y = fma(w, bq.y, val.y);
        }
      } else {
        val = make_double2(-2.0 * val.x, -2.0 * val.y);
      }
    }
    t[e] = val;
  }
}

// One (pattern, output mode) entry of the gradient: which columns of the
// pattern's sweeps hold the mode.
enum : int32_t {
  ENT_SINGLE = 0,    // grouped pattern, single-photon mode: column idx of every sweep
  ENT_COLLIDED = 1,  // grouped pattern, collided mode idx: column 0 of every sweep, times its coefficient
  ENT_WHOLE = 2      // pattern swept whole: every column of its one sweep that holds the mode
};
struct EntryDesc {
  int32_t pat, kind, idx, mode;
};

// D[e][k] = sum over the sweeps v of entry e's pattern of w_v *
// (coefficient) * cm_v[k][column] for the columns of v that hold the entry's
// mode (cm_v: the n x ncols column derivatives of sweep v).  One wavefront
// per (e, k): lane t sums a contiguous slice of the sweeps in order, then the
// lanes meet in a fixed butterfly, so the result depends only on the inputs.
// The grid strides over the (e, k) pairs.
__global__ __launch_bounds__(64) void k_boson_class_grad(
    const double2* __restrict__ cm, const int64_t* __restrict__ moff, const int32_t* __restrict__ vncols,
    const int32_t* __restrict__ vcol, const int32_t* __restrict__ colmodes, const int32_t* __restrict__ vcoef,
    const double* __restrict__ coefs, const double* __restrict__ w, const int32_t* __restrict__ pv,
    const EntryDesc* __restrict__ ent, int64_t nent, int n, double2* __restrict__ D) {
  const int lane = threadIdx.x;
  for (int64_t t = blockIdx.x; t < nent * n; t += gridDim.x) {
    const int64_t e = t / n;
    const int k = (int)(t % n);
    const EntryDesc d = ent[e];
    const int64_t v0 = pv[d.pat], cnt = pv[d.pat + 1] - v0;
    const int64_t b0 = v0 + cnt * lane / 64, b1 = v0 + cnt * (lane + 1) / 64;
    double sr = 0.0, si = 0.0;
    for (int64_t v = b0; v < b1; ++v) {
      const int nc = vncols[v];
      const double2* c = cm + moff[v] + (int64_t)k * nc;
      if (d.kind == ENT_SINGLE) {
        const double2 x = c[d.idx];
        sr = fma(w[v], x.x, sr);
        si = fma(w[v], x.y, si);
      } else if (d.kind == ENT_COLLIDED) {
        const double cf = w[v] * coefs[vcoef[v] + d.idx];
        const double2 x = c[0];
        sr = fma(cf, x.x, sr);
        si = fma(cf, x.y, si);
      } else {
        const int32_t* cmd = colmodes + vcol[v];
        for (int j = 0; j < nc; ++j)
          if (cmd[j] == d.mode) {
            const double2 x = c[j];
            sr = fma(w[v], x.x, sr);
            si = fma(w[v], x.y, si);
          }
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      sr += __shfl_xor(sr, off, 64);
      si += __shfl_xor(si, off, 64);
    }
    if (lane == 0) D[t] = make_double2(sr, si);
  }
}

// dU[r][k] = sum over the entries of output mode r, in order, of g_p D[e][k]
__global__ void k_boson_scatter_entries(const double2* __restrict__ D, const double2* __restrict__ gperm,
                                        const int32_t* __restrict__ ent_pat, const int32_t* __restrict__ mstart,
                                        const int32_t* __restrict__ mlist, int m, int n, double2* __restrict__ du,
                                        int64_t lddu) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)m * n) return;
  const int r = (int)(t / n), k = (int)(t % n);
  double sr = 0.0, si = 0.0;
  for (int32_t q = mstart[r]; q < mstart[r + 1]; ++q) {
    const int32_t e = mlist[q];
    const double2 g = gperm[ent_pat[e]];
    const double2 d = D[(int64_t)e * n + k];
    sr += g.x * d.x - g.y * d.y;
    si += g.x * d.y + g.y * d.x;
  }
  du[(int64_t)r * lddu + k] = make_double2(sr, si);
}

static int boson_grad_grouped(hipStream_t st, const ph_c128* U, int32_t m, int64_t ldu, const int32_t* in_modes,
                              int n, const int32_t* patterns, int64_t npat, const double* weights, double* probs,
                              ph_c128* dU, int64_t lddu, const Opts& o, int cus) {
  if ((int64_t)npat * n >= ((int64_t)1 << 31) - 1) return fail(PH_ERANGE, "n_patterns * n too large");
  Sweeps sw;
  // a grouped gradient sweep walks at least grad_min_cols(n) columns
  plan_sweeps(patterns, n, npat, o.ungrouped, std::max(GROUP_MIN_SINGLES, grad_min_cols(n)), &sw);
  const int64_t V = (int64_t)sw.w.size();
  const int rows = grad_rows(n);
  // groups of sweeps by column count; position of each sweep's results
  std::map<int, std::vector<int32_t>> groups;
  for (int64_t v = 0; v < V; ++v) groups[sw.vncols[v]].push_back((int32_t)v);
  std::vector<int32_t> vlist, vpos(V);
  std::vector<int64_t> moff(V);
  int64_t mtot = 0, max_tab = 0;
  for (auto& g : groups) {
    max_tab = std::max<int64_t>(max_tab, (int64_t)g.second.size() * g.first * rows);
    for (int32_t v : g.second) {
      vpos[v] = (int32_t)vlist.size();
      vlist.push_back(v);
      moff[v] = mtot;
      mtot += (int64_t)n * g.first;
    }
  }
  // (pattern, output mode) entries, patterns in order, modes in order of
  // first appearance; each names the columns of its pattern's sweeps that
  // hold its mode
  std::vector<int32_t> ent_pat, ent_mode;
  std::vector<EntryDesc> ent;
  ent.reserve((size_t)npat * n);
  for (int64_t p = 0; p < npat; ++p) {
    const int32_t* t = patterns + p * n;
    const int32_t e0 = (int32_t)ent.size();
    const int32_t v0 = sw.pv[p];
    const bool grouped = sw.vncoef[v0] > 0;
    for (int i = 0; i < n; ++i) {
      bool seen = false;
      for (int32_t e = e0; e < (int32_t)ent.size() && !seen; ++e) seen = ent[e].mode == t[i];
      if (seen) continue;
      EntryDesc d{(int32_t)p, ENT_WHOLE, 0, t[i]};
      if (grouped) {
        d.kind = -1;
        for (int j = 0; j < sw.vncols[v0] && d.kind < 0; ++j)
          if (sw.colmodes[sw.vcol[v0] + j] == t[i]) d = EntryDesc{(int32_t)p, ENT_SINGLE, j, t[i]};
        for (int q = 0; q < sw.vncoef[v0] && d.kind < 0; ++q)
          if (sw.collmodes[sw.vcoef[v0] + q] == t[i]) d = EntryDesc{(int32_t)p, ENT_COLLIDED, q, t[i]};
        if (d.kind < 0) return fail(PH_EINVAL, "pattern %lld: mode %d has no sweep column", (long long)p, t[i]);
      }
      ent.push_back(d);
      ent_pat.push_back((int32_t)p);
      ent_mode.push_back(t[i]);
    }
  }
  const int64_t E = (int64_t)ent.size();
  std::vector<int32_t> mstart(m + 1, 0), mlist(E);
  for (int64_t e = 0; e < E; ++e) mstart[ent_mode[e] + 1]++;
  for (int r = 0; r < m; ++r) mstart[r + 1] += mstart[r];
  {
    std::vector<int32_t> fill(mstart.begin(), mstart.end() - 1);
    for (int64_t e = 0; e < E; ++e) mlist[fill[ent_mode[e]]++] = (int32_t)e;
  }
  // device layout (workspace slot WS_BOSON_GROUPED)
  auto one = [](size_t x) { return std::max<size_t>(x, 1); };
  enum { P_IN, P_PAT, P_VCOL, P_VCOEF, P_VNCOEF, P_VNCOLS, P_COLM, P_COLLM, P_PV, P_VLIST, P_VPOS, P_ENTPAT,
         P_MSTART, P_MLIST, P_ENT, P_COEFS, P_W, P_MOFF, NP_UP,
         B_TAB = NP_UP, B_CM, B_POUT, B_PERMS, B_GPERM, B_D, NB_ALL };
  size_t sz[NB_ALL] = {};
  sz[P_IN] = one(n) * 4;
  sz[P_PAT] = one(npat * n) * 4;
  sz[P_VCOL] = sz[P_VCOEF] = sz[P_VNCOEF] = sz[P_VNCOLS] = one(V) * 4;
  sz[P_COLM] = one(sw.colmodes.size()) * 4;
  sz[P_COLLM] = one(sw.collmodes.size()) * 4;
  sz[P_PV] = one(npat + 1) * 4;
  sz[P_VLIST] = sz[P_VPOS] = one(V) * 4;
  sz[P_ENTPAT] = one(E) * 4;
  sz[P_MSTART] = one(m + 1) * 4;
  sz[P_MLIST] = one(E) * 4;
  sz[P_ENT] = one(E) * sizeof(EntryDesc);
  sz[P_COEFS] = one(sw.coefs.size()) * 8;
  sz[P_W] = one(V) * 8;
  sz[P_MOFF] = one(V) * 8;
  sz[B_TAB] = one(max_tab) * 16;
  sz[B_CM] = one(mtot) * 16;
  sz[B_POUT] = one(V) * 16;
  sz[B_PERMS] = sz[B_GPERM] = one(npat) * 16;
  sz[B_D] = one(E * n) * 16;
  size_t off[NB_ALL + 1];
  off[0] = 0;
  for (int q = 0; q < NB_ALL; ++q) off[q + 1] = off[q] + up256(sz[q]);
  void* ws = nullptr;
  int rc = workspace_slot(st, off[NB_ALL], WS_BOSON_GROUPED, &ws);
  if (rc) return rc;
  char* d = static_cast<char*>(ws);
  auto I32 = [&](int q) { return reinterpret_cast<int32_t*>(d + off[q]); };
  auto F64 = [&](int q) { return reinterpret_cast<double*>(d + off[q]); };
  auto C128 = [&](int q) { return reinterpret_cast<double2*>(d + off[q]); };
  const Piece pc[NP_UP] = {{in_modes, (size_t)n * 4},
                           {patterns, (size_t)(npat * n) * 4},
                           {sw.vcol.data(), (size_t)V * 4},
                           {sw.vcoef.data(), (size_t)V * 4},
                           {sw.vncoef.data(), (size_t)V * 4},
                           {sw.vncols.data(), (size_t)V * 4},
                           {sw.colmodes.data(), sw.colmodes.size() * 4},
                           {sw.collmodes.data(), sw.collmodes.size() * 4},
                           {sw.pv.data(), (size_t)(npat + 1) * 4},
                           {vlist.data(), (size_t)V * 4},
                           {vpos.data(), (size_t)V * 4},
                           {ent_pat.data(), (size_t)E * 4},
                           {mstart.data(), (size_t)(m + 1) * 4},
                           {mlist.data(), (size_t)E * 4},
                           {ent.data(), (size_t)E * sizeof(EntryDesc)},
                           {sw.coefs.data(), sw.coefs.size() * 8},
                           {sw.w.data(), (size_t)V * 8},
                           {moff.data(), (size_t)V * 8}};
  if ((rc = upload_at(st, d, off, pc, NP_UP))) return rc;
  // one gradient sweep launch per column count
  int64_t first = 0;
  for (auto& g : groups) {
    const int ncols = g.first;
    const int64_t cnt = (int64_t)g.second.size();
    hipLaunchKernelGGL(k_boson_gtab, dim3((unsigned)cnt), dim3(256), 0, st, reinterpret_cast<const double2*>(U), ldu,
                       I32(P_IN), n, rows, I32(P_VLIST) + first, I32(P_VCOL), ncols, I32(P_VCOEF), I32(P_VNCOEF),
                       I32(P_COLM), I32(P_COLLM), F64(P_COEFS), C128(B_TAB));
    rc = grad_sweep(C128(B_TAB), n, ncols, cnt, nullptr, C128(B_POUT) + first, C128(B_CM) + moff[g.second[0]], o,
                    st, cus);
    if (rc) return rc;
    first += cnt;
  }
  const unsigned pb = (unsigned)((npat + 255) / 256);
  hipLaunchKernelGGL(k_boson_combine, dim3((unsigned)npat), dim3(64), 0, st, C128(B_POUT), I32(P_VPOS), F64(P_W),
                     I32(P_PV), npat, o.plain ? 1 : 0, C128(B_PERMS));
  hipLaunchKernelGGL(k_boson_normalize, dim3(pb), dim3(256), 0, st, C128(B_PERMS), I32(P_IN), I32(P_PAT), n, npat,
                     weights, probs, C128(B_GPERM));
  if (E > 0)
    hipLaunchKernelGGL(k_boson_class_grad, dim3((unsigned)std::min<int64_t>(E * n, (int64_t)1 << 20)), dim3(64), 0,
                       st, C128(B_CM), reinterpret_cast<const int64_t*>(d + off[P_MOFF]), I32(P_VNCOLS), I32(P_VCOL),
                       I32(P_COLM), I32(P_VCOEF), F64(P_COEFS), F64(P_W), I32(P_PV),
                       reinterpret_cast<const EntryDesc*>(d + off[P_ENT]), E, n, C128(B_D));
  const int64_t tot = (int64_t)m * n;
  hipLaunchKernelGGL(k_boson_scatter_entries, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, C128(B_D),
                     C128(B_GPERM), I32(P_ENTPAT), I32(P_MSTART), I32(P_MLIST), m, n, reinterpret_cast<double2*>(dU),
                     lddu);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PH_OK : hip_fail(e, "boson grad launch");
}

}  // namespace ph

using namespace ph;

namespace ph {
static int boson_probs_grad_cols(hipStream_t st, const ph_c128* U, int32_t m, int64_t ldu, const int32_t* in_modes,
                                 int32_t n, const int32_t* patterns, int64_t n_patterns, const double* weights,
                                 double* probs, ph_c128* dU, int64_t lddu, const Opts& o, int cus);
}  // namespace ph

extern "C" int ph_boson_probs(const ph_c128* U, int32_t m, int64_t ldu, const int32_t* in_modes, int32_t n,
                              const int32_t* patterns, int64_t n_patterns, double* probs, const ph_opts* opt,
                              void* stream) {
  PH_TRACE("ph_boson_probs");
  Opts o;
  int rc = read_opts(opt, &o);
  if (rc) return rc;
  if ((rc = check_boson_args(U, m, ldu, in_modes, n, patterns, n_patterns, PH_NMAX))) return rc;
  if (n_patterns > 0 && !probs) return fail(PH_EINVAL, "probs is NULL");
  if (n_patterns == 0) return PH_OK;
  if (num_cus() <= 0) return PH_EUNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  if (n >= GROUP_MIN_SINGLES + 1 && o.algo == PH_GLYNN)
    return boson_probs_grouped(st, U, ldu, in_modes, n, patterns, n_patterns, o, probs);
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
  PH_TRACE("ph_boson_probs_grad");
  Opts o;
  int rc = read_opts(opt, &o);
  if (rc) return rc;
  if (o.algo != PH_GLYNN) return fail(PH_EINVAL, "the gradient supports PH_GLYNN only");
  if ((rc = check_boson_args(U, m, ldu, in_modes, n, patterns, n_patterns, PH_NMAX_GRAD))) return rc;
  if (n < 1) return fail(PH_EINVAL, "n=%d < 1", n);
  if (!dU) return fail(PH_EINVAL, "dU is NULL");
  const int64_t need_ld = o.du_full ? m : n;
  if (lddu < need_ld) return fail(PH_EINVAL, "lddu=%lld < %lld", (long long)lddu, (long long)need_ld);
  const int cus = num_cus();
  if (cus <= 0) return PH_EUNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  if (o.du_full) {
    // per-photon columns into a workspace of their own, then folded onto the
    // columns of U in a fixed order
    void* ws = nullptr;
    if ((rc = workspace_slot(st, (size_t)m * n * sizeof(double2), WS_BOSON_FOLD, &ws))) return rc;
    Opts on = o;
    on.du_full = false;
    rc = boson_probs_grad_cols(st, U, m, ldu, in_modes, n, patterns, n_patterns, weights, probs,
                               static_cast<ph_c128*>(ws), n, on, cus);
    if (rc) return rc;
    InModes im{};
    for (int k = 0; k < n; ++k) im.v[k] = in_modes[k];
    const int64_t tot = (int64_t)m * m;
    hipLaunchKernelGGL(k_boson_fold_photons, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                       static_cast<const double2*>(ws), n, im, m, reinterpret_cast<double2*>(dU), lddu);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? PH_OK : hip_fail(e, "boson fold launch");
  }
  return boson_probs_grad_cols(st, U, m, ldu, in_modes, n, patterns, n_patterns, weights, probs, dU, lddu, o, cus);
}

namespace ph {

// dU (m x n, row stride lddu): one column per input photon.
static int boson_probs_grad_cols(hipStream_t st, const ph_c128* U, int32_t m, int64_t ldu, const int32_t* in_modes,
                                 int32_t n, const int32_t* patterns, int64_t n_patterns, const double* weights,
                                 double* probs, ph_c128* dU, int64_t lddu, const Opts& o, int cus) {
  int rc;
  if (n >= GROUP_MIN_SINGLES + 1 && n_patterns > 0)
    return boson_grad_grouped(st, U, m, ldu, in_modes, n, patterns, n_patterns, weights, probs, dU, lddu, o, cus);
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

}  // namespace ph
