// Boson samples drawn by the chain rule over the output photons.
//
// The paper's simulation exists to produce boson-sampling outputs, whose
// probabilities are main-text Eq. (1), but it gives no sampling procedure.
// This is Clifford and Clifford's exact chain-rule algorithm (2018), written
// for batches of samples:
//
//   A = U[:, in_modes] (m x n, rows = output modes, distinct input modes);
//   the columns are taken in the order perm (one permutation per sample);
//   photon k = 1..n goes to mode r_k with probability proportional to
//     w_k(i) = |Per(A[(r_1..r_{k-1}, i), cols 1..k])|^2
//            = |sum_l A[i][col l] P_l|^2,
//   P_l = Per(A[(r_1..r_{k-1}), cols 1..k without l]), the minors along the
//   last row of any k x k matrix with those first k - 1 rows: the gradient
//   sweep of that matrix gives them all at once.
//
// Per step k the batch of k x k matrices (last row zero) goes through the
// gradient sweep; one block per sample then forms the m weights, their
// running sum in a fixed order, and takes the first mode whose running sum
// exceeds u_k times the total.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "permhip.h"
#include "ph_host.hpp"
#include "ph_internal.hpp"

namespace ph {

int row_minors_launch(const double2* tabs, int n_rows, int64_t batch, double2* out, hipStream_t st, int cus);
constexpr int MINORS_ROWS_MIN = 12;  // smaller steps take the gradient sweep

constexpr int SAMPLE_THREADS = 256;
constexpr int64_t SAMPLE_GROUP = 16384;  // samples per pass over the n steps

// a[i * n + j] = U[i][in_modes[j]]
__global__ void k_sample_columns(const double2* __restrict__ u, int64_t ldu, const int32_t* __restrict__ in_modes,
                                 int m, int n, double2* __restrict__ a) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < (int64_t)m * n) {
    const int64_t i = e / n;
    const int j = (int)(e % n);
    a[e] = u[i * ldu + in_modes[j]];
  }
}

// Matrix s of step k (k x k, row-major, contiguous): row t < k - 1 holds
// A[rows[s][t]][perm[s][l]] for l < k; the last row is zero (its minors do
// not depend on it).
__global__ void k_sample_build(const double2* __restrict__ a, int n, const int32_t* __restrict__ perms,
                               const int32_t* __restrict__ rows, int k, double2* __restrict__ mats) {
  const int64_t s = blockIdx.x;
  const int32_t* pm = perms + s * n;
  const int32_t* rw = rows + s * n;
  double2* out = mats + s * (int64_t)k * k;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int t = e / k, l = e % k;
    out[e] = t < k - 1 ? a[(int64_t)rw[t] * n + pm[l]] : make_double2(0.0, 0.0);
  }
}

// BB/FG table of step k for sample s (k - 1 rows, k columns, column-major,
// column stride k - 1): T[0] = A[rows, perm[0]], T[j] = -2 A[rows, perm[j]].
__global__ void k_sample_tables(const double2* __restrict__ a, int n, const int32_t* __restrict__ perms,
                                const int32_t* __restrict__ rows, int k, double2* __restrict__ tabs) {
  const int64_t s = blockIdx.x;
  const int32_t* pm = perms + s * n;
  const int32_t* rw = rows + s * n;
  const int nr = k - 1;
  double2* out = tabs + s * (int64_t)nr * k;
  for (int e = threadIdx.x; e < nr * k; e += blockDim.x) {
    const int j = e / nr, i = e % nr;
    double2 v = a[(int64_t)rw[i] * n + pm[j]];
    if (j > 0) v = make_double2(-2.0 * v.x, -2.0 * v.y);
    out[e] = v;
  }
}

__device__ __forceinline__ double weight_of(const double2* __restrict__ ai, const int* cols, const double2* P,
                                            int k) {
  double re = 0.0, im = 0.0;
  for (int l = 0; l < k; ++l) {
    const double2 x = ai[cols[l]];
    re = fma(x.x, P[l].x, fma(-x.y, P[l].y, re));
    im = fma(x.x, P[l].y, fma(x.y, P[l].x, im));
  }
  return re * re + im * im;
}

// Step k for sample s: the weights of all m modes and the choice.  The k
// minors of sample s are minors[s * stride + off + l], conjugated when conj
// is set (the gradient sweep writes conj(minor)); minors = NULL at k = 1,
// where the only minor is the empty permanent 1.
__global__ __launch_bounds__(SAMPLE_THREADS) void k_sample_step(const double2* __restrict__ a, int m, int n,
                                                                const int32_t* __restrict__ perms,
                                                                const double2* __restrict__ minors,
                                                                int64_t stride, int64_t off, int conj, int k,
                                                                const double* __restrict__ uniforms,
                                                                int32_t* __restrict__ rows) {
  __shared__ double2 P[PH_NMAX_GRAD];
  __shared__ int cols[PH_NMAX_GRAD];
  __shared__ double part[SAMPLE_THREADS];
  __shared__ int pick_slice;
  __shared__ double pick_base, pick_target;
  const int64_t s = blockIdx.x;
  const int t = threadIdx.x;
  if (t < k) {
    cols[t] = perms[s * n + t];
    if (minors) {
      const double2 g = minors[s * stride + off + t];
      P[t] = make_double2(g.x, conj ? -g.y : g.y);
    } else {
      P[t] = make_double2(1.0, 0.0);
    }
  }
  __syncthreads();
  // thread t owns the modes [m t / T, m (t + 1) / T)
  const int i0 = (int)((int64_t)m * t / SAMPLE_THREADS), i1 = (int)((int64_t)m * (t + 1) / SAMPLE_THREADS);
  double sum = 0.0;
  for (int i = i0; i < i1; ++i) sum += weight_of(a + (int64_t)i * n, cols, P, k);
  part[t] = sum;
  __syncthreads();
  if (t == 0) {
    double total = 0.0;
    for (int q = 0; q < SAMPLE_THREADS; ++q) total += part[q];
    const double target = uniforms[s * n + (k - 1)] * total;
    double base = 0.0;
    int slice = -1, last = -1;
    double last_base = 0.0;
    for (int q = 0; q < SAMPLE_THREADS; ++q) {
      if (part[q] > 0.0) {
        last = q;
        last_base = base;
      }
      if (base + part[q] > target && part[q] > 0.0) {
        slice = q;
        break;
      }
      base += part[q];
    }
    if (slice < 0) {  // target at the very top (rounding): the last mode with weight
      slice = last;
      base = last_base;
    }
    if (slice < 0) rows[s * n + (k - 1)] = 0;  // no positive weight (zero or NaN input): mode 0
    pick_slice = slice;
    pick_base = base;
    pick_target = target;
  }
  __syncthreads();
  if (t == pick_slice) {
    const double target = pick_target;
    double run = 0.0;
    int choice = -1, last = -1;
    for (int i = i0; i < i1; ++i) {
      const double w = weight_of(a + (int64_t)i * n, cols, P, k);
      run += w;
      if (w > 0.0) last = i;
      if (pick_base + run > target && w > 0.0) {
        choice = i;
        break;
      }
    }
    rows[s * n + (k - 1)] = choice >= 0 ? choice : last;
  }
}

// out[s] = rows[s] sorted ascending.
__global__ void k_sample_sort(const int32_t* __restrict__ rows, int n, int64_t nsamples, int32_t* __restrict__ out) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= nsamples) return;
  int32_t v[PH_NMAX_GRAD];
  for (int j = 0; j < n; ++j) v[j] = rows[s * n + j];
  for (int j = 1; j < n; ++j) {
    const int32_t x = v[j];
    int q = j - 1;
    while (q >= 0 && v[q] > x) {
      v[q + 1] = v[q];
      --q;
    }
    v[q + 1] = x;
  }
  for (int j = 0; j < n; ++j) out[s * n + j] = v[j];
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace ph

using namespace ph;

extern "C" int ph_boson_sample(const ph_c128* U, int32_t m, int64_t ldu, const int32_t* in_modes, int32_t n,
                               int64_t nsamples, const int32_t* perms, const double* uniforms, int32_t* out_modes,
                               const ph_opts* opt, void* stream) {
  PH_TRACE("ph_boson_sample");
  Opts o;
  int rc = read_opts(opt, &o);
  if (rc) return rc;
  if (o.algo != PH_GLYNN) return fail(PH_EINVAL, "ph_boson_sample supports PH_GLYNN only");
  if (m < 1) return fail(PH_EINVAL, "m=%d < 1", m);
  if (ldu < m) return fail(PH_EINVAL, "ldu=%lld < m=%d", (long long)ldu, m);
  if (n < 1) return fail(PH_EINVAL, "n=%d < 1", n);
  if (n > PH_NMAX_GRAD) return fail(PH_ERANGE, "n=%d > %d", n, PH_NMAX_GRAD);
  if (nsamples < 0) return fail(PH_EINVAL, "nsamples=%lld < 0", (long long)nsamples);
  if (!in_modes) return fail(PH_EINVAL, "in_modes is NULL");
  std::vector<char> seen(m, 0);
  for (int j = 0; j < n; ++j) {
    if (in_modes[j] < 0 || in_modes[j] >= m) return fail(PH_EINVAL, "in_modes[%d]=%d outside [0, %d)", j, in_modes[j], m);
    if (seen[in_modes[j]]) return fail(PH_EINVAL, "in_modes[%d]=%d repeats a mode", j, in_modes[j]);
    seen[in_modes[j]] = 1;
  }
  if (nsamples == 0) return PH_OK;
  if (!U || !out_modes || !perms || !uniforms) return fail(PH_EINVAL, "U, perms, uniforms or out_modes is NULL");
  std::vector<char> hit(n);
  for (int64_t s = 0; s < nsamples; ++s) {
    std::fill(hit.begin(), hit.end(), 0);
    for (int j = 0; j < n; ++j) {
      const int32_t c = perms[s * n + j];
      if (c < 0 || c >= n || hit[c]) return fail(PH_EINVAL, "perms[%lld] is not a permutation of 0..%d", (long long)s, n - 1);
      hit[c] = 1;
      const double u = uniforms[s * n + j];
      if (!(u >= 0.0 && u < 1.0)) return fail(PH_EINVAL, "uniforms[%lld][%d]=%g outside [0, 1)", (long long)s, j, u);
    }
  }
  const int cus = num_cus();
  if (cus <= 0) return PH_EUNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  const int64_t G = std::min<int64_t>(nsamples, SAMPLE_GROUP);
  // slot WS_SAMPLER: in_modes | perms, uniforms (one group, as uploaded) | A | rows | mats | grad
  size_t off[8];
  off[0] = 0;
  off[1] = off[0] + align256((size_t)n * 4);
  off[2] = off[1] + align256((size_t)G * n * 4);
  off[3] = off[2] + align256((size_t)G * n * 8);
  off[4] = off[3] + align256((size_t)m * n * 16);
  off[5] = off[4] + align256((size_t)G * n * 4);
  off[6] = off[5] + align256((size_t)G * n * n * 16);
  off[7] = off[6] + align256((size_t)G * n * n * 16);
  void* ws = nullptr;
  if ((rc = workspace_slot(st, off[7], WS_SAMPLER, &ws))) return rc;
  char* base = static_cast<char*>(ws);
  int32_t* d_in = reinterpret_cast<int32_t*>(base + off[0]);
  int32_t* d_perm = reinterpret_cast<int32_t*>(base + off[1]);
  double2* d_a = reinterpret_cast<double2*>(base + off[3]);
  int32_t* d_rows = reinterpret_cast<int32_t*>(base + off[4]);
  double2* d_mats = reinterpret_cast<double2*>(base + off[5]);
  double2* d_grad = reinterpret_cast<double2*>(base + off[6]);
  Piece pin[1] = {{in_modes, (size_t)n * 4}};
  if ((rc = upload(st, d_in, pin, 1))) return rc;
  const int64_t me = (int64_t)m * n;
  hipLaunchKernelGGL(k_sample_columns, dim3((unsigned)((me + 255) / 256)), dim3(256), 0, st,
                     reinterpret_cast<const double2*>(U), ldu, d_in, m, n, d_a);
  for (int64_t s0 = 0; s0 < nsamples; s0 += G) {
    const int64_t g = std::min(G, nsamples - s0);
    Piece pc[2] = {{perms + s0 * n, (size_t)g * n * 4}, {uniforms + s0 * n, (size_t)g * n * 8}};
    // this group's perms land at d_perm, its uniforms right after (256-aligned)
    if ((rc = upload(st, d_perm, pc, 2))) return rc;
    const double* du = reinterpret_cast<const double*>(reinterpret_cast<char*>(d_perm) + align256((size_t)g * n * 4));
    for (int k = 1; k <= n; ++k) {
      const double2* mn = nullptr;
      int64_t stride = 0, moff = 0;
      int conj = 0;
      if (k - 1 >= MINORS_ROWS_MIN) {
        // minors along the last row only (the grad buffer holds the tables)
        hipLaunchKernelGGL(k_sample_tables, dim3((unsigned)g), dim3(64), 0, st, d_a, n, d_perm, d_rows, k, d_grad);
        if ((rc = row_minors_launch(d_grad, k - 1, g, d_mats, st, cus))) return rc;
        mn = d_mats;
        stride = k;
      } else if (k >= 2) {
        hipLaunchKernelGGL(k_sample_build, dim3((unsigned)g), dim3(64), 0, st, d_a, n, d_perm, d_rows, k, d_mats);
        if ((rc = perm_grad_launch(d_mats, k, g, nullptr, nullptr, d_grad, o, st, cus))) return rc;
        mn = d_grad;
        stride = (int64_t)k * k;
        moff = (int64_t)(k - 1) * k;
        conj = 1;
      }
      hipLaunchKernelGGL(k_sample_step, dim3((unsigned)g), dim3(SAMPLE_THREADS), 0, st, d_a, m, n, d_perm, mn,
                         stride, moff, conj, k, du, d_rows);
    }
    if (o.unsorted) {
      hipError_t e = hipMemcpyAsync(out_modes + s0 * n, d_rows, (size_t)g * n * 4, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return hip_fail(e, "sample copy");
    } else {
      hipLaunchKernelGGL(k_sample_sort, dim3((unsigned)((g + 255) / 256)), dim3(256), 0, st, d_rows, n, g,
                         out_modes + s0 * n);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "sampler launch");
  }
  return PH_OK;
}
