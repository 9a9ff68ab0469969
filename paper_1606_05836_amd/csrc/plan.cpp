// Batched permanents: plan construction (size sort, work items, workspace,
// chunk-length tuning) and one hipGraph per plan holding the reset, prep,
// per-bucket sweep and finalize kernels.
#include <hip/hip_runtime.h>
#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "permhip.h"
#include "ph_host.hpp"
#include "ph_internal.hpp"

namespace ph {

// ----------------------------------------------------------- the plan object

struct KernelNode {
  hipGraphNode_t node = nullptr;
  hipKernelNodeParams params{};
  std::vector<void*> argv;  // pointers into `store`
  std::vector<char> store;  // argument values
};

struct PlanImpl {
  int dev = 0;
  int algo = 0;
  bool plain = false;
  int64_t batch = 0;
  std::vector<int32_t> n;
  std::vector<int64_t> off;   // element offsets of the matrices in A_packed
  std::vector<int32_t> c;     // chunk log2 per matrix (original order)
  std::vector<int32_t> ncols; // columns walked per matrix (original order)
  bool ext_tables = false;    // tables written by the caller: no prep kernel
  std::vector<int64_t> tab_off;  // element offset of each table in d_tabs (original order)
  int64_t n_items = 0;
  char* dmem = nullptr;
  MatDesc* d_mats = nullptr;
  WorkItem* d_items = nullptr;
  uint32_t* d_counters = nullptr;
  double4* d_parts = nullptr;
  double2* d_tabs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<KernelNode> nodes;  // reset, prep, buckets..., finalize
  int prep_idx = -1, fin_idx = -1;
  const void* last_a = nullptr;
  void* last_out = nullptr;
  hipStream_t last_stream = nullptr;
  bool launched = false;
  // recorded after every execution: a replay on another stream first waits
  // for it, since the graph's counters and partials are the plan's own
  hipEvent_t done = nullptr;
  // matrices of order >= SOLO_NMIN (and no caller-built tables) go through
  // the one-matrix sweep after the graph, which splits each term over two
  // lanes; the graph's finalize writes a placeholder that this overwrites
  std::vector<int64_t> solo;
  Opts opts;
  // waves per SIMD of each size bucket's sweep (0: as many as fit), and the
  // (chunk log2, waves) chosen per order
  int bucket_waves[NBUCKETS] = {};
  std::map<int, std::pair<int, int>> shape;
};

constexpr int SOLO_NMIN = 45;

template <typename T>
static void push_arg(KernelNode& k, const T& v) {
  const size_t at = k.store.size();
  k.store.resize(at + sizeof(T));
  std::memcpy(k.store.data() + at, &v, sizeof(T));
}

static void seal_args(KernelNode& k, const std::vector<size_t>& sizes) {
  k.argv.clear();
  size_t at = 0;
  for (size_t s : sizes) {
    k.argv.push_back(k.store.data() + at);
    at += s;
  }
  k.params.kernelParams = k.argv.data();
  k.params.extra = nullptr;
}

static void destroy_impl(PlanImpl* p) {
  if (!p) return;
  // each execution waited for the previous one, so the last stream's work
  // is the last to touch the plan's memory
  // (teardown: an error here has nothing left to undo, so it is not reported)
  if (p->launched) (void)hipStreamSynchronize(p->last_stream);
  if (p->done) (void)hipEventDestroy(p->done);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->dmem) (void)hipFree(p->dmem);
  delete p;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ------------------------------------------------------------- shape tuning

#ifndef PH_BUILD_ID
#define PH_BUILD_ID "unversioned"
#endif

// A tuned shape is valid for one build of the kernels (PH_BUILD_ID, a hash
// of the kernel sources set by the build), one device kind and one order.
struct TuneKey {
  std::string build, arch;
  int cus, n, algo, plain;
  bool operator<(const TuneKey& o) const {
    return std::tie(build, arch, cus, n, algo, plain) < std::tie(o.build, o.arch, o.cus, o.n, o.algo, o.plain);
  }
};
struct Shape {
  int c = 0;      // log2 chunk length
  int waves = 0;  // wavefronts per SIMD (workgroups of 4 waves per CU)
};

static std::mutex g_tune_mu;
static std::map<TuneKey, Shape> g_tune;
static bool g_tune_loaded = false;

// Range of chunk lengths a plan may use for order n.  The upper bound is the
// drift budget: row sums are re-seeded every 2^c steps, and c <= 14 keeps the
// accumulated rounding of the incremental updates far below the 1e-10
// relative-error target (measured: one 2^19-step chunk at n = 20 still stays
// under 2e-12).  A batch also wants >= 4 super-chunks per matrix so that all
// four wavefronts of a workgroup have work.
static void chunk_range(int n, int algo, int* lo, int* hi) {
  const int nb = gray_bits(n, algo);
  const int cmin = min_chunk_log2(nb);
  int h = std::min(14, nb - 8);
  h = std::max(h, cmin);
  h = std::min(h, nb);
  int l = std::max(cmin, std::min(h, 6));
  *lo = l;
  *hi = h;
}

static int default_chunk(int n, int algo) {
  int lo, hi;
  chunk_range(n, algo, &lo, &hi);
  return std::max(lo, std::min(hi, 12));
}

// Workgroups per CU the batched sweep of order n can hold (its bucket's
// kernel and LDS).
static int bucket_occupancy(int n, int algo) {
  const int bk = bucket_of(n);
  if (bk < 0) return 1;
  int per_cu = 0;
  const size_t lds = (size_t)BUCKET_HI[bk] * BUCKET_HI[bk] * sizeof(double2);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batched_kernel(bk, algo), 256, lds) != hipSuccess)
    return 1;
  return std::max(per_cu, 1);
}

static std::string cache_path() {
  const char* p = getenv("PERMHIP_TUNE_CACHE");
  return p ? std::string(p) : std::string();
}

// One entry per line: build arch cus n algo plain c waves.  Entries of other
// builds are kept in the file but never used.
static void load_cache_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const std::string path = cache_path();
  if (path.empty()) return;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    TuneKey k;
    Shape v;
    if (is >> k.build >> k.arch >> k.cus >> k.n >> k.algo >> k.plain >> v.c >> v.waves) g_tune[k] = v;
  }
}

// Written to a file of this process's own and renamed over the cache, so a
// process reading the cache never sees a half-written file (with several
// writers the last rename wins; every entry it drops is tuned again).
static void save_cache_locked() {
  const std::string path = cache_path();
  if (path.empty()) return;
  const std::string tmp = path + ".tmp." + std::to_string((long long)getpid());
  {
    std::ofstream f(tmp, std::ios::trunc);
    for (auto& kv : g_tune)
      f << kv.first.build << ' ' << kv.first.arch << ' ' << kv.first.cus << ' ' << kv.first.n << ' '
        << kv.first.algo << ' ' << kv.first.plain << ' ' << kv.second.c << ' ' << kv.second.waves << '\n';
    if (!f) {
      f.close();
      std::remove(tmp.c_str());
      return;
    }
  }
  if (std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
}

int plan_build(const int32_t* n_host, const int64_t* off_host, int64_t batch, const Opts& o, const int32_t* c_force,
               hipStream_t st, PlanImpl** out, const int32_t* ncols_host = nullptr);

// Terms one tuning run may sweep: candidates are timed on synthetic batches
// of about this many terms.  Orders with more terms per matrix than this are
// not timed (a run would be a whole permanent per candidate, seconds to
// hours); they take the default length and as many waves as fit, whose seed
// work is well under 1% of the sweep at that size.
constexpr int TUNE_LOG2_TERMS = 27;

// Time the batched sweep for every (chunk length, waves per SIMD) candidate
// on a synthetic batch of order-n matrices (about 2^27 terms) and keep the
// fastest.
static int tune_shape(int n, int algo, bool plain, hipStream_t st, Shape* out) {
  int lo, hi;
  chunk_range(n, algo, &lo, &hi);
  const int nb = gray_bits(n, algo);
  const int occ = bucket_occupancy(n, algo);
  if (nb > TUNE_LOG2_TERMS || (lo == hi && occ == 1)) {
    out->c = default_chunk(n, algo);
    out->waves = 0;
    return PH_OK;
  }
  const int64_t copies = (int64_t)1 << std::min(TUNE_LOG2_TERMS - nb, 14);
  const int64_t elems = copies * n * n;
  double2* a = nullptr;
  double2* res = nullptr;
  hipError_t e = hipMalloc(&a, elems * sizeof(double2) + copies * sizeof(double2) + 256);
  if (e != hipSuccess) return fail(PH_ENOMEM, "tuning buffer: %s", hipGetErrorString(e));
  res = a + elems;
  launch_fill_synthetic(a, elems, st);
  std::vector<int32_t> ns(copies, n), cs(copies);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = PH_OK;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
    rc = hip_fail(e, "tuning events");
  Opts o;
  o.algo = algo;
  o.plain = plain;
  float best = 1e30f;
  Shape best_s{default_chunk(n, algo), 0};
  for (int c = lo; c <= hi && rc == PH_OK; ++c) {
    for (int w = 1; w <= occ && rc == PH_OK; ++w) {
      std::fill(cs.begin(), cs.end(), c);
      o.waves = w;
      PlanImpl* p = nullptr;
      rc = plan_build(ns.data(), nullptr, copies, o, cs.data(), st, &p);
      if (rc) break;
      float ms = 1e30f;
      for (int rep = 0; rep < 2 && rc == PH_OK; ++rep) {
        if ((e = hipEventRecord(e0, st)) != hipSuccess) {
          rc = hip_fail(e, "tuning event");
          break;
        }
        if ((rc = plan_exec(p, a, res, st))) break;
        float t = 0;
        if ((e = hipEventRecord(e1, st)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
            (e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) {
          rc = hip_fail(e, "tuning timing");
          break;
        }
        if (rep == 1) ms = t;
      }
      destroy_impl(p);
      if (rc == PH_OK && ms < best) {
        best = ms;
        best_s = Shape{c, w == occ ? 0 : w};
      }
    }
  }
  // (teardown of the tuning buffers: errors here are not reported over rc)
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  (void)hipFree(a);
  *out = best_s;
  return rc;
}

// The shape for order n: from this process's tuning, the cache file, or a
// new tuning run (saved to both).
int tuned_shape(int n, int algo, bool plain, hipStream_t st, Shape* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  TuneKey k{PH_BUILD_ID, prop.gcnArchName, prop.multiProcessorCount, n, algo, plain ? 1 : 0};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_locked();
    auto it = g_tune.find(k);
    if (it != g_tune.end()) {
      *out = it->second;
      return PH_OK;
    }
  }
  Shape sh;
  int rc = tune_shape(n, algo, plain, st, &sh);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[k] = sh;
  save_cache_locked();
  *out = sh;
  return PH_OK;
}

// ------------------------------------------------------------- plan building

// Record reset -> prep -> sweep buckets (largest first) -> finalize as one
// graph and instantiate it.
static hipError_t build_graph(PlanImpl* p, const Opts& o, const std::vector<std::pair<int64_t, int64_t>>& bucket_items) {
  hipError_t e = hipGraphCreate(&p->graph, 0);
  if (e != hipSuccess) return e;
  const int cus = num_cus();
  const int64_t batch = p->batch;
  hipGraphNode_t prev = nullptr;
  p->nodes.clear();
  p->nodes.reserve(NBUCKETS + 3);
  auto add = [&](KernelNode&& kn) -> hipError_t {
    p->nodes.push_back(std::move(kn));
    KernelNode& k = p->nodes.back();
    k.params.kernelParams = k.argv.data();
    hipError_t r = hipGraphAddKernelNode(&k.node, p->graph, prev ? &prev : nullptr, prev ? 1 : 0, &k.params);
    if (r == hipSuccess) prev = k.node;
    return r;
  };
  {
    KernelNode k;
    uint32_t* cnt = p->d_counters;
    int count = NBUCKETS;
    push_arg(k, cnt);
    push_arg(k, count);
    seal_args(k, {sizeof(cnt), sizeof(count)});
    k.params.func = const_cast<void*>(reset_kernel());
    k.params.gridDim = dim3(1);
    k.params.blockDim = dim3(64);
    k.params.sharedMemBytes = 0;
    if ((e = add(std::move(k))) != hipSuccess) return e;
  }
  if (batch > 0 && !p->ext_tables) {
    KernelNode k;
    MatDesc* dm = p->d_mats;
    const double2* a = nullptr;
    int algo = o.algo;
    push_arg(k, dm);
    push_arg(k, a);
    push_arg(k, algo);
    seal_args(k, {sizeof(dm), sizeof(a), sizeof(algo)});
    k.params.func = const_cast<void*>(prep_batched_kernel());
    k.params.gridDim = dim3((unsigned)batch);
    k.params.blockDim = dim3(256);
    k.params.sharedMemBytes = 0;
    if ((e = add(std::move(k))) != hipSuccess) return e;
    p->prep_idx = (int)p->nodes.size() - 1;
  }
  for (int bk = NBUCKETS - 1; bk >= 0; --bk) {
    if (bucket_items[bk].first < 0) continue;
    KernelNode k;
    const void* kern = batched_kernel(bk, o.algo);
    const size_t lds = (size_t)BUCKET_HI[bk] * BUCKET_HI[bk] * sizeof(double2);
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, lds);
    if (e != hipSuccess) return e;
    per_cu = std::max(per_cu, 1);
    if (p->bucket_waves[bk] > 0) per_cu = std::min(per_cu, p->bucket_waves[bk]);
    const int64_t nit = bucket_items[bk].second - bucket_items[bk].first;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * per_cu, nit));
    MatDesc* dm = p->d_mats;
    WorkItem* di = p->d_items;
    int64_t ib = bucket_items[bk].first, ie = bucket_items[bk].second;
    uint32_t* cnt = p->d_counters + bk;
    double4* parts = p->d_parts;
    int plain = o.plain ? 1 : 0;
    push_arg(k, dm);
    push_arg(k, di);
    push_arg(k, ib);
    push_arg(k, ie);
    push_arg(k, cnt);
    push_arg(k, parts);
    push_arg(k, plain);
    seal_args(k, {sizeof(dm), sizeof(di), sizeof(ib), sizeof(ie), sizeof(cnt), sizeof(parts), sizeof(plain)});
    k.params.func = const_cast<void*>(kern);
    k.params.gridDim = dim3((unsigned)grid);
    k.params.blockDim = dim3(256);
    k.params.sharedMemBytes = (unsigned)lds;
    if ((e = add(std::move(k))) != hipSuccess) return e;
  }
  if (batch > 0) {
    KernelNode k;
    MatDesc* dm = p->d_mats;
    double4* parts = p->d_parts;
    int algo = o.algo, plain = o.plain ? 1 : 0;
    double2* outp = nullptr;
    push_arg(k, dm);
    push_arg(k, parts);
    push_arg(k, algo);
    push_arg(k, plain);
    push_arg(k, outp);
    seal_args(k, {sizeof(dm), sizeof(parts), sizeof(algo), sizeof(plain), sizeof(outp)});
    k.params.func = const_cast<void*>(finalize_batched_kernel());
    k.params.gridDim = dim3((unsigned)batch);
    k.params.blockDim = dim3(64);
    k.params.sharedMemBytes = 0;
    if ((e = add(std::move(k))) != hipSuccess) return e;
    p->fin_idx = (int)p->nodes.size() - 1;
  }
  return hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
}

int plan_build(const int32_t* n_host, const int64_t* off_host, int64_t batch, const Opts& o, const int32_t* c_force,
               hipStream_t st, PlanImpl** out, const int32_t* ncols_host) {
  int dev = 0;
  const hipError_t ed = hipGetDevice(&dev);
  if (ed != hipSuccess) return hip_fail(ed, "hipGetDevice");
  auto* p = new PlanImpl;
  p->dev = dev;
  p->algo = o.algo;
  p->plain = o.plain;
  p->opts = o;
  p->batch = batch;
  p->n.assign(n_host, n_host + batch);
  p->ext_tables = ncols_host != nullptr;
  if (ncols_host)
    p->ncols.assign(ncols_host, ncols_host + batch);
  else
    p->ncols = p->n;
  p->off.resize(batch);
  p->c.resize(batch);
  int64_t run = 0;
  for (int64_t b = 0; b < batch; ++b) {
    p->off[b] = off_host ? off_host[b] : run;
    run += (int64_t)p->n[b] * p->n[b];
  }
  // chunk lengths and waves per SIMD, per order: forced, from the options,
  // or tuned
  std::map<int, std::pair<int, int>>& chosen = p->shape;
  for (int64_t b = 0; b < batch; ++b) {
    const int n = p->n[b];
    if (n == 0) {
      p->c[b] = 0;
      continue;
    }
    if (c_force) {
      p->c[b] = c_force[b];
      chosen.emplace(n, std::make_pair(c_force[b], o.waves));
      continue;
    }
    auto it = chosen.find(n);
    if (it == chosen.end()) {
      Shape sh;
      if (o.chunk_log2 > 0) {
        sh.c = o.chunk_log2;
      } else {
        int rc = tuned_shape(n, o.algo, o.plain, st, &sh);
        if (rc) {
          destroy_impl(p);
          return rc;
        }
      }
      if (o.waves > 0) sh.waves = o.waves;
      const int nb = gray_bits(n, o.algo);
      sh.c = std::max(min_chunk_log2(nb), std::min(sh.c, nb));
      it = chosen.emplace(n, std::make_pair(sh.c, sh.waves)).first;
    }
    p->c[b] = it->second.first;
    if (p->ncols[b] != n) {
      // fewer columns: keep at least 256 chunks (one per lane of the four
      // wavefronts of a workgroup) where possible
      const int nb = gray_bits(p->ncols[b], o.algo);
      p->c[b] = std::max(min_chunk_log2(nb), std::min(p->c[b], std::max(min_chunk_log2(nb), nb - 8)));
    }
  }
  // each bucket's sweep runs with the waves chosen for the order that holds
  // most of its terms
  {
    std::map<int, double> terms_of_n;
    for (int64_t b = 0; b < batch; ++b)
      if (p->n[b] > 0) terms_of_n[p->n[b]] += std::ldexp(1.0, gray_bits(p->ncols[b], o.algo));
    double most[NBUCKETS] = {};
    for (auto& tn : terms_of_n) {
      const int bk = bucket_of(tn.first);
      if (bk >= 0 && tn.second > most[bk]) {
        most[bk] = tn.second;
        p->bucket_waves[bk] = chosen.count(tn.first) ? chosen[tn.first].second : o.waves;
      }
    }
  }
  // order: bucket (largest first), then n descending, then batch index
  std::vector<int64_t> order(batch);
  for (int64_t b = 0; b < batch; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return p->n[x] > p->n[y]; });
  // descriptors, tables, items
  std::vector<MatDesc> mats(batch);
  std::vector<WorkItem> items;
  std::vector<std::pair<int64_t, int64_t>> bucket_items(NBUCKETS, {-1, -1});
  size_t tab_elems = 0;
  for (int64_t s = 0; s < batch; ++s) {
    const int64_t b = order[s];
    const int n = p->n[b];
    MatDesc& m = mats[s];
    m.a_off = p->off[b];
    m.lda = n;
    m.tab = reinterpret_cast<double2*>((uintptr_t)(tab_elems * sizeof(double2)));  // relocated below
    if (p->ext_tables) {
      if (p->tab_off.empty()) p->tab_off.assign(batch, 0);
      p->tab_off[b] = (int64_t)tab_elems;
    }
    m.n = n;
    m.c = p->c[b];
    m.ncols = p->ncols[b];
    m.reserved = 0;
    m.out_index = b;
    tab_elems += table_elems(n);
    const int64_t first = (int64_t)items.size();
    const bool solo = !p->ext_tables && n >= SOLO_NMIN;
    if (solo) p->solo.push_back(b);
    if (n > 0 && !solo) {
      const int bk = bucket_of(n);
      const int nb = gray_bits(m.ncols, o.algo);
      const uint64_t nchunks = (uint64_t)1 << (nb - m.c);
      const int64_t nsuper = (int64_t)((nchunks + 63) / 64);
      for (int64_t s0 = 0; s0 < nsuper; s0 += 4) {
        WorkItem w;
        w.mat = (int32_t)s;
        w.rounds = (int32_t)std::min<int64_t>(4, nsuper - s0);
        w.super0 = s0;
        items.push_back(w);
      }
      auto& bi = bucket_items[bk];
      if (bi.first < 0) bi.first = first;
      bi.second = (int64_t)items.size();
    }
    m.part_begin = first * 4;
    m.part_end = (int64_t)items.size() * 4;
  }
  p->n_items = (int64_t)items.size();
  // one device allocation for everything the graph touches
  const size_t sz_mats = align256(batch * sizeof(MatDesc));
  const size_t sz_items = align256(std::max<size_t>(1, items.size()) * sizeof(WorkItem));
  const size_t sz_cnt = align256(NBUCKETS * sizeof(uint32_t));
  const size_t sz_parts = align256(std::max<size_t>(1, items.size() * 4) * sizeof(double4));
  const size_t sz_tabs = align256(std::max<size_t>(1, tab_elems) * sizeof(double2));
  hipError_t e = hipMalloc(&p->dmem, sz_mats + sz_items + sz_cnt + sz_parts + sz_tabs);
  if (e != hipSuccess) {
    destroy_impl(p);
    return fail(PH_ENOMEM, "plan workspace: %s", hipGetErrorString(e));
  }
  char* q = p->dmem;
  p->d_mats = reinterpret_cast<MatDesc*>(q);
  q += sz_mats;
  p->d_items = reinterpret_cast<WorkItem*>(q);
  q += sz_items;
  p->d_counters = reinterpret_cast<uint32_t*>(q);
  q += sz_cnt;
  p->d_parts = reinterpret_cast<double4*>(q);
  q += sz_parts;
  p->d_tabs = reinterpret_cast<double2*>(q);
  for (auto& m : mats) m.tab = p->d_tabs + reinterpret_cast<uintptr_t>(m.tab) / sizeof(double2);
  e = hipMemcpy(p->d_mats, mats.data(), batch * sizeof(MatDesc), hipMemcpyHostToDevice);
  if (e == hipSuccess && !items.empty())
    e = hipMemcpy(p->d_items, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    destroy_impl(p);
    return hip_fail(e, "plan upload");
  }
  e = build_graph(p, o, bucket_items);
  if (e != hipSuccess) {
    destroy_impl(p);
    return hip_fail(e, "plan graph");
  }
  *out = p;
  return PH_OK;
}

// Point the prep node at `a` and the finalize node at `out`.
static hipError_t set_io(PlanImpl* p, const double2* a, double2* out) {
  hipError_t e = hipSuccess;
  if (p->prep_idx >= 0 && a != p->last_a) {
    KernelNode& k = p->nodes[p->prep_idx];
    std::memcpy(k.argv[1], &a, sizeof(a));
    e = hipGraphExecKernelNodeSetParams(p->exec, k.node, &k.params);
    if (e != hipSuccess) return e;
    p->last_a = a;
  }
  if (p->fin_idx >= 0 && out != p->last_out) {
    KernelNode& k = p->nodes[p->fin_idx];
    std::memcpy(k.argv[4], &out, sizeof(out));
    e = hipGraphExecKernelNodeSetParams(p->exec, k.node, &k.params);
    if (e != hipSuccess) return e;
    p->last_out = out;
  }
  return e;
}

int plan_exec(PlanImpl* p, const double2* a, double2* out, hipStream_t st) {
  hipError_t e;
  if (!p->done) {
    e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreateWithFlags");
  }
  // the previous execution may still run on another stream: order this one
  // after it (same stream: already ordered)
  if (p->launched && st != p->last_stream) {
    e = hipStreamWaitEvent(st, p->done, 0);
    if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  }
  e = set_io(p, a, out);
  if (e != hipSuccess) return hip_fail(e, "hipGraphExecKernelNodeSetParams");
  e = hipGraphLaunch(p->exec, st);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  p->launched = true;
  p->last_stream = st;
  int rc = PH_OK;
  if (!p->solo.empty()) {
    const int cus = num_cus();
    if (cus <= 0) return PH_EUNSUPPORTED;
    for (int64_t b : p->solo) {
      const int n = p->n[b];
      rc = perm_single(a + p->off[b], n, n, out + b, p->opts, st, cus);
      if (rc) break;
    }
  }
  e = hipEventRecord(p->done, st);
  if (rc == PH_OK && e != hipSuccess) return hip_fail(e, "hipEventRecord");
  return rc;
}

double2* plan_table(PlanImpl* p, int64_t b) { return p->d_tabs + p->tab_off[b]; }

const std::vector<int64_t>& plan_table_offsets(PlanImpl* p) { return p->tab_off; }

double2* plan_tables_base(PlanImpl* p) { return p->d_tabs; }

static int check_batch_args(const int32_t* n_host, int64_t batch) {
  if (batch < 0) return fail(PH_EINVAL, "batch=%lld < 0", (long long)batch);
  if (batch > ((int64_t)1 << 30)) return fail(PH_EINVAL, "batch=%lld too large", (long long)batch);
  if (batch > 0 && !n_host) return fail(PH_EINVAL, "n_host is NULL");
  for (int64_t b = 0; b < batch; ++b) {
    if (n_host[b] < 0) return fail(PH_EINVAL, "n[%lld]=%d < 0", (long long)b, n_host[b]);
    if (n_host[b] > PH_NMAX) return fail(PH_ERANGE, "n[%lld]=%d > %d", (long long)b, n_host[b], PH_NMAX);
  }
  return PH_OK;
}

}  // namespace ph

using namespace ph;

extern "C" int ph_plan_create(const int32_t* n_host, const int64_t* offsets_host, int64_t batch, const ph_opts* opt,
                              void* stream, void** plan) {
  PH_TRACE("ph_plan_create");
  Opts o;
  int rc = read_opts(opt, &o);
  if (rc) return rc;
  if (!plan) return fail(PH_EINVAL, "plan is NULL");
  *plan = nullptr;
  if ((rc = check_batch_args(n_host, batch))) return rc;
  if (offsets_host)
    for (int64_t b = 0; b < batch; ++b)
      if (offsets_host[b] < 0) return fail(PH_EINVAL, "offsets[%lld] < 0", (long long)b);
  if (num_cus() <= 0) return PH_EUNSUPPORTED;
  PlanImpl* p = nullptr;
  rc = plan_build(n_host, offsets_host, batch, o, nullptr, (hipStream_t)stream, &p);
  if (rc) return rc;
  *plan = p;
  return PH_OK;
}

extern "C" int ph_plan_execute(void* plan, const ph_c128* A_packed, ph_c128* out, void* stream) {
  PH_TRACE("ph_plan_execute");
  if (!plan) return fail(PH_EINVAL, "plan is NULL");
  auto* p = static_cast<PlanImpl*>(plan);
  if (p->batch > 0 && (!A_packed || !out)) return fail(PH_EINVAL, "A_packed or out is NULL");
  int dev = 0;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != p->dev) return fail(PH_EINVAL, "plan was created on device %d, current device is %d", p->dev, dev);
  return plan_exec(p, reinterpret_cast<const double2*>(A_packed), reinterpret_cast<double2*>(out),
                   (hipStream_t)stream);
}

extern "C" int ph_plan_shape(const void* plan, int32_t n, int32_t* chunk_log2, int32_t* waves) {
  if (!plan) return fail(PH_EINVAL, "plan is NULL");
  if (!chunk_log2 || !waves) return fail(PH_EINVAL, "chunk_log2 or waves is NULL");
  const auto* p = static_cast<const PlanImpl*>(plan);
  auto it = p->shape.find(n);
  if (it == p->shape.end()) return fail(PH_EINVAL, "the plan holds no matrix of order %d", n);
  *chunk_log2 = it->second.first;
  *waves = it->second.second;
  return PH_OK;
}

extern "C" int ph_plan_destroy(void* plan) {
  if (!plan) return fail(PH_EINVAL, "plan is NULL");
  destroy_impl(static_cast<PlanImpl*>(plan));
  return PH_OK;
}

// ph_perm_batched keeps the last few plans (per device, stream, options and
// sizes) so that repeated calls with the same shapes skip planning and stay
// asynchronous.
namespace ph {
struct CacheKey {
  int dev;
  hipStream_t st;
  int algo, plain, chunk, waves;
  std::vector<int32_t> n;
  std::vector<int64_t> off;
  std::vector<int32_t> ncols;  // caller-built tables (empty for ordinary batches)
  bool operator==(const CacheKey& o) const {
    return dev == o.dev && st == o.st && algo == o.algo && plain == o.plain && chunk == o.chunk &&
           waves == o.waves && n == o.n && off == o.off && ncols == o.ncols;
  }
};
static std::mutex g_cache_mu;
static std::vector<std::pair<CacheKey, PlanImpl*>> g_plans;  // most recent last
constexpr size_t PLAN_CACHE = 4;
}  // namespace ph

extern "C" int ph_perm_batched(const ph_c128* A_packed, const int64_t* offsets_host, const int32_t* n_host,
                               int64_t batch, ph_c128* out, const ph_opts* opt, void* stream) {
  PH_TRACE("ph_perm_batched");
  Opts o;
  int rc = read_opts(opt, &o);
  if (rc) return rc;
  if ((rc = check_batch_args(n_host, batch))) return rc;
  if (batch > 0 && (!A_packed || !out)) return fail(PH_EINVAL, "A_packed or out is NULL");
  CacheKey key;
  hipError_t e = hipGetDevice(&key.dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  key.st = (hipStream_t)stream;
  key.algo = o.algo;
  key.plain = o.plain;
  key.chunk = o.chunk_log2;
  key.waves = o.waves;
  key.n.assign(n_host, n_host + batch);
  if (offsets_host) key.off.assign(offsets_host, offsets_host + batch);
  std::lock_guard<std::mutex> lk(g_cache_mu);
  PlanImpl* p = nullptr;
  for (size_t i = 0; i < g_plans.size(); ++i) {
    if (g_plans[i].first == key) {
      auto hit = g_plans[i];
      g_plans.erase(g_plans.begin() + i);
      g_plans.push_back(hit);
      p = hit.second;
      break;
    }
  }
  if (!p) {
    void* h = nullptr;
    rc = ph_plan_create(n_host, offsets_host, batch, opt, stream, &h);
    if (rc) return rc;
    p = static_cast<PlanImpl*>(h);
    if (g_plans.size() >= PLAN_CACHE) {
      destroy_impl(g_plans.front().second);  // waits for its stream first
      g_plans.erase(g_plans.begin());
    }
    g_plans.emplace_back(std::move(key), p);
  }
  return ph_plan_execute(p, A_packed, out, stream);
}

namespace ph {

// Batched sweep over caller-built tables (rows n[b], walked columns ncols[b]),
// through the same plan cache: `fill` enqueues the writes of the tables
// (plan_table / plan_tables_base) on `st`, then the plan runs and out[b]
// receives 2^-(n[b]-1) (BB/FG) times the sweep's sum for table b.
int plan_ext_run(const int32_t* n_host, const int32_t* ncols_host, int64_t batch, const Opts& o, hipStream_t st,
                 const std::function<int(PlanImpl*)>& fill, double2* out) {
  CacheKey key;
  const hipError_t e = hipGetDevice(&key.dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  key.st = st;
  key.algo = o.algo;
  key.plain = o.plain;
  key.chunk = o.chunk_log2;
  key.waves = o.waves;
  key.n.assign(n_host, n_host + batch);
  key.ncols.assign(ncols_host, ncols_host + batch);
  std::lock_guard<std::mutex> lk(g_cache_mu);
  PlanImpl* p = nullptr;
  for (size_t i = 0; i < g_plans.size(); ++i) {
    if (g_plans[i].first == key) {
      auto hit = g_plans[i];
      g_plans.erase(g_plans.begin() + i);
      g_plans.push_back(hit);
      p = hit.second;
      break;
    }
  }
  if (!p) {
    int rc = plan_build(n_host, nullptr, batch, o, nullptr, st, &p, ncols_host);
    if (rc) return rc;
    if (g_plans.size() >= PLAN_CACHE) {
      destroy_impl(g_plans.front().second);  // waits for its stream first
      g_plans.erase(g_plans.begin());
    }
    g_plans.emplace_back(std::move(key), p);
  }
  int rc = fill(p);
  if (rc) return rc;
  return plan_exec(p, nullptr, out, st);
}

}  // namespace ph
