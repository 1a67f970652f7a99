// Host side of the tridiagonal eigenvector library: argument checks,
// workspace layout, cluster-chain planning and the C-ABI entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include "te_host.h"
#include "te_plan.h"

namespace te {

thread_local int g_last_hip = 0;

int hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return TE_ERR_HIP;
}

namespace {

#define TE_CHECK(call)                          \
  do {                                          \
    hipError_t _e = (call);                     \
    if (_e != hipSuccess) return hip_fail(_e);  \
  } while (0)

// ---- per-phase device timing (hipEvents on the launch stream) ----
enum Phase { PH_SETUP, PH_BISECT, PH_CLUSTER, PH_INVIT, PH_TRANSPOSE, PH_SMALL, PH_COOP,
             PH_FINAL, PH_COUNT };

std::mutex g_tmu;
bool g_timing = false;
double g_ms[PH_COUNT] = {};
long long g_cnt[PH_COUNT] = {};

struct PhaseTimer {
  bool on;
  hipStream_t s;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;
  explicit PhaseTimer(hipStream_t st) : s(st) {
    std::lock_guard<std::mutex> lk(g_tmu);
    on = g_timing;
  }
  void begin(int ph) {
    if (!on) return;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
    (void)hipEventRecord(a, s);
    ev.push_back({ph, {a, b}});
  }
  void end() {
    if (!on || ev.empty()) return;
    (void)hipEventRecord(ev.back().second.second, s);
  }
  // Call after the stream has been synchronized.
  void collect() {
    if (!on) return;
    std::lock_guard<std::mutex> lk(g_tmu);
    for (auto &x : ev) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, x.second.first, x.second.second) == hipSuccess) {
        g_ms[x.first] += ms;
        g_cnt[x.first] += 1;
      }
    }
    release();
  }
  void release() {
    for (auto &x : ev) {
      (void)hipEventDestroy(x.second.first);
      (void)hipEventDestroy(x.second.second);
    }
    ev.clear();
  }
  ~PhaseTimer() { release(); }
};

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }
inline size_t even(size_t x) { return (x + 1) & ~(size_t)1; }

// Per-problem sizes of the workspace pieces (bytes, each aligned).  The
// interleaved iterate and LU factors (V, Ll, Lu1i, Lu2, Lu3) are read for the
// last time by k_transpose; Y, Yr, T and Tr are first written by the chain
// kernels, which run after it on the same stream, so both sets live in one
// region ("overlay") of the larger of their two sizes.
struct ProbLayout {
  size_t e2, nrm, pos, cls, clz, ncl, V, Y, Yr, T, overlay, Sw, Lrec, Lswb, prm, info;
  size_t total() const {
    return e2 + nrm + pos + cls + clz + ncl + overlay + Sw + Lrec + Lswb + prm + info;
  }
};

ProbLayout prob_layout(int n, int m) {
  ProbLayout L;
  const size_t nm = (size_t)n * (size_t)m;
  L.e2 = align_up(sizeof(double) * (size_t)std::max(n - 1, 1));
  L.nrm = align_up(sizeof(double) * (size_t)m);
  L.pos = align_up(sizeof(int) * (size_t)m);
  L.cls = align_up(sizeof(int) * (size_t)m);
  L.clz = align_up(sizeof(int) * (size_t)m);
  L.ncl = align_up(sizeof(int));
  L.V = align_up(sizeof(double) * nm);   // also each of Ll, Lu1i, Lu2, Lu3
  const size_t ldy = even((size_t)n), ldm = even((size_t)m);
  L.Y = align_up(sizeof(double) * ldy * (size_t)m);
  L.Yr = align_up(sizeof(double) * (size_t)n * ldm);
  L.T = align_up(sizeof(double) * ldm * ldm);   // also Tr
  L.overlay = std::max(5 * L.V, L.Y + L.Yr + 2 * L.T);
  L.Sw = align_up(nm);
  L.Lrec = align_up(4 * sizeof(double) * nm);
  L.Lswb = align_up(nm);
  L.prm = align_up(sizeof(Params));
  L.info = align_up(sizeof(int) * ((size_t)m + 1));
  return L;
}

// Bump allocator over a caller- or library-owned device block.
struct Carve {
  char *base;
  size_t off, cap;
  template <class T>
  T *take(size_t bytes) {
    T *p = reinterpret_cast<T *>(base + off);
    off += align_up(bytes);
    return p;
  }
};


// The workspace arrays of one problem (everything but prm and info), carved
// in the order of ProbLayout; the overlay region holds V, Ll, Lu1i, Lu2, Lu3
// and, later in the call, Y, Yr, T, Tr.
void carve_problem(Carve &cv, Prob &P, int n, int m) {
  const ProbLayout L = prob_layout(n, m);
  const size_t nm = (size_t)n * m;
  P.e2 = cv.take<double>(sizeof(double) * std::max(n - 1, 1));
  P.nrm = cv.take<double>(sizeof(double) * m);
  P.pos = cv.take<int>(sizeof(int) * m);
  P.cl_start = cv.take<int>(sizeof(int) * m);
  P.cl_size = cv.take<int>(sizeof(int) * m);
  P.ncl = cv.take<int>(sizeof(int));
  char *ov = cv.take<char>(L.overlay);
  P.V = reinterpret_cast<double *>(ov);
  P.Ll = reinterpret_cast<double *>(ov + L.V);
  P.Lu1i = reinterpret_cast<double *>(ov + 2 * L.V);
  P.Lu2 = reinterpret_cast<double *>(ov + 3 * L.V);
  P.Lu3 = reinterpret_cast<double *>(ov + 4 * L.V);
  P.ldy = (int)even((size_t)n);
  P.ldm = (int)even((size_t)m);
  P.Y = reinterpret_cast<double *>(ov);
  P.Yr = reinterpret_cast<double *>(ov + L.Y);
  P.T = reinterpret_cast<double *>(ov + L.Y + L.Yr);
  P.Tr = reinterpret_cast<double *>(ov + L.Y + L.Yr + L.T);
  P.Lsw = cv.take<unsigned char>(nm);
  P.Lrec = cv.take<double>(4 * sizeof(double) * nm);
  P.Lswb = cv.take<unsigned char>(nm);
}

// Everything one call needs after the problems are described.
struct Run {
  std::vector<Prob> hp;             // host copies of the problem descriptors
  std::vector<int64_t> loff;        // lane offsets (nprob + 1)
  Prob *dprobs = nullptr;
  int64_t *dloff = nullptr;
  int nmax = 0, mmax = 0;
  int64_t mtotal = 0;
};

size_t fixed_bytes(int nprob) {
  return align_up(sizeof(Prob) * (size_t)nprob) + align_up(sizeof(int64_t) * ((size_t)nprob + 1));
}

size_t chain_bytes(int nmax, int mmax, int nslots, int coop_wgs, int nitems) {
  size_t b = 0;
  b += align_up(sizeof(double) * chain_scratch_doubles(nmax, mmax, std::max(coop_wgs, 1)) *
                (size_t)std::max(nslots, 1));
  b += align_up(sizeof(ChainItem) * (size_t)std::max(nitems, 1));
  b += align_up(sizeof(Group) * (size_t)std::max(coop_wgs, 1));
  b += align_up(sizeof(int) * (size_t)std::max(coop_wgs, 1));      // wg_group
  b += align_up(sizeof(unsigned) * kBarWords * (size_t)std::max(coop_wgs, 1)); // barriers
  b += align_up(sizeof(int) * 2);                                  // abort flag, counter
  return b;
}

// Split the large clusters into cooperative groups: sizes proportional to the
// chain cost (size^2 * n), at least one workgroup each; with more clusters than
// workgroups, single-workgroup groups take clusters longest-first.
void plan_groups(const std::vector<ChainItem> &items, const std::vector<double> &cost, int nwg,
                 std::vector<Group> &groups, std::vector<int> &wg_group,
                 std::vector<ChainItem> &ordered) {
  groups.clear();
  ordered.clear();
  wg_group.assign((size_t)nwg, -1);
  const int K = (int)items.size();
  if (K == 0 || nwg <= 0) return;
  std::vector<int> idx(K);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  if (K <= nwg) {
    double tot = 0.0;
    for (int k = 0; k < K; k++) tot += cost[k];
    std::vector<int> g(K, 1);
    int used = K;
    // hand out the remaining workgroups by largest remaining cost per WG
    std::vector<double> share(K);
    for (int a = 0; a < K; a++) share[a] = cost[idx[a]] / tot * nwg;
    for (int a = 0; a < K; a++) {
      const int want = std::max(1, (int)share[a]);
      const int extra = std::min(want - 1, nwg - used);
      g[a] += std::max(extra, 0);
      used += std::max(extra, 0);
    }
    while (used < nwg) {  // leftovers to the most loaded per workgroup
      int best = 0;
      for (int a = 1; a < K; a++)
        if (cost[idx[a]] / g[a] > cost[idx[best]] / g[best]) best = a;
      g[best]++;
      used++;
    }
    int wg0 = 0;
    for (int a = 0; a < K; a++) {
      Group G{wg0, g[a], (int)ordered.size(), 1};
      ordered.push_back(items[idx[a]]);
      for (int w = 0; w < g[a]; w++) wg_group[wg0 + w] = (int)groups.size();
      groups.push_back(G);
      wg0 += g[a];
    }
  } else {
    std::vector<std::vector<int>> lists(nwg);
    std::vector<double> load(nwg, 0.0);
    for (int a = 0; a < K; a++) {
      int best = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      lists[best].push_back(idx[a]);
      load[best] += cost[idx[a]];
    }
    for (int w = 0; w < nwg; w++) {
      Group G{w, 1, (int)ordered.size(), (int)lists[w].size()};
      for (int k : lists[w]) ordered.push_back(items[k]);
      wg_group[w] = (int)groups.size();
      groups.push_back(G);
    }
  }
}

}  // namespace

Resolved resolve(const te_opts *o) {
  Resolved r{TE_DEFAULT_ITERS, TE_DEFAULT_SEED, 1e-3, 0, 0, TE_ORTH_CWY};
  if (o) {
    r.orth = o->orth;
    if (o->iters > 0) r.iters = o->iters;
    if (o->stop == TE_STOP_GROWTH) r.iters = -1;   // the kernels' encoding of the growth rule
    if (o->seed) r.seed = o->seed;
    if (o->cluster_rtol > 0.0) r.rtol = o->cluster_rtol;
    if (o->coop_wgs > 0) r.coop_wgs = o->coop_wgs;
    r.ws_budget = o->ws_budget;
  }
  return r;
}

DeviceLimits limits() {
  static std::mutex mu;
  static DeviceLimits cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DeviceLimits{};
  std::lock_guard<std::mutex> lk(mu);
  if (dev < 0 || dev >= 64) return DeviceLimits{};
  if (cache[dev].device != dev) {
    // Keep freed stream-ordered allocations in the device's default pool, so
    // repeated calls do not map and unmap their (possibly tens of GB of)
    // workspace every time.
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    DeviceLimits L;
    L.device = dev;
    L.coop = coop_max_wgs(dev);
    L.small = small_max_wgs(dev);
    L.mgs = mgs_max_wgs(dev);
    cache[dev] = L;
  }
  return cache[dev];
}

void DeviceGate::lock_shared() {
  std::unique_lock<std::mutex> lk(mu);
  cv.wait(lk, [&] { return !writer && writers_waiting == 0; });
  readers++;
}

void DeviceGate::unlock_shared() {
  {
    std::lock_guard<std::mutex> lk(mu);
    readers--;
  }
  cv.notify_all();
}

void DeviceGate::lock_exclusive() {
  std::unique_lock<std::mutex> lk(mu);
  writers_waiting++;
  cv.wait(lk, [&] { return !writer && readers == 0; });
  writers_waiting--;
  writer = true;
}

void DeviceGate::unlock_exclusive() {
  {
    std::lock_guard<std::mutex> lk(mu);
    writer = false;
  }
  cv.notify_all();
}

DeviceGate &device_gate(int device) {
  static DeviceGate gates[64];
  return gates[device & 63];
}

SharedHold::SharedHold() {
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64) g_ = &device_gate(dev);
  acquire();
}

void SharedHold::acquire() {
  if (g_ && !held_) {
    g_->lock_shared();
    held_ = true;
  }
}

void SharedHold::release() {
  if (g_ && held_) {
    g_->unlock_shared();
    held_ = false;
  }
}

namespace {

// Library-owned workspace blocks of one call: freed on every return path.
// On an early (error) return the stream is synchronized first, so that no
// enqueued kernel still uses the memory when it is released.
struct OwnedBlocks {
  hipStream_t s;
  std::vector<void *> blocks;
  bool released = false;
  explicit OwnedBlocks(hipStream_t st) : s(st) {}
  ~OwnedBlocks() {
    if (released || blocks.empty()) return;
    (void)hipStreamSynchronize(s);
    for (void *p : blocks) (void)hipFreeAsync(p, s);
    (void)hipStreamSynchronize(s);
    (void)hipGetLastError();
  }
  OwnedBlocks(const OwnedBlocks &) = delete;
  OwnedBlocks &operator=(const OwnedBlocks &) = delete;
};

// Launch the cooperative chain kernel under the device gate (see DeviceGate)
// and wait for it to complete.  The caller holds no shared hold and has
// synchronized its stream.
int run_coop(const DeviceLimits &lim, const Prob *probs, const ChainItem *items,
             const Group *groups, const int *wg_group, unsigned *bars, int *abort_flag,
             ChainScratch scr, int nwg, int iters, PhaseTimer &tm, hipStream_t stream) {
  DeviceGate &g = device_gate(lim.device);
  std::lock_guard<std::mutex> one(g.coop);
  if (!g.started_host) {
    int *h = nullptr;
    if (hipHostMalloc((void **)&h, sizeof(int) * (size_t)lim.coop, hipHostMallocCoherent) ==
        hipSuccess) {
      int *dp = nullptr;
      if (hipHostGetDevicePointer((void **)&dp, h, 0) == hipSuccess) {
        g.started_host = h;
        g.started_dev = dp;
        g.started_cap = lim.coop;
      } else {
        (void)hipHostFree(h);
      }
    }
    (void)hipGetLastError();
  }
  int *started = (g.started_dev && nwg <= g.started_cap) ? g.started_dev : nullptr;
  if (started) {
    for (int w = 0; w < nwg; w++) __atomic_store_n(&g.started_host[w], 0, __ATOMIC_RELAXED);
    __atomic_thread_fence(__ATOMIC_SEQ_CST);
  }
  g.lock_exclusive();
  tm.begin(PH_COOP);
  hipError_t e = launch_chain_coop(probs, items, groups, wg_group, bars, abort_flag, started, scr,
                                   nwg, iters, stream);
  tm.end();
  if (e != hipSuccess) {
    g.unlock_exclusive();
    return hip_fail(e);
  }
  // Hold the device until every workgroup is resident (or the grid is done).
  for (;;) {
    if (started) {
      int cnt = 0;
      for (int w = 0; w < nwg; w++) cnt += __atomic_load_n(&g.started_host[w], __ATOMIC_ACQUIRE);
      if (cnt == nwg) break;
    }
    const hipError_t q = hipStreamQuery(stream);
    if (q == hipSuccess) break;
    if (q != hipErrorNotReady) {
      g.unlock_exclusive();
      return hip_fail(q);
    }
    std::this_thread::sleep_for(std::chrono::microseconds(started ? 10 : 200));
  }
  g.unlock_exclusive();
  TE_CHECK(hipStreamSynchronize(stream));  // one cooperative grid in flight at a time
  return 0;
}

}  // namespace

// The whole method for a set of problems.  ws may be null (library-owned
// workspace via hipMallocAsync).  W_given: device array of mtotal eigenvalues
// or null.
int solve_problems(const std::vector<ProblemDesc> &pd, const double *W_given, const Resolved &opt,
                   void *ws, size_t ws_bytes, int *info, hipStream_t stream) {
  const int nprob = (int)pd.size();
  DeviceLimits lim = limits();
  if (lim.device < 0 || lim.coop <= 0 || lim.small <= 0) return TE_ERR_NO_DEVICE;
  const bool mgs = opt.orth == TE_ORTH_MGS;
  if (mgs) {
    if (lim.mgs <= 0) return TE_ERR_NO_DEVICE;
    for (const auto &D : pd)
      if (D.n > TE_MGS_MAX_N) return TE_ERR_UNSUPPORTED;
  }
  SharedHold hold;

  Run R;
  R.hp.resize(nprob);
  R.loff.resize(nprob + 1);
  R.loff[0] = 0;
  size_t per_prob = 0;
  for (int b = 0; b < nprob; b++) {
    const int m = pd[b].iu - pd[b].il + 1;
    R.nmax = std::max(R.nmax, pd[b].n);
    R.mmax = std::max(R.mmax, m);
    R.loff[b + 1] = R.loff[b] + m;
    per_prob += prob_layout(pd[b].n, m).total();
  }
  R.mtotal = R.loff[nprob];

  // Workspace: fixed part + problems; the chain part is sized after planning.
  const size_t first_bytes = fixed_bytes(nprob) + per_prob;
  bool own = (ws == nullptr);
  char *base = static_cast<char *>(ws);
  OwnedBlocks owned(stream);
  if (own) {
    TE_CHECK(hipMallocAsync((void **)&base, first_bytes, stream));
    owned.blocks.push_back(base);
  } else if (ws_bytes < first_bytes) {
    return TE_ERR_WORKSPACE;
  }
  Carve cv{base, 0, own ? first_bytes : ws_bytes};
  R.dprobs = cv.take<Prob>(sizeof(Prob) * nprob);
  R.dloff = cv.take<int64_t>(sizeof(int64_t) * (nprob + 1));
  std::vector<Params> hprm(nprob);
  for (int b = 0; b < nprob; b++) {
    const int n = pd[b].n, m = pd[b].iu - pd[b].il + 1;
    Prob &P = R.hp[b];
    std::memset(&P, 0, sizeof(P));
    P.d = pd[b].d;
    P.e = pd[b].e;
    P.n = n;
    P.m = m;
    P.ldz = pd[b].ldz;
    P.kbase = pd[b].il;
    P.W = pd[b].W;
    P.Z = pd[b].Z;
    carve_problem(cv, P, n, m);
    P.prm = cv.take<Params>(sizeof(Params));
    int *pinfo = cv.take<int>(sizeof(int) * ((size_t)m + 1));
    P.info = pd[b].info ? pd[b].info : (info && nprob == 1) ? info : pinfo;
    std::memset(&hprm[b], 0, sizeof(Params));
    hprm[b].rtol = opt.rtol;
  }
  TE_CHECK(hipMemcpyAsync(R.dprobs, R.hp.data(), sizeof(Prob) * nprob, hipMemcpyHostToDevice,
                          stream));
  TE_CHECK(hipMemcpyAsync(R.dloff, R.loff.data(), sizeof(int64_t) * (nprob + 1),
                          hipMemcpyHostToDevice, stream));
  for (int b = 0; b < nprob; b++) {
    TE_CHECK(hipMemcpyAsync(R.hp[b].prm, &hprm[b], sizeof(Params), hipMemcpyHostToDevice, stream));
    TE_CHECK(launch_fill_i32(R.hp[b].info, (size_t)R.hp[b].m + 1, 0, stream));
  }

  // a1-a6
  PhaseTimer tm(stream);
  tm.begin(PH_SETUP);
  TE_CHECK(launch_setup(R.dprobs, nprob, stream));
  tm.end();
  tm.begin(PH_BISECT);
  if (W_given) TE_CHECK(launch_copy_w(R.dprobs, nprob, R.dloff, R.mtotal, W_given, stream));
  else TE_CHECK(launch_bisect(R.dprobs, nprob, R.dloff, R.mtotal, stream));
  tm.end();
  tm.begin(PH_CLUSTER);
  TE_CHECK(launch_cluster(R.dprobs, nprob, stream));
  tm.end();
  tm.begin(PH_INVIT);
  TE_CHECK(launch_invit(R.dprobs, nprob, R.dloff, R.mtotal, opt.iters, opt.seed, stream));
  tm.end();
  tm.begin(PH_TRANSPOSE);
  TE_CHECK(launch_transpose(R.dprobs, nprob, R.nmax, R.mmax, stream));
  tm.end();

  // Cluster tables back to the host for the chain plan.
  std::vector<int> ncl(nprob);
  std::vector<std::vector<int>> cst(nprob), csz(nprob);
  for (int b = 0; b < nprob; b++)
    TE_CHECK(hipMemcpyAsync(&ncl[b], R.hp[b].ncl, sizeof(int), hipMemcpyDeviceToHost, stream));
  TE_CHECK(hipStreamSynchronize(stream));
  for (int b = 0; b < nprob; b++) {
    cst[b].resize(std::max(ncl[b], 1));
    csz[b].resize(std::max(ncl[b], 1));
    if (ncl[b] > 0) {
      TE_CHECK(hipMemcpyAsync(cst[b].data(), R.hp[b].cl_start, sizeof(int) * ncl[b],
                              hipMemcpyDeviceToHost, stream));
      TE_CHECK(hipMemcpyAsync(csz[b].data(), R.hp[b].cl_size, sizeof(int) * ncl[b],
                              hipMemcpyDeviceToHost, stream));
    }
  }
  TE_CHECK(hipStreamSynchronize(stream));

  // chains (clusters of two or more) and the kernel each runs in (te_plan.h)
  std::vector<ChainItem> chains;
  std::vector<int> chain_n, chain_size;
  for (int b = 0; b < nprob; b++) {
    for (int c = 0; c < ncl[b]; c++) {
      if (csz[b][c] < 2) continue;
      chains.push_back(ChainItem{b, cst[b][c], csz[b][c], 0});
      chain_n.push_back(R.hp[b].n);
      chain_size.push_back(csz[b][c]);
    }
  }
  const std::vector<char> kern = chain_kernels(chain_n, chain_size, (size_t)lim.coop, mgs);
  std::vector<ChainItem> small_items, large_items;
  std::vector<double> small_cost, large_cost;
  for (int pass = 0; pass < 2; pass++) {   // cooperative chains first, promoted ones after
    for (size_t k = 0; k < chains.size(); k++) {
      const double cost = (double)chain_size[k] * chain_size[k] * chain_n[k];
      if (pass == 0 && kern[k] == kChainCoop) {
        large_items.push_back(chains[k]);
        large_cost.push_back(cost);
      } else if (pass == 1 && kern[k] == kChainPromoted) {
        large_items.push_back(chains[k]);
        large_cost.push_back(cost);
      } else if (pass == 1 && kern[k] == kChainOneWg) {
        small_items.push_back(chains[k]);
        small_cost.push_back(cost);
      }
    }
  }
  {  // small items longest first
    std::vector<int> idx(small_items.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(),
                     [&](int a, int b) { return small_cost[a] > small_cost[b]; });
    std::vector<ChainItem> s2;
    for (int k : idx) s2.push_back(small_items[k]);
    small_items.swap(s2);
  }
  int coop_nwg = std::min(lim.coop, opt.coop_wgs > 0 ? opt.coop_wgs : lim.coop);
  std::vector<Group> groups;
  std::vector<int> wg_group;
  std::vector<ChainItem> large_ordered;
  plan_groups(large_items, large_cost, coop_nwg, groups, wg_group, large_ordered);
  const int small_nwg = std::min((int)small_items.size(), mgs ? lim.mgs : lim.small);
  const int nslots = std::max(small_nwg, (int)groups.size());
  const int nitems = (int)(small_items.size() + large_ordered.size());

  char *cbase = nullptr;
  const size_t cbytes = chain_bytes(R.nmax, R.mmax, nslots, coop_nwg, nitems);
  if (own) {
    TE_CHECK(hipMallocAsync((void **)&cbase, cbytes, stream));
    owned.blocks.push_back(cbase);
  } else {
    if (cv.off + cbytes > cv.cap) return TE_ERR_WORKSPACE;
    cbase = base + cv.off;
  }
  Carve cc{cbase, 0, cbytes};
  ChainScratch scr;
  scr.stride = chain_scratch_doubles(R.nmax, R.mmax, std::max(coop_nwg, 1));
  scr.base = cc.take<double>(sizeof(double) * scr.stride * std::max(nslots, 1));
  ChainItem *ditems = cc.take<ChainItem>(sizeof(ChainItem) * std::max(nitems, 1));
  Group *dgroups = cc.take<Group>(sizeof(Group) * std::max(coop_nwg, 1));
  int *dwg = cc.take<int>(sizeof(int) * std::max(coop_nwg, 1));
  unsigned *dbars = cc.take<unsigned>(sizeof(unsigned) * kBarWords * std::max(coop_nwg, 1));
  int *dflags = cc.take<int>(sizeof(int) * 2);   // [0] abort, [1] work counter

  std::vector<ChainItem> all_items(small_items);
  all_items.insert(all_items.end(), large_ordered.begin(), large_ordered.end());
  if (nitems > 0)
    TE_CHECK(hipMemcpyAsync(ditems, all_items.data(), sizeof(ChainItem) * nitems,
                            hipMemcpyHostToDevice, stream));
  TE_CHECK(launch_fill_i32(dflags, 2, 0, stream));
  if (small_nwg > 0) {
    tm.begin(PH_SMALL);
    if (mgs)
      TE_CHECK(launch_chain_mgs(R.dprobs, ditems, (int)small_items.size(), nullptr, dflags + 1,
                                dflags, scr, small_nwg, opt.iters, stream));
    else
      TE_CHECK(launch_chain_small(R.dprobs, ditems, (int)small_items.size(), dflags + 1, dflags,
                                  scr, small_nwg, opt.iters, stream));
    tm.end();
  }
  if (!groups.empty()) {
    std::vector<Group> g2(groups);
    for (auto &G : g2) G.it0 += (int)small_items.size();
    TE_CHECK(hipMemcpyAsync(dgroups, g2.data(), sizeof(Group) * g2.size(), hipMemcpyHostToDevice,
                            stream));
    TE_CHECK(hipMemcpyAsync(dwg, wg_group.data(), sizeof(int) * coop_nwg, hipMemcpyHostToDevice,
                            stream));
    TE_CHECK(launch_fill_i32((int *)dbars, kBarWords * (size_t)coop_nwg, 0, stream));
    TE_CHECK(hipStreamSynchronize(stream));
    hold.release();
    const int rc = run_coop(lim, R.dprobs, ditems, dgroups, dwg, dbars, dflags, scr, coop_nwg,
                            opt.iters, tm, stream);
    hold.acquire();
    if (rc) return rc;
  }
  tm.begin(PH_FINAL);
  TE_CHECK(launch_finalize(R.dprobs, nprob, R.dloff, R.mtotal, stream));
  tm.end();
  int abort_flag = 0;
  TE_CHECK(hipMemcpyAsync(&abort_flag, dflags, sizeof(int), hipMemcpyDeviceToHost, stream));
  TE_CHECK(hipStreamSynchronize(stream));
  tm.collect();
  if (own) {
    owned.released = true;
    TE_CHECK(hipFreeAsync(cbase, stream));
    TE_CHECK(hipFreeAsync(base, stream));
    TE_CHECK(hipStreamSynchronize(stream));
  }
  return abort_flag ? TE_ERR_KERNEL : 0;
}

// Workspace bytes solve_problems needs for a set of problems (upper bound).
size_t problems_bytes(const std::vector<ProblemDesc> &pd, size_t b0, size_t b1,
                      const DeviceLimits &lim) {
  size_t bytes = fixed_bytes((int)(b1 - b0));
  int nmax = 0, mmax = 0, msum = 0;
  for (size_t b = b0; b < b1; b++) {
    const int m = pd[b].iu - pd[b].il + 1;
    bytes += prob_layout(pd[b].n, m).total();
    nmax = std::max(nmax, pd[b].n);
    mmax = std::max(mmax, m);
    msum += m;
  }
  return bytes + chain_bytes(nmax, mmax, std::max({lim.small, lim.coop, lim.mgs}), lim.coop, msum);
}

uint64_t default_budget() {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return (uint64_t)8 << 30;
  const uint64_t cap = (uint64_t)64 << 30;
  return std::min<uint64_t>(cap, fr / 2);
}

// Consecutive problems grouped greedily into sub-batches that fit the budget.
int solve_batched(const std::vector<ProblemDesc> &pd, const Resolved &opt, hipStream_t stream) {
  DeviceLimits lim = limits();
  if (lim.device < 0 || lim.coop <= 0 || lim.small <= 0) return TE_ERR_NO_DEVICE;
  const uint64_t budget = opt.ws_budget ? opt.ws_budget : default_budget();
  size_t b0 = 0;
  while (b0 < pd.size()) {
    size_t b1 = b0 + 1;
    if (problems_bytes(pd, b0, b1, lim) > budget) return TE_ERR_WORKSPACE;
    while (b1 < pd.size() && problems_bytes(pd, b0, b1 + 1, lim) <= budget) b1++;
    std::vector<ProblemDesc> sub(pd.begin() + b0, pd.begin() + b1);
    const int rc = solve_problems(sub, nullptr, opt, nullptr, 0, nullptr, stream);
    if (rc) return rc;
    b0 = b1;
  }
  return 0;
}


// Argument checks of the batched entry points (positions as in
// tridiag_eigvecs_batched) and the problem descriptors.
int batch_descs(const double *d_all, const double *e_all, const int64_t *off, const int *il,
                const int *iu, double *W_all, const int64_t *woff, double *Z_all,
                const int64_t *zoff, int B, const te_opts *opt, std::vector<ProblemDesc> &pd) {
  if (!d_all) return -1;
  if (!off) return -3;
  if (!il) return -4;
  if (!iu) return -5;
  if (!W_all) return -6;
  if (!woff) return -7;
  if (!Z_all) return -8;
  if (!zoff) return -9;
  if (B < 1) return -10;
  if (opt && (opt->iters < 0 || opt->cluster_rtol < 0.0 || opt->coop_wgs < 0 ||
              (opt->orth != TE_ORTH_CWY && opt->orth != TE_ORTH_MGS) ||
              (opt->stop != TE_STOP_FIXED && opt->stop != TE_STOP_GROWTH))) return -11;
  pd.assign((size_t)B, ProblemDesc{});
  bool any_e = false;
  for (int b = 0; b < B; b++) {
    const int64_t nb = off[b + 1] - off[b];
    if (nb < 1 || nb > (1 << 30)) return -3;
    if (il[b] < 1 || il[b] > nb) return -4;
    if (iu[b] < il[b] || iu[b] > nb) return -5;
    if (nb > 1) any_e = true;
    pd[b].d = d_all + off[b];
    pd[b].e = e_all ? e_all + (off[b] - b) : nullptr;
    pd[b].n = (int)nb;
    pd[b].il = il[b];
    pd[b].iu = iu[b];
    pd[b].W = W_all + woff[b];
    pd[b].Z = Z_all + zoff[b];
    pd[b].ldz = (int)nb;
  }
  if (any_e && !e_all) return -2;
  return 0;
}

// ---------------------------------------------------------------------------
// Graph-captured batched path.  The batch is cut into segments whose
// workspace fits the budget (consecutive problems, as in solve_batched); each
// segment runs the whole method with every step on the device: the chain plan
// comes from k_plan_* instead of a host round trip, and every chain (whatever
// its size) runs in one workgroup of the persistent small-chain kernel.  All
// segments are captured into one graph; its launch is one hipGraphLaunch.
// Segments share one workspace region (they run one after another); their
// descriptors, parameters and info flags live in per-segment regions written
// once at creation.
// ---------------------------------------------------------------------------
namespace {

struct GraphSeg {
  int nprob = 0;
  Prob *dprobs = nullptr;
  int64_t *dloff = nullptr;
  int nmax = 0, mmax = 0;
  int64_t mtotal = 0;
  int *info = nullptr;   // contiguous info arrays of the segment's problems
  size_t info_ints = 0;
  ChainScratch scr{};
  ChainItem *items = nullptr;
  int item_cap = 0;
  int *nitems = nullptr, *bins = nullptr;
  int *flags = nullptr;  // abort, counter (in the segment's own region)
};

size_t seg_fixed_bytes(const std::vector<ProblemDesc> &pd, size_t b0, size_t b1) {
  size_t b = fixed_bytes((int)(b1 - b0)) + align_up(sizeof(int) * 2);  // + abort flag, counter
  for (size_t k = b0; k < b1; k++)
    b += align_up(sizeof(Params)) + align_up(sizeof(int) * ((size_t)(pd[k].iu - pd[k].il + 1) + 1));
  return b;
}

size_t seg_shared_bytes(const std::vector<ProblemDesc> &pd, size_t b0, size_t b1, int nslots) {
  size_t b = 0;
  int nmax = 0, mmax = 0;
  size_t cap = 0;
  for (size_t k = b0; k < b1; k++) {
    const int m = pd[k].iu - pd[k].il + 1;
    const ProbLayout L = prob_layout(pd[k].n, m);
    b += L.total() - L.prm - L.info;
    nmax = std::max(nmax, pd[k].n);
    mmax = std::max(mmax, m);
    cap += (size_t)(m / 2);
  }
  b += align_up(sizeof(double) * chain_scratch_doubles(nmax, mmax, 1) * (size_t)std::max(nslots, 1));
  b += align_up(sizeof(ChainItem) * std::max<size_t>(cap, 1));
  b += align_up(sizeof(int) * (2 * kPlanBins + 4));
  return b;
}

// Cut [0, B) into consecutive segments of at most `budget` bytes each.
bool plan_segments(const std::vector<ProblemDesc> &pd, int nslots, uint64_t budget,
                   std::vector<std::pair<size_t, size_t>> &seg) {
  seg.clear();
  size_t b0 = 0;
  while (b0 < pd.size()) {
    size_t b1 = b0 + 1;
    auto need = [&](size_t e) { return seg_fixed_bytes(pd, b0, e) + seg_shared_bytes(pd, b0, e, nslots); };
    if (need(b1) > budget) return false;
    while (b1 < pd.size() && need(b1 + 1) <= budget) b1++;
    seg.push_back({b0, b1});
    b0 = b1;
  }
  return true;
}

// Carve segment [b0, b1): fixed part from fx, problem arrays and chain state
// from sh.  Uploads the descriptors and parameters (synchronous copies).
int carve_segment(const std::vector<ProblemDesc> &pd, size_t b0, size_t b1, const Resolved &opt,
                  int nslots, Carve &fx, Carve &sh, GraphSeg &G) {
  const int nprob = (int)(b1 - b0);
  G.nprob = nprob;
  std::vector<Prob> hp((size_t)nprob);
  std::vector<int64_t> loff((size_t)nprob + 1, 0);
  std::vector<Params> hprm((size_t)nprob);
  G.dprobs = fx.take<Prob>(sizeof(Prob) * nprob);
  G.dloff = fx.take<int64_t>(sizeof(int64_t) * (nprob + 1));
  // parameters first, then the info arrays back to back, so that one fill
  // clears every info array and nothing else
  for (int q = 0; q < nprob; q++) hp[q].prm = fx.take<Params>(sizeof(Params));
  size_t cap = 0;
  char *info0 = nullptr, *info1 = nullptr;
  for (int q = 0; q < nprob; q++) {
    const ProblemDesc &D = pd[b0 + q];
    const int n = D.n, m = D.iu - D.il + 1;
    loff[q + 1] = loff[q] + m;
    G.nmax = std::max(G.nmax, n);
    G.mmax = std::max(G.mmax, m);
    cap += (size_t)(m / 2);
    Prob &P = hp[q];
    Params *prm = P.prm;
    std::memset(&P, 0, sizeof(P));
    P.d = D.d; P.e = D.e; P.n = n; P.m = m; P.ldz = D.ldz; P.kbase = D.il; P.W = D.W; P.Z = D.Z;
    P.prm = prm;
    P.info = fx.take<int>(sizeof(int) * ((size_t)m + 1));
    if (!info0) info0 = reinterpret_cast<char *>(P.info);
    info1 = reinterpret_cast<char *>(P.info) + align_up(sizeof(int) * ((size_t)m + 1));
    carve_problem(sh, P, n, m);
    std::memset(&hprm[q], 0, sizeof(Params));
    hprm[q].rtol = opt.rtol;
  }
  G.mtotal = loff[nprob];
  G.info = reinterpret_cast<int *>(info0);
  G.info_ints = (size_t)(info1 - info0) / sizeof(int);
  G.scr.stride = chain_scratch_doubles(G.nmax, G.mmax, 1);
  G.scr.base = sh.take<double>(sizeof(double) * G.scr.stride * (size_t)std::max(nslots, 1));
  G.item_cap = (int)std::max<size_t>(cap, 1);
  G.items = sh.take<ChainItem>(sizeof(ChainItem) * (size_t)G.item_cap);
  int *ints = sh.take<int>(sizeof(int) * (2 * kPlanBins + 4));
  G.bins = ints;
  G.nitems = ints + 2 * kPlanBins;
  // the flags stay readable after later segments have reused the shared region
  G.flags = fx.take<int>(sizeof(int) * 2);
  if (fx.off > fx.cap || sh.off > sh.cap) return TE_ERR_WORKSPACE;
  TE_CHECK(hipMemcpy(G.dprobs, hp.data(), sizeof(Prob) * nprob, hipMemcpyHostToDevice));
  TE_CHECK(hipMemcpy(G.dloff, loff.data(), sizeof(int64_t) * (nprob + 1), hipMemcpyHostToDevice));
  for (int q = 0; q < nprob; q++)
    TE_CHECK(hipMemcpy(hp[q].prm, &hprm[q], sizeof(Params), hipMemcpyHostToDevice));
  return 0;
}

// Every step of one segment, device-only (capturable).
int enqueue_segment(const GraphSeg &G, const Resolved &opt, int nt, int nwg, hipStream_t s) {
  TE_CHECK(launch_fill_i32(G.info, G.info_ints, 0, s));
  TE_CHECK(launch_setup(G.dprobs, G.nprob, s));
  TE_CHECK(launch_bisect(G.dprobs, G.nprob, G.dloff, G.mtotal, s));
  TE_CHECK(launch_cluster(G.dprobs, G.nprob, s));
  TE_CHECK(launch_invit(G.dprobs, G.nprob, G.dloff, G.mtotal, opt.iters, opt.seed, s));
  TE_CHECK(launch_transpose(G.dprobs, G.nprob, G.nmax, G.mmax, s));
  TE_CHECK(launch_plan(G.dprobs, G.nprob, G.bins, G.items, G.nitems, s));
  TE_CHECK(launch_fill_i32(G.flags, 2, 0, s));
  if (opt.orth == TE_ORTH_MGS)
    TE_CHECK(launch_chain_mgs(G.dprobs, G.items, G.item_cap, G.nitems, G.flags + 1, G.flags,
                              G.scr, nwg, opt.iters, s));
  else
    TE_CHECK(launch_chain_small_dev(G.dprobs, G.items, G.item_cap, G.nitems, G.flags + 1,
                                    G.flags, G.scr, nwg, nt, opt.iters, s));
  TE_CHECK(launch_finalize(G.dprobs, G.nprob, G.dloff, G.mtotal, s));
  return 0;
}

// ---- autotune table: (ceil log2 max n, ceil log2 mean n) -> configuration ----
int ceil_log2(double x) {
  int e = 0;
  while ((double)(1LL << e) < x && e < 62) e++;
  return e;
}

std::pair<int, int> tune_key(const std::vector<ProblemDesc> &pd) {
  double nmax = 1, nsum = 0;
  for (const auto &D : pd) {
    nmax = std::max(nmax, (double)D.n);
    nsum += D.n;
  }
  return {ceil_log2(nmax), ceil_log2(nsum / (double)std::max<size_t>(pd.size(), 1))};
}

std::mutex g_tune_mu;
bool g_tune_loaded = false;
std::vector<std::pair<std::pair<int, int>, te_graph_cfg>> g_tune;

const char *tune_file() {
  const char *f = getenv("TE_TUNE_FILE");
  return (f && f[0]) ? f : nullptr;
}

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char *f = tune_file();
  if (!f) return;
  FILE *fp = fopen(f, "r");
  if (!fp) return;
  char line[256];
  while (fgets(line, sizeof line, fp)) {
    int nb, mb, nt, per;
    if (line[0] == '#') continue;
    if (sscanf(line, "%d %d %d %d", &nb, &mb, &nt, &per) == 4 &&
        (nt == 256 || nt == 512) && per >= 1) {
      te_graph_cfg c{nt, per};
      bool found = false;
      for (auto &e : g_tune)
        if (e.first == std::make_pair(nb, mb)) { e.second = c; found = true; }
      if (!found) g_tune.push_back({{nb, mb}, c});
    }
  }
  fclose(fp);
}

bool tune_lookup(std::pair<int, int> key, te_graph_cfg &out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  for (const auto &e : g_tune)
    if (e.first == key) { out = e.second; return true; }
  return false;
}

void tune_store(std::pair<int, int> key, const te_graph_cfg &c, double ms) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  bool found = false;
  for (auto &e : g_tune)
    if (e.first == key) { e.second = c; found = true; }
  if (!found) g_tune.push_back({key, c});
  const char *f = tune_file();
  if (!f) return;
  if (FILE *fp = fopen(f, "a")) {
    fprintf(fp, "%d %d %d %d  # %.3f ms on the tuning sample\n", key.first, key.second,
            c.chain_threads, c.chains_per_cu, ms);
    fclose(fp);
  }
}

// Resident chain workgroups per CU for nt threads (0 if the variant does not fit).
int per_cu_max(int device, int nt) {
  const int ncu = device_cus(device);
  if (ncu <= 0) return 0;
  return small_max_wgs(device, nt) / ncu;
}

// Resident MGS chain workgroups (kMgsThreads threads) per CU.
int mgs_per_cu_max(int device) {
  const int ncu = device_cus(device);
  return ncu > 0 ? mgs_max_wgs(device) / ncu : 0;
}

// The MGS chains run in workgroups of kMgsThreads threads.
bool cfg_valid(int device, const te_graph_cfg &c, bool mgs) {
  if (mgs)
    return c.chain_threads == kMgsThreads && c.chains_per_cu >= 1 &&
           c.chains_per_cu <= mgs_per_cu_max(device);
  if (c.chain_threads != 256 && c.chain_threads != 512) return false;
  return c.chains_per_cu >= 1 && c.chains_per_cu <= per_cu_max(device, c.chain_threads);
}

}  // namespace

}  // namespace te

struct te_batch_graph {
  int device = -1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void *mem = nullptr;
  size_t bytes = 0;
  int nseg = 0;
  std::vector<int *> abort_flags;  // one per segment, cleared by the graph itself
  te_graph_cfg cfg{};
  ~te_batch_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (mem) {
      (void)hipDeviceSynchronize();
      (void)hipFree(mem);
    }
    (void)hipGetLastError();
  }
};

namespace te {
namespace {

// Builds and instantiates the graph of the whole batch with configuration c.
int build_graph(const std::vector<ProblemDesc> &pd, const Resolved &opt, const te_graph_cfg &c,
                te_batch_graph &g) {
  const DeviceLimits lim = limits();
  if (lim.device < 0) return TE_ERR_NO_DEVICE;
  g.device = lim.device;
  g.cfg = c;
  const int nwg = device_cus(lim.device) * c.chains_per_cu;
  const uint64_t budget = opt.ws_budget ? opt.ws_budget : default_budget();
  std::vector<std::pair<size_t, size_t>> seg;
  if (!plan_segments(pd, nwg, budget, seg)) return TE_ERR_WORKSPACE;
  size_t fixed = 0, shared = 0;
  for (auto &q : seg) {
    fixed += seg_fixed_bytes(pd, q.first, q.second);
    shared = std::max(shared, seg_shared_bytes(pd, q.first, q.second, nwg));
  }
  g.bytes = fixed + shared;
  if (hipMalloc(&g.mem, g.bytes) != hipSuccess) {
    (void)hipGetLastError();
    g.mem = nullptr;
    return TE_ERR_WORKSPACE;
  }
  char *base = static_cast<char *>(g.mem);
  Carve fx{base, 0, fixed};
  std::vector<GraphSeg> G(seg.size());
  for (size_t k = 0; k < seg.size(); k++) {
    Carve sh{base + fixed, 0, shared};
    const int rc = carve_segment(pd, seg[k].first, seg[k].second, opt, nwg, fx, sh, G[k]);
    if (rc) return rc;
  }
  g.nseg = (int)seg.size();
  for (const auto &q : G) g.abort_flags.push_back(q.flags);
  hipStream_t cs = nullptr;
  TE_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  int rc = 0;
  if (e == hipSuccess) {
    for (size_t k = 0; k < G.size() && rc == 0; k++)
      rc = enqueue_segment(G[k], opt, c.chain_threads, nwg, cs);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (rc == 0 && e2 != hipSuccess) rc = hip_fail(e2);
    g.graph = graph;
    if (rc == 0) {
      const hipError_t e3 = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
      if (e3 != hipSuccess) rc = hip_fail(e3);
    }
  } else {
    rc = hip_fail(e);
  }
  (void)hipStreamDestroy(cs);
  return rc;
}

te_graph_cfg default_cfg(int device, bool mgs) {
  if (mgs) return te_graph_cfg{kMgsThreads, std::max(mgs_per_cu_max(device), 1)};
  te_graph_cfg c{256, std::max(per_cu_max(device, 256), 1)};
  return c;
}

}  // namespace
}  // namespace te

using namespace te;

extern "C" {

int te_last_hip_error(void) { return g_last_hip; }

void te_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_tmu);
  g_timing = on != 0;
}

void te_timing_reset(void) {
  std::lock_guard<std::mutex> lk(g_tmu);
  for (int p = 0; p < PH_COUNT; p++) { g_ms[p] = 0.0; g_cnt[p] = 0; }
}

int te_timing_read(double *ms, long long *launches, int cap) {
  std::lock_guard<std::mutex> lk(g_tmu);
  for (int p = 0; p < PH_COUNT && p < cap; p++) {
    if (ms) ms[p] = g_ms[p];
    if (launches) launches[p] = g_cnt[p];
  }
  return PH_COUNT;
}

int tridiag_eigvecs(const double *d, const double *e, int n, int il, int iu, double *W, double *Z,
                    int ldz, hipStream_t stream) {
  if (!d) return -1;
  if (!e && n > 1) return -2;
  if (n < 1) return -3;
  if (il < 1 || il > n) return -4;
  if (iu < il || iu > n) return -5;
  if (!W) return -6;
  if (!Z) return -7;
  if (ldz < n) return -8;
  std::vector<ProblemDesc> pd{{d, e, n, il, iu, W, Z, ldz}};
  return solve_problems(pd, nullptr, resolve(nullptr), nullptr, 0, nullptr, stream);
}

int tridiag_eigvecs_given_w(const double *d, const double *e, int n, int m, const double *W,
                            double *Z, int ldz, hipStream_t stream) {
  if (!d) return -1;
  if (!e && n > 1) return -2;
  if (n < 1) return -3;
  if (m < 1 || m > n) return -4;
  if (!W) return -5;
  if (!Z) return -6;
  if (ldz < n) return -7;
  // W is both the input and (copied onto itself) the output eigenvalue array.
  std::vector<ProblemDesc> pd{{d, e, n, 1, m, const_cast<double *>(W), Z, ldz}};
  double *Wtmp = nullptr;
  hipError_t he = hipMallocAsync((void **)&Wtmp, sizeof(double) * m, stream);
  if (he != hipSuccess) return hip_fail(he);
  he = hipMemcpyAsync(Wtmp, W, sizeof(double) * m, hipMemcpyDeviceToDevice, stream);
  if (he != hipSuccess) return hip_fail(he);
  const int rc = solve_problems(pd, Wtmp, resolve(nullptr), nullptr, 0, nullptr, stream);
  he = hipFreeAsync(Wtmp, stream);
  if (rc == 0 && he != hipSuccess) return hip_fail(he);
  return rc;
}

size_t tridiag_eigvecs_workspace_bytes(int n, int il, int iu) {
  if (n < 1 || il < 1 || iu < il || iu > n) return 0;
  const int m = iu - il + 1;
  DeviceLimits lim = limits();
  const int coop = lim.coop > 0 ? lim.coop : 4096;
  const int small = lim.small > 0 ? lim.small : 4096;
  return fixed_bytes(1) + prob_layout(n, m).total() +
         chain_bytes(n, m, std::max(coop, small), coop, m);
}

int tridiag_eigvecs_ex(const double *d, const double *e, int n, int il, int iu,
                       const double *W_given, double *W, double *Z, int ldz, const te_opts *opt,
                       void *ws, size_t ws_bytes, int *info, hipStream_t stream) {
  if (!d) return -1;
  if (!e && n > 1) return -2;
  if (n < 1) return -3;
  if (il < 1 || il > n) return -4;
  if (iu < il || iu > n) return -5;
  if (!W) return -7;
  if (!Z) return -8;
  if (ldz < n) return -9;
  if (opt && (opt->iters < 0 || opt->cluster_rtol < 0.0 || opt->coop_wgs < 0 ||
              (opt->orth != TE_ORTH_CWY && opt->orth != TE_ORTH_MGS) ||
              (opt->stop != TE_STOP_FIXED && opt->stop != TE_STOP_GROWTH))) return -10;
  if (!ws) return -11;
  if (ws_bytes < tridiag_eigvecs_workspace_bytes(n, il, iu)) return -12;
  if (((uintptr_t)ws) % kAlign) return -11;
  std::vector<ProblemDesc> pd{{d, e, n, il, iu, W, Z, ldz}};
  return solve_problems(pd, W_given, resolve(opt), ws, ws_bytes, info, stream);
}

// ---- Entry point that allocates nothing ----
// Its workspace is this file-scope device array (one copy per device, kept
// for the life of the process).  Host code never passes the array's name to a
// kernel or a copy: its device address is taken once per device with
// hipGetSymbolAddress and every use goes through that pointer.
static __device__ __align__(256) unsigned char scratch[TE_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (null on failure).
void *scratch_ptr(int dev, int *rc) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *rc = te::hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol);
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

size_t tridiag_eigvecs_noalloc_bytes(int n, int il, int iu) {
  if (n < 1 || il < 1 || iu < il || iu > n) return 0;
  const int m = iu - il + 1;
  te::DeviceLimits lim = te::limits();
  const int coop = lim.coop > 0 ? lim.coop : 4096;
  const int small = lim.small > 0 ? lim.small : 4096;
  // a chain has two or more members, so at most m / 2 chains need a slot
  const int slots = std::min(std::max(coop, small), std::max(m / 2, 1));
  return te::fixed_bytes(1) + te::prob_layout(n, m).total() +
         te::chain_bytes(n, m, slots, coop, m);
}

int tridiag_eigvecs_noalloc(const double *d, const double *e, int n, int il, int iu,
                            const double *W_given, double *W, double *Z, int ldz,
                            const te_opts *opt, int *info, hipStream_t stream) {
  if (!d) return -1;
  if (!e && n > 1) return -2;
  if (n < 1) return -3;
  if (il < 1 || il > n) return -4;
  if (iu < il || iu > n) return -5;
  if (!W) return -7;
  if (!Z) return -8;
  if (ldz < n) return -9;
  if (opt && (opt->iters < 0 || opt->cluster_rtol < 0.0 || opt->coop_wgs < 0 ||
              (opt->orth != TE_ORTH_CWY && opt->orth != TE_ORTH_MGS) ||
              (opt->stop != TE_STOP_FIXED && opt->stop != TE_STOP_GROWTH))) return -10;
  const size_t need = tridiag_eigvecs_noalloc_bytes(n, il, iu);
  if (need > TE_NOALLOC_SCRATCH_BYTES) return TE_ERR_WORKSPACE;
  int dev = -1;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return te::hip_fail(he);
  if (dev < 0 || dev >= kMaxDevices) return TE_ERR_NO_DEVICE;
  int rc = 0;
  void *ws = scratch_ptr(dev, &rc);
  if (!ws) return rc;
  std::vector<te::ProblemDesc> pd{{d, e, n, il, iu, W, Z, ldz}};
  return te::solve_problems(pd, W_given, te::resolve(opt), ws, TE_NOALLOC_SCRATCH_BYTES, info,
                            stream);
}

// ---- Splitting into unreduced blocks ----
// Every block is an independent problem of the multi-problem path: first the
// eigenvalues of every block (one bisection launch over all blocks), then,
// on the host, the order of all eigenvalues (value, then block, then index
// in the block) and the blocks' shares of il..iu, then the blocks' eigenpairs
// from those eigenvalues (start-vector key s + 1 + l for eigenvalue l of the
// block at row s), and last one scatter launch into the caller's columns.
int tridiag_eigvecs_split(const double *d, const double *e, int n, int il, int iu, double *W,
                          double *Z, int ldz, const te_opts *opt, int *info, int *nblocks,
                          hipStream_t stream) {
  if (!d) return -1;
  if (!e && n > 1) return -2;
  if (n < 1) return -3;
  if (il < 1 || il > n) return -4;
  if (iu < il || iu > n) return -5;
  if (!W) return -6;
  if (!Z) return -7;
  if (ldz < n) return -8;
  if (opt && (opt->iters < 0 || opt->cluster_rtol < 0.0 || opt->coop_wgs < 0 ||
              (opt->orth != TE_ORTH_CWY && opt->orth != TE_ORTH_MGS) ||
              (opt->stop != TE_STOP_FIXED && opt->stop != TE_STOP_GROWTH))) return -9;
  if (limits().device < 0) return TE_ERR_NO_DEVICE;
  const int m = iu - il + 1;
  OwnedBlocks owned(stream);
  auto dalloc = [&](size_t bytes, void **p) -> int {
    TE_CHECK(hipMallocAsync(p, std::max<size_t>(bytes, 256), stream));
    owned.blocks.push_back(*p);
    return 0;
  };

  // blocks
  std::vector<int> bs{0};
  {
    SharedHold hold;
    std::vector<unsigned char> hf((size_t)std::max(n - 1, 1), 0);
    if (n > 1) {
      unsigned char *df = nullptr;
      if (int rc = dalloc((size_t)n, (void **)&df)) return rc;
      TE_CHECK(launch_split_flags(d, e, n, df, stream));
      TE_CHECK(hipMemcpyAsync(hf.data(), df, (size_t)(n - 1), hipMemcpyDeviceToHost, stream));
      TE_CHECK(hipStreamSynchronize(stream));
    }
    for (int i = 0; i < n - 1; i++)
      if (hf[i]) bs.push_back(i + 1);
    bs.push_back(n);
  }
  const int nb = (int)bs.size() - 1;
  if (nblocks) *nblocks = nb;

  // eigenvalues of every block
  std::vector<double> hw((size_t)n);
  double *Wall = nullptr;
  {
    SharedHold hold;
    size_t bytes = fixed_bytes(nb) + align_up(sizeof(double) * n);
    for (int b = 0; b < nb; b++)
      bytes += align_up(sizeof(double) * std::max(bs[b + 1] - bs[b] - 1, 1)) +
               align_up(sizeof(Params));
    char *base = nullptr;
    if (int rc = dalloc(bytes, (void **)&base)) return rc;
    Carve cv{base, 0, bytes};
    Prob *dp = cv.take<Prob>(sizeof(Prob) * nb);
    int64_t *dloff = cv.take<int64_t>(sizeof(int64_t) * (nb + 1));
    Wall = cv.take<double>(sizeof(double) * n);
    std::vector<Prob> hp((size_t)nb);
    std::vector<Params> hprm((size_t)nb);
    std::vector<int64_t> loff((size_t)nb + 1);
    for (int b = 0; b < nb; b++) {
      const int s0 = bs[b], nbk = bs[b + 1] - bs[b];
      Prob &P = hp[b];
      std::memset(&P, 0, sizeof(P));
      P.d = d + s0;
      P.e = e ? e + s0 : nullptr;
      P.n = nbk; P.m = nbk; P.kbase = 1; P.W = Wall + s0; P.ldz = nbk;
      P.e2 = cv.take<double>(sizeof(double) * std::max(nbk - 1, 1));
      P.prm = cv.take<Params>(sizeof(Params));
      std::memset(&hprm[b], 0, sizeof(Params));
      hprm[b].rtol = 1e-3;
      loff[b] = s0;
    }
    loff[nb] = n;
    TE_CHECK(hipMemcpyAsync(dp, hp.data(), sizeof(Prob) * nb, hipMemcpyHostToDevice, stream));
    TE_CHECK(hipMemcpyAsync(dloff, loff.data(), sizeof(int64_t) * (nb + 1),
                            hipMemcpyHostToDevice, stream));
    for (int b = 0; b < nb; b++)
      TE_CHECK(hipMemcpyAsync(hp[b].prm, &hprm[b], sizeof(Params), hipMemcpyHostToDevice,
                              stream));
    TE_CHECK(launch_setup(dp, nb, stream));
    TE_CHECK(launch_bisect(dp, nb, dloff, n, stream));
    TE_CHECK(hipMemcpyAsync(hw.data(), Wall, sizeof(double) * n, hipMemcpyDeviceToHost, stream));
    TE_CHECK(hipStreamSynchronize(stream));
  }

  // order of all eigenvalues; each block's share of il..iu is a contiguous range
  std::vector<int> blk_of((size_t)n), ord((size_t)n), pos((size_t)n);
  for (int b = 0; b < nb; b++)
    for (int i = bs[b]; i < bs[b + 1]; i++) blk_of[i] = b;
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int a, int b) {
    if (hw[a] != hw[b]) return hw[a] < hw[b];
    if (blk_of[a] != blk_of[b]) return blk_of[a] < blk_of[b];
    return a < b;
  });
  for (int k = 0; k < n; k++) pos[ord[k]] = k - (il - 1);
  struct Sel { int b, lo, hi; };
  std::vector<Sel> sel;
  size_t zsum = 0;
  for (int b = 0; b < nb; b++) {
    int lo = -1, hi = -2;
    for (int i = bs[b]; i < bs[b + 1]; i++)
      if (pos[i] >= 0 && pos[i] < m) { if (lo < 0) lo = i - bs[b]; hi = i - bs[b]; }
    if (lo >= 0) {
      sel.push_back({b, lo, hi});
      zsum += (size_t)(bs[b + 1] - bs[b]) * (size_t)(hi - lo + 1);
    }
  }

  // the selected blocks' eigenpairs from their eigenvalues
  double *Wsel = nullptr, *Wt = nullptr, *Zt = nullptr;
  int *It = nullptr;
  SplitCol *dcols = nullptr;
  if (int rc = dalloc(sizeof(double) * m, (void **)&Wsel)) return rc;
  if (int rc = dalloc(sizeof(double) * m, (void **)&Wt)) return rc;
  if (int rc = dalloc(sizeof(double) * zsum, (void **)&Zt)) return rc;
  if (int rc = dalloc(sizeof(int) * ((size_t)m + sel.size()), (void **)&It)) return rc;
  if (int rc = dalloc(sizeof(SplitCol) * m, (void **)&dcols)) return rc;
  std::vector<ProblemDesc> pd;
  std::vector<SplitCol> hc((size_t)m);
  size_t woff = 0, zoff = 0, ioff = 0;
  for (const Sel &q : sel) {
    const int s0 = bs[q.b], nbk = bs[q.b + 1] - bs[q.b], mb = q.hi - q.lo + 1;
    TE_CHECK(hipMemcpyAsync(Wsel + woff, Wall + s0 + q.lo, sizeof(double) * mb,
                            hipMemcpyDeviceToDevice, stream));
    ProblemDesc D{d + s0, e ? e + s0 : nullptr, nbk, s0 + 1 + q.lo, s0 + 1 + q.hi, Wt + woff,
                  Zt + zoff, nbk, It + ioff};
    pd.push_back(D);
    for (int j = 0; j < mb; j++) {
      SplitCol &c = hc[(size_t)pos[s0 + q.lo + j]];
      c.src = Zt + zoff + (size_t)j * nbk;
      c.w = Wt + woff + j;
      c.st = It + ioff + 1 + j;
      c.s = s0;
      c.nb = nbk;
      c.p = pos[s0 + q.lo + j];
      c.pad = 0;
    }
    woff += (size_t)mb;
    zoff += (size_t)nbk * mb;
    ioff += (size_t)mb + 1;
  }
  const int rc = solve_problems(pd, Wsel, resolve(opt), nullptr, 0, nullptr, stream);
  if (rc) return rc;

  // into the caller's columns
  {
    SharedHold hold;
    TE_CHECK(hipMemcpyAsync(dcols, hc.data(), sizeof(SplitCol) * m, hipMemcpyHostToDevice, stream));
    if (info) TE_CHECK(launch_fill_i32(info, 1, 0, stream));
    TE_CHECK(launch_split_scatter(dcols, m, n, W, Z, (size_t)ldz, info, stream));
    TE_CHECK(hipStreamSynchronize(stream));
  }
  owned.released = true;
  for (void *p : owned.blocks) TE_CHECK(hipFreeAsync(p, stream));
  TE_CHECK(hipStreamSynchronize(stream));
  return 0;
}

int bidiag_svd(const double *a, const double *b, int n, int il, int iu, double *S, double *U,
               int ldu, double *V, int ldv, const te_opts *opt, int *info, hipStream_t stream) {
  if (!a) return -1;
  if (!b && n > 1) return -2;
  if (n < 1 || n > (1 << 30)) return -3;
  if (il < 1 || il > n) return -4;
  if (iu < il || iu > n) return -5;
  if (!S) return -6;
  if (!U) return -7;
  if (ldu < n) return -8;
  if (!V) return -9;
  if (ldv < n) return -10;
  if (opt && (opt->iters < 0 || opt->cluster_rtol < 0.0 || opt->coop_wgs < 0 ||
              (opt->orth != TE_ORTH_CWY && opt->orth != TE_ORTH_MGS) ||
              (opt->stop != TE_STOP_FIXED && opt->stop != TE_STOP_GROWTH))) return -11;
  if (limits().device < 0) return TE_ERR_NO_DEVICE;
  const int N = 2 * n, m = iu - il + 1;
  OwnedBlocks owned(stream);
  double *dg = nullptr, *eg = nullptr, *Zg = nullptr;
  for (auto pr : {std::make_pair((void **)&dg, sizeof(double) * N),
                  std::make_pair((void **)&eg, sizeof(double) * N),
                  std::make_pair((void **)&Zg, sizeof(double) * (size_t)N * m)}) {
    TE_CHECK(hipMallocAsync(pr.first, pr.second, stream));
    owned.blocks.push_back(*pr.first);
  }
  {
    SharedHold hold;
    TE_CHECK(launch_gk_build(a, b, n, dg, eg, stream));
  }
  // +sigma_il .. +sigma_iu are the tridiagonal's eigenvalues n + il .. n + iu
  std::vector<ProblemDesc> pd{{dg, eg, N, n + il, n + iu, S, Zg, N, info}};
  const int rc = solve_problems(pd, nullptr, resolve(opt), nullptr, 0, nullptr, stream);
  if (rc) return rc;
  {
    SharedHold hold;
    TE_CHECK(launch_gk_split(Zg, n, m, U, (size_t)ldu, V, (size_t)ldv, stream));
    TE_CHECK(hipStreamSynchronize(stream));
  }
  owned.released = true;
  for (void *p : owned.blocks) TE_CHECK(hipFreeAsync(p, stream));
  TE_CHECK(hipStreamSynchronize(stream));
  return 0;
}

int tridiag_eigvals(const double *d, const double *e, int n, int il, int iu, double *W,
                    hipStream_t stream) {
  if (!d) return -1;
  if (!e && n > 1) return -2;
  if (n < 1) return -3;
  if (il < 1 || il > n) return -4;
  if (iu < il || iu > n) return -5;
  if (!W) return -6;
  if (limits().device < 0) return TE_ERR_NO_DEVICE;
  SharedHold hold;
  const int m = iu - il + 1;
  const size_t bytes = fixed_bytes(1) + align_up(sizeof(double) * std::max(n - 1, 1)) +
                       align_up(sizeof(Params));
  char *base = nullptr;
  TE_CHECK(hipMallocAsync((void **)&base, bytes, stream));
  Carve cv{base, 0, bytes};
  Prob *dp = cv.take<Prob>(sizeof(Prob));
  int64_t *dloff = cv.take<int64_t>(sizeof(int64_t) * 2);
  Prob P;
  std::memset(&P, 0, sizeof(P));
  P.d = d; P.e = e; P.n = n; P.m = m; P.kbase = il; P.W = W; P.ldz = n;
  P.e2 = cv.take<double>(sizeof(double) * std::max(n - 1, 1));
  P.prm = cv.take<Params>(sizeof(Params));
  Params hp;
  std::memset(&hp, 0, sizeof(hp));
  hp.rtol = 1e-3;
  const int64_t loff[2] = {0, m};
  TE_CHECK(hipMemcpyAsync(dp, &P, sizeof(P), hipMemcpyHostToDevice, stream));
  TE_CHECK(hipMemcpyAsync(dloff, loff, sizeof(loff), hipMemcpyHostToDevice, stream));
  TE_CHECK(hipMemcpyAsync(P.prm, &hp, sizeof(hp), hipMemcpyHostToDevice, stream));
  TE_CHECK(launch_setup(dp, 1, stream));
  TE_CHECK(launch_bisect(dp, 1, dloff, m, stream));
  TE_CHECK(hipFreeAsync(base, stream));
  TE_CHECK(hipStreamSynchronize(stream));
  return 0;
}

int tridiag_clusters(const double *W, int m, double tol, int *start, int *size, int *ncl,
                     hipStream_t stream) {
  if (!W) return -1;
  if (m < 1) return -2;
  if (!(tol >= 0.0)) return -3;
  if (!start) return -4;
  if (!size) return -5;
  if (!ncl) return -6;
  if (limits().device < 0) return TE_ERR_NO_DEVICE;
  SharedHold hold;
  const size_t bytes = fixed_bytes(1) + align_up(sizeof(Params)) + align_up(sizeof(int) * m);
  char *base = nullptr;
  TE_CHECK(hipMallocAsync((void **)&base, bytes, stream));
  Carve cv{base, 0, bytes};
  Prob *dp = cv.take<Prob>(sizeof(Prob));
  Prob P;
  std::memset(&P, 0, sizeof(P));
  P.m = m; P.W = const_cast<double *>(W); P.cl_start = start; P.cl_size = size; P.ncl = ncl;
  P.prm = cv.take<Params>(sizeof(Params));
  P.pos = cv.take<int>(sizeof(int) * m);
  Params hp;
  std::memset(&hp, 0, sizeof(hp));
  hp.tol = tol;
  TE_CHECK(hipMemcpyAsync(dp, &P, sizeof(P), hipMemcpyHostToDevice, stream));
  TE_CHECK(hipMemcpyAsync(P.prm, &hp, sizeof(hp), hipMemcpyHostToDevice, stream));
  TE_CHECK(launch_cluster(dp, 1, stream));
  TE_CHECK(hipFreeAsync(base, stream));
  TE_CHECK(hipStreamSynchronize(stream));
  return 0;
}

int tridiag_eigvecs_batched(const double *d_all, const double *e_all, const int64_t *off,
                            const int *il, const int *iu, double *W_all, const int64_t *woff,
                            double *Z_all, const int64_t *zoff, int B, const te_opts *opt,
                            hipStream_t stream) {
  std::vector<ProblemDesc> pd;
  const int rc = te::batch_descs(d_all, e_all, off, il, iu, W_all, woff, Z_all, zoff, B, opt, pd);
  if (rc) return rc;
  return solve_batched(pd, resolve(opt), stream);
}

int tridiag_eigvecs_batched_ex(const double *d_all, const double *e_all, const int64_t *off,
                               const int *il, const int *iu, double *W_all, const int64_t *woff,
                               double *Z_all, const int64_t *zoff, int B, const te_opts *opt,
                               int *info_all, const int64_t *ioff, hipStream_t stream) {
  std::vector<ProblemDesc> pd;
  const int rc = te::batch_descs(d_all, e_all, off, il, iu, W_all, woff, Z_all, zoff, B, opt, pd);
  if (rc) return rc;
  if (!info_all) return -12;
  if (!ioff) return -13;
  // the problems' status regions [ioff[b], ioff[b] + 1 + m_b) must not overlap
  std::vector<std::pair<int64_t, int64_t>> span((size_t)B);
  for (int b = 0; b < B; b++) {
    if (ioff[b] < 0) return -13;
    span[b] = {ioff[b], ioff[b] + 1 + (iu[b] - il[b] + 1)};
  }
  std::sort(span.begin(), span.end());
  for (int b = 1; b < B; b++)
    if (span[b].first < span[b - 1].second) return -13;
  for (int b = 0; b < B; b++) pd[b].info = info_all + ioff[b];
  return solve_batched(pd, resolve(opt), stream);
}

te_batch_graph *te_batch_graph_create(const double *d_all, const double *e_all, const int64_t *off,
                                      const int *il, const int *iu, double *W_all,
                                      const int64_t *woff, double *Z_all, const int64_t *zoff,
                                      int B, const te_opts *opt, const te_graph_cfg *cfg,
                                      int *rc) {
  int r = 0;
  te_batch_graph *g = nullptr;
  try {
    std::vector<te::ProblemDesc> pd;
    r = te::batch_descs(d_all, e_all, off, il, iu, W_all, woff, Z_all, zoff, B, opt, pd);
    const bool mgs = opt && opt->orth == TE_ORTH_MGS;
    if (r == 0 && mgs)
      for (const auto &D : pd)
        if (D.n > TE_MGS_MAX_N) r = TE_ERR_UNSUPPORTED;
    if (r == 0) {
      const te::DeviceLimits lim = te::limits();
      if (lim.device < 0 || lim.small <= 0 || (mgs && lim.mgs <= 0)) {
        r = TE_ERR_NO_DEVICE;
      } else {
        te_graph_cfg c = te::default_cfg(lim.device, mgs);
        te_graph_cfg t;
        if (cfg) {
          if (!te::cfg_valid(lim.device, *cfg, mgs)) r = -12;
          else c = *cfg;
        } else if (!mgs && te::tune_lookup(te::tune_key(pd), t) &&
                   te::cfg_valid(lim.device, t, false)) {
          c = t;
        }
        if (r == 0) {
          g = new te_batch_graph();
          r = te::build_graph(pd, te::resolve(opt), c, *g);
          if (r) {
            delete g;
            g = nullptr;
          }
        }
      }
    }
  } catch (const std::bad_alloc &) {
    delete g;
    g = nullptr;
    r = TE_ERR_WORKSPACE;
  }
  if (rc) *rc = r;
  return g;
}

int te_batch_graph_launch(te_batch_graph *g, hipStream_t stream) {
  if (!g || !g->exec) return -1;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != g->device) return TE_ERR_NO_DEVICE;
  te::SharedHold hold;
  hipError_t e = hipGraphLaunch(g->exec, stream);
  if (e != hipSuccess) return te::hip_fail(e);
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return te::hip_fail(e);
  for (int *f : g->abort_flags) {  // a chain wait that timed out fails the call
    int a = 0;
    e = hipMemcpy(&a, f, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return te::hip_fail(e);
    if (a) return TE_ERR_KERNEL;
  }
  return 0;
}

int te_batch_graph_info(const te_batch_graph *g, te_graph_cfg *cfg, int *segments,
                        uint64_t *device_bytes) {
  if (!g) return -1;
  if (cfg) *cfg = g->cfg;
  if (segments) *segments = g->nseg;
  if (device_bytes) *device_bytes = g->bytes;
  return 0;
}

void te_batch_graph_destroy(te_batch_graph *g) { delete g; }

int te_batch_autotune(const double *d_all, const double *e_all, const int64_t *off, const int *il,
                      const int *iu, double *W_all, const int64_t *woff, double *Z_all,
                      const int64_t *zoff, int B, const te_opts *opt, te_graph_cfg *best,
                      te_graph_cfg *tried, double *ms, int cap, int *ntried) {
  std::vector<te::ProblemDesc> pd;
  int r = te::batch_descs(d_all, e_all, off, il, iu, W_all, woff, Z_all, zoff, B, opt, pd);
  if (r) return r;
  if (opt && opt->orth != TE_ORTH_CWY) return TE_ERR_UNSUPPORTED;
  const te::DeviceLimits lim = te::limits();
  if (lim.device < 0 || lim.small <= 0) return TE_ERR_NO_DEVICE;
  // Sample: every stride-th problem, at most about 2048 problems (enough for
  // segments as full as the batch's own: with a thinner sample the tuner
  // favoured one chain per CU, which loses on full segments).
  const size_t stride = std::max<size_t>(1, pd.size() / 2048);
  std::vector<te::ProblemDesc> sample;
  for (size_t b = 0; b < pd.size(); b += stride) sample.push_back(pd[b]);
  std::vector<te_graph_cfg> cand;
  for (int nt : {256, 512}) {
    const int pmax = te::per_cu_max(lim.device, nt);
    for (int per = 1; per <= pmax; per *= 2) cand.push_back(te_graph_cfg{nt, per});
    if (pmax >= 1 && (pmax & (pmax - 1)) != 0) cand.push_back(te_graph_cfg{nt, pmax});
  }
  if (cand.empty()) return TE_ERR_NO_DEVICE;
  const te::Resolved o = te::resolve(opt);
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return TE_ERR_HIP;
  hipEvent_t a = nullptr, z = nullptr;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&z);
  double best_ms = 1e300;
  te_graph_cfg bc = cand[0];
  int k = 0;
  for (const auto &c : cand) {
    te_batch_graph g;
    r = te::build_graph(sample, o, c, g);
    if (r) break;
    double t = 1e300;
    for (int rep = 0; rep < 2 && r == 0; rep++) {  // the first launch warms up
      te::SharedHold hold;
      (void)hipEventRecord(a, s);
      hipError_t e = hipGraphLaunch(g.exec, s);
      (void)hipEventRecord(z, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) { r = te::hip_fail(e); break; }
      float f = 0.f;
      if (rep > 0 && hipEventElapsedTime(&f, a, z) == hipSuccess) t = f;
    }
    if (r) break;
    if (k < cap) {
      if (tried) tried[k] = c;
      if (ms) ms[k] = t;
    }
    k++;
    if (t < best_ms) { best_ms = t; bc = c; }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(z);
  (void)hipStreamDestroy(s);
  if (ntried) *ntried = k;
  if (r) return r;
  te::tune_store(te::tune_key(pd), bc, best_ms);
  if (best) *best = bc;
  return 0;
}

}  // extern "C"
