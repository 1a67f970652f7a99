// Serving engine: eigenvector requests of different sizes are admitted under a
// device-memory budget into rounds, and rounds run concurrently on several
// streams ("lanes").  A round is one pass of the whole method over all of its
// requests (every phase one launch over the round's problems; their cluster
// chains run side by side), so requests that queue up while the device is busy
// are batched together as soon as memory and a lane free up.
//
// Requests are split into two classes by the size of their per-eigenvalue
// state (n * m entries): light ones, which finish in milliseconds, and heavy
// ones, whose cluster chains can take seconds.  A round holds requests of one
// class, so a light request never waits for the chains of a heavy one that
// happened to be admitted with it; the oldest waiting request decides which
// class the next free lane takes, and admission within a class is FIFO.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "te_host.h"
#include "te_sched.h"

namespace te {
namespace {

using Clock = std::chrono::steady_clock;

// Requests with at least this many per-eigenvalue entries (n * m) are heavy.
constexpr int64_t kHeavyEntries = (int64_t)1 << 22;
constexpr int kDefaultLanes = 3;

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct Request {
  int64_t id = 0;
  std::vector<double> d, e;  // host copies of the inputs
  int n = 0, il = 0, iu = 0, m = 0;
  double *W = nullptr, *Z = nullptr;  // caller's outputs
  int ldz = 0;
  bool heavy = false;
  int rc = 0;
  bool done = false;
  double t_submit = 0, t_start = 0, t_done = 0;
};

// Device bytes of a request's inputs and outputs while it is in flight.
size_t io_bytes(const Request &r) {
  return al(sizeof(double) * r.n) + al(sizeof(double) * std::max(r.n - 1, 1)) +
         al(sizeof(double) * r.m) + al(sizeof(double) * (size_t)r.n * r.m);
}

}  // namespace

struct Server {
  int device = 0;
  uint64_t budget = 0;
  Resolved opt{};
  DeviceLimits lim{};
  Clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv;  // queue, memory and completion changes
  std::deque<Request *> light, heavy;
  std::unordered_map<int64_t, std::unique_ptr<Request>> all;
  int64_t next_id = 1;
  uint64_t used = 0;
  bool stop = false;

  std::vector<hipStream_t> streams;
  std::vector<std::thread> lanes;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

  // Device bytes a round of these requests needs in total.
  size_t round_bytes(const std::vector<Request *> &rs) const {
    std::vector<ProblemDesc> pd(rs.size());
    size_t io = 0;
    for (size_t k = 0; k < rs.size(); k++) {
      pd[k] = ProblemDesc{nullptr, nullptr, rs[k]->n, rs[k]->il, rs[k]->iu, nullptr, nullptr,
                          rs[k]->n};
      io += io_bytes(*rs[k]);
    }
    return io + problems_bytes(pd, 0, pd.size(), lim);
  }

  void finish(const std::vector<Request *> &rs, int rc) {
    const double t = now();
    for (Request *r : rs) {
      r->rc = rc;
      r->t_done = t;
      r->done = true;
    }
  }

  // Under mu: take the next round, or return false when the caller must wait.
  bool form_round(std::vector<Request *> &round, size_t &bytes) {
    auto need = [&](const std::vector<Request *> &rs) { return round_bytes(rs); };
    for (;;) {
      const int r = sched_next(light, heavy, budget, used, need, round, bytes);
      if (r == 0) return false;
      if (r == 2) {  // can never be admitted
        round[0]->t_start = now();
        finish(round, TE_ERR_WORKSPACE);
        cv.notify_all();
        continue;
      }
      used += bytes;
      const double t = now();
      for (Request *q : round) q->t_start = t;
      return true;
    }
  }

  int run_round(const std::vector<Request *> &rs, hipStream_t s) {
    std::vector<size_t> offs(rs.size());
    size_t tot = 0;
    for (size_t k = 0; k < rs.size(); k++) {
      offs[k] = tot;
      tot += io_bytes(*rs[k]);
    }
    char *base = nullptr;
    hipError_t he = hipMallocAsync((void **)&base, tot, s);
    if (he != hipSuccess) return hip_fail(he);
    std::vector<ProblemDesc> pd(rs.size());
    for (size_t k = 0; k < rs.size(); k++) {
      const Request &r = *rs[k];
      char *p = base + offs[k];
      double *dd = reinterpret_cast<double *>(p);
      p += al(sizeof(double) * r.n);
      double *de = reinterpret_cast<double *>(p);
      p += al(sizeof(double) * std::max(r.n - 1, 1));
      double *dW = reinterpret_cast<double *>(p);
      p += al(sizeof(double) * r.m);
      double *dZ = reinterpret_cast<double *>(p);
      he = hipMemcpyAsync(dd, r.d.data(), sizeof(double) * r.n, hipMemcpyHostToDevice, s);
      if (he == hipSuccess && r.n > 1)
        he = hipMemcpyAsync(de, r.e.data(), sizeof(double) * (r.n - 1), hipMemcpyHostToDevice, s);
      if (he != hipSuccess) {
        (void)hipFreeAsync(base, s);
        return hip_fail(he);
      }
      pd[k] = ProblemDesc{dd, de, r.n, r.il, r.iu, dW, dZ, r.n};
    }
    int rc = solve_problems(pd, nullptr, opt, nullptr, 0, nullptr, s);
    for (size_t k = 0; k < rs.size() && rc == 0; k++) {
      const Request &r = *rs[k];
      he = hipMemcpyAsync(r.W, pd[k].W, sizeof(double) * r.m, hipMemcpyDefault, s);
      if (he == hipSuccess)
        he = hipMemcpy2DAsync(r.Z, sizeof(double) * r.ldz, pd[k].Z, sizeof(double) * r.n,
                              sizeof(double) * r.n, r.m, hipMemcpyDefault, s);
      if (he != hipSuccess) rc = hip_fail(he);
    }
    he = hipFreeAsync(base, s);
    if (rc == 0 && he != hipSuccess) rc = hip_fail(he);
    he = hipStreamSynchronize(s);
    if (rc == 0 && he != hipSuccess) rc = hip_fail(he);
    return rc;
  }

  void lane_main(int k) {
    (void)hipSetDevice(device);
    std::vector<Request *> round;
    for (;;) {
      size_t bytes = 0;
      {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
          if (form_round(round, bytes)) break;
          if (stop && light.empty() && heavy.empty()) return;
          cv.wait(lk);
        }
      }
      const int rc = run_round(round, streams[k]);
      {
        std::lock_guard<std::mutex> lk(mu);
        used -= bytes;
        finish(round, rc);
        for (Request *r : round) {   // the host copies of the inputs are spent
          std::vector<double>().swap(r->d);
          std::vector<double>().swap(r->e);
        }
      }
      cv.notify_all();
    }
  }
};

}  // namespace te

using namespace te;

struct te_server {
  Server s;
};

namespace {
te_server *create_server(const DeviceLimits &lim, uint64_t hbm_budget, int lanes,
                         const te_opts *opt);
}  // namespace

extern "C" {

te_server *te_server_create(uint64_t hbm_budget, int lanes, const te_opts *opt) {
  if (lanes < 0 || lanes > 64) return nullptr;
  if (opt && (opt->iters < 0 || opt->cluster_rtol < 0.0 || opt->coop_wgs < 0 ||
              (opt->orth != TE_ORTH_CWY && opt->orth != TE_ORTH_MGS) ||
              (opt->stop != TE_STOP_FIXED && opt->stop != TE_STOP_GROWTH))) return nullptr;
  DeviceLimits lim = limits();
  if (lim.device < 0 || lim.coop <= 0 || lim.small <= 0) return nullptr;
  try {
    return create_server(lim, hbm_budget, lanes, opt);
  } catch (...) {  // thread or memory exhaustion: no server
    return nullptr;
  }
}

}  // extern "C"

namespace {

te_server *create_server(const DeviceLimits &lim, uint64_t hbm_budget, int lanes,
                         const te_opts *opt) {
  std::unique_ptr<te_server> h(new te_server);
  Server &S = h->s;
  S.device = lim.device;
  S.lim = lim;
  S.opt = resolve(opt);
  // Cooperative chains fill the device unless the caller caps them: the long
  // chains of the largest requests dominate a busy server's time, and a
  // quarter of the CUs left to the other lanes gained them less than it cost
  // those chains.
  if (S.opt.coop_wgs <= 0) S.opt.coop_wgs = lim.coop;
  S.budget = hbm_budget ? hbm_budget : default_budget();
  S.t0 = Clock::now();
  const int nl = lanes > 0 ? lanes : kDefaultLanes;
  for (int k = 0; k < nl; k++) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : S.streams) (void)hipStreamDestroy(x);
      return nullptr;
    }
    S.streams.push_back(st);
  }
  try {
    for (int k = 0; k < nl; k++) S.lanes.emplace_back([&S, k] { S.lane_main(k); });
  } catch (...) {  // stop the lanes that did start, then give up
    {
      std::lock_guard<std::mutex> lk(S.mu);
      S.stop = true;
    }
    S.cv.notify_all();
    for (auto &t : S.lanes) t.join();
    for (hipStream_t x : S.streams) (void)hipStreamDestroy(x);
    throw;
  }
  return h.release();
}

}  // namespace

extern "C" {

int te_server_submit(te_server *srv, const double *d, const double *e, int n, int il, int iu,
                     double *W, double *Z, int ldz, int64_t *id) {
  if (!srv) return -1;
  if (!d) return -2;
  if (!e && n > 1) return -3;
  if (n < 1) return -4;
  if (il < 1 || il > n) return -5;
  if (iu < il || iu > n) return -6;
  if (!W) return -7;
  if (!Z) return -8;
  if (ldz < n) return -9;
  if (!id) return -10;
  Server &S = srv->s;
  std::unique_ptr<Request> r(new Request);
  r->n = n;
  r->il = il;
  r->iu = iu;
  r->m = iu - il + 1;
  r->d.assign(d, d + n);
  if (n > 1) r->e.assign(e, e + (n - 1));
  r->W = W;
  r->Z = Z;
  r->ldz = ldz;
  r->heavy = (int64_t)n * r->m >= kHeavyEntries;
  {
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.stop) return TE_ERR_NO_DEVICE;
    r->id = S.next_id++;
    r->t_submit = S.now();
    *id = r->id;
    (r->heavy ? S.heavy : S.light).push_back(r.get());
    S.all.emplace(r->id, std::move(r));
  }
  S.cv.notify_all();
  return 0;
}

int te_server_poll(te_server *srv, int64_t id, int *rc) {
  if (!srv) return -1;
  Server &S = srv->s;
  std::lock_guard<std::mutex> lk(S.mu);
  auto it = S.all.find(id);
  if (it == S.all.end()) return -2;
  if (!it->second->done) return 0;
  if (rc) *rc = it->second->rc;
  return 1;
}

int te_server_wait(te_server *srv, int64_t id, int *rc) {
  if (!srv) return -1;
  Server &S = srv->s;
  std::unique_lock<std::mutex> lk(S.mu);
  auto it = S.all.find(id);
  if (it == S.all.end()) return -2;
  Request *r = it->second.get();
  S.cv.wait(lk, [&] { return r->done; });
  if (rc) *rc = r->rc;
  return 1;
}

int te_server_times(te_server *srv, int64_t id, double *t_submit, double *t_start,
                    double *t_done) {
  if (!srv) return -1;
  Server &S = srv->s;
  std::lock_guard<std::mutex> lk(S.mu);
  auto it = S.all.find(id);
  if (it == S.all.end()) return -2;
  const Request &r = *it->second;
  if (t_submit) *t_submit = r.t_submit;
  if (t_start) *t_start = r.t_start;
  if (t_done) *t_done = r.t_done;
  return r.done ? 1 : 0;
}

int te_server_release(te_server *srv, int64_t id) {
  if (!srv) return -1;
  Server &S = srv->s;
  std::lock_guard<std::mutex> lk(S.mu);
  auto it = S.all.find(id);
  if (it == S.all.end()) return -2;
  if (!it->second->done) return 0;
  S.all.erase(it);
  return 1;
}

void te_server_destroy(te_server *srv) {
  if (!srv) return;
  Server &S = srv->s;
  {
    std::lock_guard<std::mutex> lk(S.mu);
    S.stop = true;
  }
  S.cv.notify_all();
  for (auto &t : S.lanes) t.join();
  for (hipStream_t st : S.streams) (void)hipStreamDestroy(st);
  delete srv;
}

}  // extern "C"
