// Host-only simulation of the serving engine's admission policy (te_sched.h)
// with a virtual clock and a fake executor: a Poisson request trace of mixed
// sizes goes through `lanes` lanes under an HBM budget; every invariant of
// the policy is checked as the simulation runs, and the latency percentiles
// are printed as JSON.  Built and run by tests/test_sched_cpu.py.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <vector>

#include "te_sched.h"

struct Req {
  int64_t id;
  int n, m;
  bool heavy;
  double arrival, start = -1, done = -1;
  bool rejected = false;
  int order = -1;   // admission order within its class
};

static size_t need1(const Req *r) {   // a device-memory model of one request
  return (size_t)90 * r->n * r->m + (size_t)16 * r->m * r->m + 4096;
}

static double service(const Req *r) {  // the fake executor: seconds alone on the device
  const double nm = (double)r->n * r->m;
  return r->heavy ? 2e-11 * nm * r->m : 2e-9 * nm + 1e-3;
}

#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      std::exit(1);                                               \
    }                                                             \
  } while (0)

int main(int argc, char **argv) {
  const int count = argc > 1 ? std::atoi(argv[1]) : 300;
  const double qps = argc > 2 ? std::atof(argv[2]) : 2.0;
  const uint64_t budget = argc > 3 ? std::strtoull(argv[3], nullptr, 10) : (uint64_t)32 << 30;
  const int lanes = argc > 4 ? std::atoi(argv[4]) : 3;
  std::mt19937_64 g(12345);
  std::exponential_distribution<double> gap(qps);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  std::vector<Req> reqs(count);
  double t = 0.0;
  for (int k = 0; k < count; k++) {
    t += gap(g);
    Req &r = reqs[k];
    r.id = k + 1;
    r.n = (int)std::lround(std::exp(std::log(256.0) + u(g) * (std::log(16384.0) - std::log(256.0))));
    r.m = u(g) < 0.5 ? r.n : std::max(1, (int)std::lround(0.1 * r.n));
    r.heavy = (int64_t)r.n * r.m >= ((int64_t)1 << 22);
    r.arrival = t;
  }
  auto need = [](const std::vector<Req *> &rs) {
    size_t b = 0;
    for (const Req *r : rs) b += need1(r);
    return b;
  };

  std::deque<Req *> light, heavy;
  std::vector<double> lane_free(lanes, 0.0);
  struct Running { double end; size_t bytes; std::vector<Req *> rs; int lane; };
  std::vector<Running> running;
  uint64_t used = 0;
  int next_arrival = 0, order_light = 0, order_heavy = 0, rounds = 0, multi = 0;
  double now = 0.0;
  int64_t last_light = 0, last_heavy = 0;
  while (true) {
    // admit whatever can start now
    for (int l = 0; l < lanes; l++) {
      if (lane_free[l] > now) continue;
      bool busy = false;
      for (const Running &x : running) busy |= x.lane == l;
      if (busy) continue;
      for (;;) {
        std::vector<Req *> round;
        size_t bytes = 0;
        const int r = te::sched_next(light, heavy, budget, used, need, round, bytes);
        if (r == 0) break;
        if (r == 2) {
          CHECK(round.size() == 1 && need1(round[0]) > budget);
          round[0]->rejected = true;
          round[0]->start = round[0]->done = now;
          continue;
        }
        CHECK(bytes == need(round) && used + bytes <= budget);
        const bool hv = round[0]->heavy;
        double svc = 0.0;
        for (Req *q : round) {
          CHECK(q->heavy == hv);                     // one class per round
          CHECK(need1(q) <= budget);
          const double a = (double)round[0]->n * round[0]->m, b = (double)q->n * q->m;
          if (hv) CHECK(a <= te::kHeavySpread * b && b <= te::kHeavySpread * a);
          int64_t &last = hv ? last_heavy : last_light;
          CHECK(q->id > last);                       // FIFO within the class
          last = q->id;
          q->order = hv ? order_heavy++ : order_light++;
          q->start = now;
          svc = std::max(svc, service(q));
        }
        // the oldest waiting request decided the class: nothing older waits in the other queue
        const std::deque<Req *> &other = hv ? light : heavy;
        if (!other.empty()) CHECK(other.front()->id > round[0]->id);
        used += bytes;
        rounds++;
        multi += round.size() > 1;
        running.push_back({now + svc, bytes, round, l});
        break;
      }
    }
    // next event: an arrival or a round's completion
    double t_arr = next_arrival < count ? reqs[next_arrival].arrival : INFINITY;
    double t_end = INFINITY;
    size_t ie = 0;
    for (size_t i = 0; i < running.size(); i++)
      if (running[i].end < t_end) { t_end = running[i].end; ie = i; }
    if (t_arr == INFINITY && t_end == INFINITY) {
      CHECK(light.empty() && heavy.empty());
      break;
    }
    if (t_arr <= t_end) {
      now = t_arr;
      Req *r = &reqs[next_arrival++];
      (r->heavy ? heavy : light).push_back(r);
    } else {
      now = t_end;
      Running x = running[ie];
      running.erase(running.begin() + ie);
      for (Req *q : x.rs) q->done = now;
      CHECK(used >= x.bytes);
      used -= x.bytes;
    }
  }
  std::vector<double> lat;
  int rejected = 0;
  double makespan = 0.0;
  for (const Req &r : reqs) {
    CHECK(r.done >= r.start && r.start >= r.arrival);
    if (r.rejected) { rejected++; continue; }
    lat.push_back(r.done - r.arrival);
    makespan = std::max(makespan, r.done);
  }
  CHECK(used == 0);
  std::sort(lat.begin(), lat.end());
  auto pct = [&](double p) {   // linear interpolation between order statistics
    const double x = p / 100.0 * (lat.size() - 1);
    const size_t i = (size_t)x;
    return i + 1 < lat.size() ? lat[i] + (x - i) * (lat[i + 1] - lat[i]) : lat[i];
  };
  std::printf("{\"requests\": %d, \"rejected\": %d, \"rounds\": %d, \"multi_request_rounds\": %d, "
              "\"p50_s\": %.6f, \"p99_s\": %.6f, \"makespan_s\": %.6f}\n",
              count, rejected, rounds, multi, pct(50), pct(99), makespan);
  return 0;
}
