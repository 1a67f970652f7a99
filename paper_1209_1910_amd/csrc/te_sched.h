// Admission policy of the serving engine, host-only C++ (no HIP), so that it
// can be driven by a simulated clock and executor as well as by the server.
//
// Requests wait in two FIFO queues, light and heavy.  The oldest waiting
// request (smallest id) decides which queue the next round takes from; the
// round takes that queue's requests in order while the device memory of the
// rounds in flight plus this round stays within the budget, up to kMaxRound.
// A heavy round ends with its longest cluster chain, which no split of the
// device shortens, so a request joins the head's heavy round only while its
// size n m is within a factor kHeavySpread of the head's.  A request that
// needs more than the whole budget can never run: it is taken out alone and
// reported as rejected.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <vector>

namespace te {

constexpr int kMaxRound = 512;        // requests per round
constexpr double kHeavySpread = 2.0;  // size ratio of requests sharing a heavy round

// R: a request type with fields id (int64_t), n, m (int).  need(round) returns
// the device bytes a round of these requests holds while it runs.
// Returns 1 when `round` (and `bytes`) hold the next round, 2 when `round`
// holds one request that can never be admitted (need > budget), 0 when the
// caller must wait (nothing queued, or the head does not fit beside the
// rounds in flight).  The chosen requests leave their queue.
template <class R, class Need>
int sched_next(std::deque<R *> &light, std::deque<R *> &heavy, uint64_t budget, uint64_t used,
               Need need, std::vector<R *> &round, size_t &bytes) {
  round.clear();
  bytes = 0;
  if (light.empty() && heavy.empty()) return 0;
  std::deque<R *> *q = &light;
  if (light.empty() || (!heavy.empty() && heavy.front()->id < light.front()->id)) q = &heavy;
  R *head = q->front();
  const size_t first = need(std::vector<R *>{head});
  if (first > budget) {
    q->pop_front();
    round.push_back(head);
    return 2;
  }
  if (used + first > budget) return 0;
  round.push_back(head);
  q->pop_front();
  bytes = first;
  while (!q->empty() && (int)round.size() < kMaxRound) {
    if (q == &heavy) {
      const double a = (double)head->n * head->m, b = (double)q->front()->n * q->front()->m;
      if (a > kHeavySpread * b || b > kHeavySpread * a) break;
    }
    round.push_back(q->front());
    const size_t b = need(round);
    if (used + b > budget) {
      round.pop_back();
      break;
    }
    bytes = b;
    q->pop_front();
  }
  return 1;
}

}  // namespace te
