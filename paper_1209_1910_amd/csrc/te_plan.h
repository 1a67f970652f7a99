// Which kernel runs each cluster chain, host-only C++ (no HIP), so that the
// rule can be exercised without a device.
//
// A chain whose Y block (n x size entries) reaches kLargeEntries runs in the
// cooperative kernel, on a group of workgroups sized by its cost size^2 n;
// smaller chains run one per workgroup.  When a call has no more chains than
// the cooperative kernel has workgroups, chains from kPromoteEntries up go to
// the cooperative kernel as well: one workgroup per chain would leave most of
// the device idle while each chain's steps run latency-bound in one workgroup
// (and before the cooperative launch), and the group planner spreads every
// workgroup over the chains by cost instead.  That is skipped when a chain
// that needs the cooperative kernel anyway costs more than kPromoteRatio times
// the largest of the promotable ones: beside it they would each take a
// workgroup from its group for little gain (promoting regardless made large
// random matrices with a few huge clusters and many mid-size ones up to 2.9x
// slower).  MGS chains always run one per workgroup.
#pragma once

#include <cstddef>
#include <vector>

namespace te {

constexpr size_t kLargeEntries = (size_t)1 << 20;
constexpr size_t kPromoteEntries = (size_t)1 << 17;
constexpr double kPromoteRatio = 8.0;

enum ChainKernel : char { kChainOneWg = 0, kChainCoop = 1, kChainPromoted = 2 };

// n[k], size[k]: order of chain k's problem and its member count (>= 2).
// coop_wgs: workgroups of the cooperative kernel.  Returns one ChainKernel
// per chain.
inline std::vector<char> chain_kernels(const std::vector<int> &n, const std::vector<int> &size,
                                       size_t coop_wgs, bool mgs) {
  const size_t K = size.size();
  std::vector<char> out(K, kChainOneWg);
  if (mgs) return out;
  double large_max = 0.0, promote_max = 0.0;
  for (size_t k = 0; k < K; k++) {
    const size_t entries = (size_t)size[k] * (size_t)n[k];
    const double cost = (double)size[k] * size[k] * n[k];
    if (entries >= kLargeEntries) {
      out[k] = kChainCoop;
      large_max = cost > large_max ? cost : large_max;
    } else if (entries >= kPromoteEntries) {
      promote_max = cost > promote_max ? cost : promote_max;
    }
  }
  if (promote_max > 0.0 && promote_max * kPromoteRatio >= large_max && K <= coop_wgs) {
    for (size_t k = 0; k < K; k++)
      if (out[k] == kChainOneWg && (size_t)size[k] * (size_t)n[k] >= kPromoteEntries)
        out[k] = kChainPromoted;
  }
  return out;
}

}  // namespace te
