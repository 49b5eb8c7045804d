// Layout builder: host COO synapse list -> grouped pull records.
//
// Post-neurons are cut into groups of 64 (one wavefront, one 64-bit spike
// word).  All synapses into a group are stored contiguously, so one workgroup
// streams them with fully coalesced 8-byte loads.  Inside a group the records
// are interleaved round-robin over the group's posts (first synapse of every
// post, then the second of every post, ...), so the 64 lanes of one load
// mostly target 64 different posts and their LDS accumulations do not collide.
#include <algorithm>
#include <numeric>

#include "sn_internal.h"

namespace snmi {

HostLayout build_layout(int32_t n, int64_t nnz, const int32_t* pre, const int32_t* post, const float* w,
                        const uint8_t* delay) {
  HostLayout L;
  const int32_t G = (n + kGroup - 1) / kGroup;
  // bucket synapses by post-neuron, keeping input order inside a bucket
  std::vector<int64_t> colptr(static_cast<size_t>(n) + 1, 0);
  for (int64_t k = 0; k < nnz; ++k) colptr[post[k] + 1]++;
  for (int32_t j = 0; j < n; ++j) colptr[j + 1] += colptr[j];
  std::vector<int64_t> order(static_cast<size_t>(nnz));
  {
    std::vector<int64_t> fill(colptr.begin(), colptr.end() - 1);
    for (int64_t k = 0; k < nnz; ++k) order[fill[post[k]]++] = k;
  }
  L.recs.resize(static_cast<size_t>(nnz));
  L.gptr.assign(static_cast<size_t>(G) + 1, 0);
  int64_t pos = 0;
  for (int32_t g = 0; g < G; ++g) {
    L.gptr[g] = static_cast<int32_t>(pos);
    const int32_t j0 = g * kGroup;
    const int32_t j1 = std::min(n, j0 + kGroup);
    int64_t maxdeg = 0;
    for (int32_t j = j0; j < j1; ++j) maxdeg = std::max(maxdeg, colptr[j + 1] - colptr[j]);
    for (int64_t r = 0; r < maxdeg; ++r) {
      for (int32_t j = j0; j < j1; ++j) {
        if (colptr[j + 1] - colptr[j] <= r) continue;
        const int64_t k = order[colptr[j] + r];
        L.recs[pos++] = Rec{w[k], pack_meta(static_cast<uint32_t>(pre[k]), delay[k],
                                            static_cast<uint32_t>(j - j0))};
      }
    }
    L.max_group_records = std::max<int32_t>(L.max_group_records, static_cast<int32_t>(pos - L.gptr[g]));
  }
  L.gptr[G] = static_cast<int32_t>(pos);
  L.gchunk.assign(static_cast<size_t>(G) + 1, 0);
  for (int32_t g = 0; g < G; ++g) {
    L.gchunk[g] = static_cast<int32_t>(L.chunks.size());
    for (int64_t s = L.gptr[g]; s < L.gptr[g + 1]; s += kChunk) {
      const uint32_t cnt = static_cast<uint32_t>(std::min<int64_t>(kChunk, L.gptr[g + 1] - s));
      L.chunks.push_back(make_uint2(static_cast<uint32_t>(s), static_cast<uint32_t>(g) | (cnt << 20)));
    }
  }
  L.gchunk[G] = static_cast<int32_t>(L.chunks.size());
  return L;
}

// Greedy contiguous split with a record cap; returns the number of slices.
static int32_t greedy_slices(const HostLayout& L, int32_t G, int64_t cap, int32_t max_groups,
                             std::vector<int32_t>* starts) {
  if (starts) starts->assign(1, 0);
  int32_t count = 1;
  int64_t recs = 0;
  int32_t groups = 0;
  for (int32_t g = 0; g < G; ++g) {
    const int64_t r = L.gptr[g + 1] - L.gptr[g];
    if (groups > 0 && (recs + r > cap || groups + 1 > max_groups)) {
      ++count;
      if (starts) starts->push_back(g);
      recs = 0;
      groups = 0;
    }
    recs += r;
    ++groups;
  }
  if (starts) starts->push_back(G);
  return count;
}

SlicePlan partition_groups(const HostLayout& L, int32_t G, int32_t slices, int32_t max_groups) {
  SlicePlan p;
  slices = std::max(1, std::min(slices, G));
  max_groups = std::max(max_groups, (G + slices - 1) / slices);
  // smallest record cap that still fits in `slices` slices
  int64_t lo = 0, hi = L.gptr[G];
  for (int32_t g = 0; g < G; ++g) lo = std::max<int64_t>(lo, L.gptr[g + 1] - L.gptr[g]);
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (greedy_slices(L, G, mid, max_groups, nullptr) <= slices) hi = mid; else lo = mid + 1;
  }
  greedy_slices(L, G, lo, max_groups, &p.wg_group);
  p.P = static_cast<int32_t>(p.wg_group.size()) - 1;
  p.wg_chunk.resize(p.wg_group.size());
  for (size_t i = 0; i < p.wg_group.size(); ++i) p.wg_chunk[i] = L.gchunk[p.wg_group[i]];
  for (int32_t w = 0; w < p.P; ++w) {
    p.ng_max = std::max(p.ng_max, p.wg_group[w + 1] - p.wg_group[w]);
    p.max_recs = std::max<int64_t>(p.max_recs, L.gptr[p.wg_group[w + 1]] - L.gptr[p.wg_group[w]]);
  }
  return p;
}

}  // namespace snmi
