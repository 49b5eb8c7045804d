// Layout builder: host COO synapse list -> grouped pull records.
//
// Post-neurons are cut into groups of 64 (one wavefront, one 64-bit spike
// word).  All synapses into a group are stored contiguously, so one workgroup
// streams them with fully coalesced 8-byte loads.  Inside a group the records
// are interleaved round-robin over the group's posts (first synapse of every
// post, then the second of every post, ...), so the 64 lanes of one load
// mostly target 64 different posts and their LDS accumulations do not collide.
#include <algorithm>
#include <cstring>
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
  L.gsplit.assign(static_cast<size_t>(G), 0);
  std::vector<int64_t> deg(kGroup);
  std::vector<int64_t> taken(kGroup);
  int64_t pos = 0;
  for (int32_t g = 0; g < G; ++g) {
    L.gptr[g] = static_cast<int32_t>(pos);
    const int32_t j0 = g * kGroup;
    const int32_t j1 = std::min(n, j0 + kGroup);
    // part 0: delay >= 2 (deliverable before the previous step's spikes
    // arrive); part 1: delay 1.  Each part round-robin over the group's posts.
    for (int part = 0; part < 2; ++part) {
      if (part == 1) L.gsplit[g] = static_cast<int32_t>(pos);
      int64_t maxdeg = 0;
      for (int32_t j = j0; j < j1; ++j) {
        int64_t c = 0;
        for (int64_t q = colptr[j]; q < colptr[j + 1]; ++q) c += ((delay[order[q]] == 1) == (part == 1));
        deg[j - j0] = c;
        taken[j - j0] = colptr[j];
        maxdeg = std::max(maxdeg, c);
      }
      for (int64_t r = 0; r < maxdeg; ++r) {
        for (int32_t j = j0; j < j1; ++j) {
          if (deg[j - j0] <= r) continue;
          int64_t q = taken[j - j0];
          while ((delay[order[q]] == 1) != (part == 1)) ++q;  // next synapse of this part
          taken[j - j0] = q + 1;
          const int64_t k = order[q];
          L.recs[pos++] = Rec{w[k], pack_meta(static_cast<uint32_t>(pre[k]), delay[k],
                                              static_cast<uint32_t>(j - j0))};
        }
      }
    }
    L.max_group_records = std::max<int32_t>(L.max_group_records, static_cast<int32_t>(pos - L.gptr[g]));
  }
  L.gptr[G] = static_cast<int32_t>(pos);
  // chunk table: every part-0 chunk (group order), then every part-1 chunk
  L.gchunk.assign(2 * (static_cast<size_t>(G) + 1), 0);
  for (int part = 0; part < 2; ++part) {
    for (int32_t g = 0; g < G; ++g) {
      L.gchunk[part * (G + 1) + g] = static_cast<int32_t>(L.chunks.size());
      const int64_t b = part == 0 ? L.gptr[g] : L.gsplit[g];
      const int64_t e = part == 0 ? L.gsplit[g] : L.gptr[g + 1];
      for (int64_t s = b; s < e; s += kChunk) {
        const uint32_t cnt = static_cast<uint32_t>(std::min<int64_t>(kChunk, e - s));
        L.chunks.push_back(make_uint2(static_cast<uint32_t>(s), static_cast<uint32_t>(g) | (cnt << 20)));
      }
    }
    L.gchunk[part * (G + 1) + G] = static_cast<int32_t>(L.chunks.size());
  }
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
  p.wg_chunk.resize(2 * p.wg_group.size());
  for (size_t i = 0; i < p.wg_group.size(); ++i) {
    p.wg_chunk[i] = L.gchunk[p.wg_group[i]];
    p.wg_chunk[p.wg_group.size() + i] = L.gchunk[G + 1 + p.wg_group[i]];
  }
  const size_t P1 = p.wg_group.size();
  for (int32_t w = 0; w < p.P; ++w) {
    p.max_chunks = std::max(p.max_chunks, (p.wg_chunk[w + 1] - p.wg_chunk[w]) + (p.wg_chunk[P1 + w + 1] - p.wg_chunk[P1 + w]));
    p.ng_max = std::max(p.ng_max, p.wg_group[w + 1] - p.wg_group[w]);
    p.max_recs = std::max<int64_t>(p.max_recs, L.gptr[p.wg_group[w + 1]] - L.gptr[p.wg_group[w]]);
  }
  return p;
}

HostPush build_push_layout(int32_t n, int32_t npad, int64_t nnz, const int32_t* pre, const int32_t* post,
                           const float* w, const uint8_t* delay) {
  HostPush P;
  P.optr.assign(static_cast<size_t>(npad) + 1, 0);
  for (int64_t k = 0; k < nnz; ++k) P.optr[pre[k] + 1]++;
  for (int32_t i = 0; i < npad; ++i) P.optr[i + 1] += P.optr[i];
  P.orecs.resize(static_cast<size_t>(nnz));
  std::vector<int32_t> fill(P.optr.begin(), P.optr.end() - 1);
  for (int64_t k = 0; k < nnz; ++k)
    P.orecs[fill[pre[k]]++] = Rec{w[k], static_cast<uint32_t>(post[k]) | ((static_cast<uint32_t>(delay[k]) - 1u) << 20)};
  (void)n;
  return P;
}

size_t dense_tiled_elems(int32_t npad, int32_t kpad) { return static_cast<size_t>(npad) * kpad; }

// bfloat16 bits of a float that is exactly representable (low half zero).
static uint16_t bf16_bits(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  return static_cast<uint16_t>(u >> 16);
}

void tile_dense_weights(const float* W, int32_t n, int32_t npad, int32_t kpad, uint16_t* out) {
  const int32_t C = npad / 16, J = kpad / 128;
  size_t o = 0;
  for (int32_t c = 0; c < C; ++c)
    for (int32_t j = 0; j < J; ++j)
      for (int32_t s = 0; s < 4; ++s)
        for (int32_t q = 0; q < 4; ++q)
          for (int32_t col = 0; col < 16; ++col)
            for (int32_t e = 0; e < 8; ++e) {
              const int32_t k = 8 * (16 * j + 4 * q + s) + e;
              const int32_t jj = 16 * c + col;
              out[o++] = (k < n && jj < n) ? bf16_bits(W[static_cast<size_t>(k) * n + jj]) : uint16_t(0);
            }
}

}  // namespace snmi
