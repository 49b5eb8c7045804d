// Layout builder: host COO synapse list -> grouped pull records.
//
// Post-neurons are cut into groups of 64 (one wavefront, one 64-bit spike
// word).  All synapses into a group are stored contiguously, so one workgroup
// streams them with fully coalesced 8-byte loads, in two parts: delay >= 2
// (deliverable before the previous step's spikes are known), then delay 1.
//
// Inside a part the records are laid out in rows of 64 where lane l of every
// row holds a synapse of post-neuron l ("lane-owned" rows): row r carries the
// r-th synapse of each post, or a filler (weight -0.0) where that post has no
// more.  A lane then sums its post's input in a register, with no atomic
// operation.  Rows stop at R, chosen per part to balance filler slots
// against the synapses of the few posts with more than R; those overflow
// records follow the rows, round-robin over their posts, padded to a
// multiple of 64, and are accumulated with LDS atomics.  Every section is a
// multiple of 64 records, so record k of a group sits in lane
// (k - gptr[g]) mod 64.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>

#include "sn_internal.h"

namespace snmi {

namespace {

// Cost model of one part: a lane-owned row costs its 64 slots, an overflow
// record about eight slots (an LDS atomic).  Returns the best row count.
int64_t lane_rows(const std::vector<int64_t>& deg) {
  int64_t maxdeg = 0;
  for (int64_t d : deg) maxdeg = std::max(maxdeg, d);
  int64_t best_r = maxdeg, best_cost = 64 * maxdeg;
  // overflow(R) = sum over posts of max(0, deg - R), scanned downwards
  std::vector<int64_t> sorted(deg);
  std::sort(sorted.begin(), sorted.end(), std::greater<int64_t>());
  int64_t over = 0;
  size_t above = 0;  // posts with deg > R
  for (int64_t R = maxdeg; R >= 0; --R) {
    while (above < sorted.size() && sorted[above] > R) ++above;
    if (R < maxdeg) over += static_cast<int64_t>(above);
    const int64_t cost = 64 * R + 8 * ((over + 63) / 64 * 64);
    if (cost < best_cost) {
      best_cost = cost;
      best_r = R;
    }
  }
  return best_r;
}

}  // namespace

HostLayout build_layout(int32_t n, int64_t nnz, const int32_t* pre, const int32_t* post, const float* w,
                        const uint8_t* delay, int32_t max_delay, int32_t phase_rows, bool lane_only, int32_t block) {
  HostLayout L;
  // delay phases (phase p: delays p * phase_rows + 1 .. (p + 1) * phase_rows);
  // part A holds the sections of phases P-1 .. 1, then phase 0 (delays >= 2)
  const int32_t P = phase_rows > 0 ? std::max<int32_t>(1, (max_delay + phase_rows - 1) / phase_rows) : 1;
  L.phases = P;
  L.phase_rows = P > 1 ? phase_rows : 0;
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
  L.recs.reserve(static_cast<size_t>(nnz) + static_cast<size_t>(nnz) / 4 + 128 * static_cast<size_t>(G));
  L.src.reserve(L.recs.capacity());
  // a synapse's weight, with -0 stored as +0 (-0 marks fillers)
  auto weight = [&](int64_t k) { return w[k] == 0.f ? 0.f : w[k]; };
  auto filler = [&](uint32_t delay, uint32_t lane) {
    L.recs.push_back(Rec{-0.f, pack_meta(0u, delay, lane)});
    L.src.push_back(-1);
  };
  L.gptr.assign(static_cast<size_t>(G) + 1, 0);
  L.gsplit.assign(static_cast<size_t>(G), 0);
  L.wsec.assign(static_cast<size_t>(G) * P, 0);
  L.block = block;
  L.ssec.assign(static_cast<size_t>(G) * (block - 1), 0);
  std::vector<std::vector<int64_t>> lists(kGroup);
  std::vector<int64_t> deg(kGroup);
  for (int32_t g = 0; g < G; ++g) {
    L.gptr[g] = static_cast<int32_t>(L.recs.size());
    const int32_t j0 = g * kGroup;
    const int32_t j1 = std::min(n, j0 + kGroup);
    // sections: phases P-1 .. 0 of part A (delay >= block), then the short
    // delays block - 1 .. 1 (block 2: part B, delay 1)
    for (int sec = 0; sec < P + block - 1; ++sec) {
      const int part = sec >= P ? 1 : 0;
      const int32_t ph = P - 1 - sec;  // phase of a part-A section
      const int32_t dshort = P + block - 1 - sec;  // delay of a short section
      const int32_t dlo = part == 1 ? dshort : P > 1 ? std::max(block, ph * phase_rows + 1) : block;
      const int32_t dhi = part == 1 ? dshort : P > 1 ? (ph + 1) * phase_rows : 64;
      if (part == 1) {
        L.ssec[static_cast<size_t>(g) * (block - 1) + dshort - 1] = static_cast<int32_t>(L.recs.size());
        if (dshort == 1) L.gsplit[g] = static_cast<int32_t>(L.recs.size());
      } else {
        L.wsec[static_cast<size_t>(g) * P + ph] = static_cast<int32_t>(L.recs.size());
      }
      for (int l = 0; l < kGroup; ++l) {
        lists[l].clear();
        const int32_t j = j0 + l;
        if (j < j1) {
          for (int64_t q = colptr[j]; q < colptr[j + 1]; ++q) {
            const int32_t dq = delay[order[q]];
            if (dq >= dlo && dq <= dhi) lists[l].push_back(order[q]);
          }
        }
        deg[l] = static_cast<int64_t>(lists[l].size());
      }
      // a filler names neuron 0 with a delay of this section and weight -0
      const uint32_t fill_delay = static_cast<uint32_t>(dlo);
      int64_t R = lane_rows(deg);
      if (lane_only)  // every synapse in its post's lane: as many rows as the largest in-degree
        for (int l = 0; l < kGroup; ++l) R = std::max(R, deg[l]);
      for (int64_t r = 0; r < R; ++r) {
        for (int l = 0; l < kGroup; ++l) {
          if (deg[l] > r) {
            const int64_t k = lists[l][r];
            L.recs.push_back(Rec{weight(k), pack_meta(static_cast<uint32_t>(pre[k]), delay[k], static_cast<uint32_t>(l))});
            L.src.push_back(static_cast<int32_t>(k));
          } else {
            filler(fill_delay, static_cast<uint32_t>(l));
          }
        }
      }
      // overflow of the posts with more than R synapses in this part
      int64_t more = 0;
      for (int l = 0; l < kGroup; ++l) more = std::max(more, deg[l] - R);
      int64_t count = 0;
      for (int64_t r = R; r < R + more; ++r) {
        for (int l = 0; l < kGroup; ++l) {
          if (deg[l] <= r) continue;
          const int64_t k = lists[l][r];
          L.recs.push_back(Rec{weight(k), pack_meta(static_cast<uint32_t>(pre[k]), delay[k], static_cast<uint32_t>(l))});
          L.src.push_back(static_cast<int32_t>(k));
          ++count;
        }
      }
      for (; count % kGroup != 0; ++count) filler(fill_delay, static_cast<uint32_t>(count % kGroup));
    }
    if (L.recs.size() > static_cast<size_t>(INT32_MAX)) {  // offsets are 32-bit on the device
      L.too_large = true;
      return L;
    }
    L.max_group_records = std::max<int32_t>(L.max_group_records, static_cast<int32_t>(L.recs.size() - L.gptr[g]));
  }
  L.gptr[G] = static_cast<int32_t>(L.recs.size());
  return L;
}

std::vector<uint32_t> compact_records(const HostLayout& L, int32_t n, int32_t max_delay, float* scale) {
  std::vector<uint32_t> out;
  const uint32_t W32 = 2u * static_cast<uint32_t>((n + kGroup - 1) / kGroup);
  const uint32_t Dr = static_cast<uint32_t>(max_delay) + 1u;
  if (L.recs.empty() || static_cast<uint64_t>(Dr) * W32 > kCompactMaxRing) return out;
  std::vector<float> w(L.recs.size());
  for (size_t i = 0; i < w.size(); ++i) w[i] = L.recs[i].w;
  const int32_t e = int8_exponent(w.data(), static_cast<int64_t>(w.size()));
  if (e < 0) return out;
  const float f = std::ldexp(1.f, e);
  out.resize(L.recs.size());
  for (size_t i = 0; i < out.size(); ++i) {
    const Rec& r = L.recs[i];
    const int32_t k = static_cast<int32_t>(r.w * f);  // exact: an integer of magnitude <= 127
    const uint32_t pre = r.meta & 0xFFFFFu, d = ((r.meta >> 20) & 63u) + 1u;
    const uint32_t delta = ((r.meta >> 26) - static_cast<uint32_t>(i % kGroup)) & 63u;  // 0: the lane's own post
    out[i] = compact_record(k, (Dr - d) * W32 + (pre >> 5), pre & 31u, delta);
  }
  *scale = std::ldexp(1.f, -e);
  return out;
}

std::vector<uint32_t> lane_records(const HostLayout& L, int32_t G, float* scale) {
  std::vector<uint32_t> out;
  if (L.recs.empty()) return out;
  std::vector<float> w(L.recs.size());
  for (size_t i = 0; i < w.size(); ++i) w[i] = L.recs[i].w;
  const int32_t e = int8_exponent(w.data(), static_cast<int64_t>(w.size()));
  if (e < 0) return out;
  const float f = std::ldexp(1.f, e);
  const uint32_t W32 = 2u * static_cast<uint32_t>(G);
  out.resize(L.recs.size());
  for (size_t i = 0; i < out.size(); ++i) {
    const Rec& r = L.recs[i];
    if ((r.meta >> 26) != static_cast<uint32_t>(i % kGroup)) return {};  // not lane-owned
    const int32_t k = static_cast<int32_t>(r.w * f);  // exact: an integer of magnitude <= 127
    const uint32_t pre = r.meta & 0xFFFFFu, d1 = (r.meta >> 20) & 63u;  // d1 = delay - 1
    // rows 0 .. block - 2 of the staged rows hold the history of later steps
    const uint32_t row = (L.phase_rows > 0 ? d1 % static_cast<uint32_t>(L.phase_rows) : d1) +
                         static_cast<uint32_t>(L.block - 1);
    const uint64_t offset = (static_cast<uint64_t>(row) * W32 + (pre >> 5)) * 4u;
    if (offset >= kLaneMaxOffset) return {};
    out[i] = lane_record(k, static_cast<uint32_t>(offset), pre & 31u);
  }
  *scale = std::ldexp(1.f, -e);
  return out;
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
  for (int32_t w = 0; w < p.P; ++w) {
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

int32_t int8_exponent(const float* W, int64_t count) {
  for (int32_t e = 0; e <= 24; ++e) {
    const float f = std::ldexp(1.f, e);
    bool ok = true;
    for (int64_t i = 0; i < count && ok; ++i) {
      const float v = W[i] * f;  // exact: scaling by a power of two
      ok = std::fabs(v) <= 127.f && v == std::nearbyint(v);
    }
    if (ok) return e;
  }
  return -1;
}

void tile_dense_weights_i8(const float* W, int32_t n, int32_t npad, int32_t kpad, int32_t e, int8_t* out) {
  const int32_t C = npad / 16, J = kpad / 128;
  const float f = std::ldexp(1.f, e);
  size_t o = 0;
  for (int32_t c = 0; c < C; ++c)
    for (int32_t j = 0; j < J; ++j)
      for (int32_t s = 0; s < 2; ++s)
        for (int32_t q = 0; q < 4; ++q)
          for (int32_t col = 0; col < 16; ++col)
            for (int32_t i = 0; i < 16; ++i) {
              const int32_t k = 32 * (4 * j + q) + 16 * s + i;
              const int32_t jj = 16 * c + col;
              out[o++] = (k < n && jj < n) ? static_cast<int8_t>(W[static_cast<size_t>(k) * n + jj] * f) : int8_t(0);
            }
}

}  // namespace snmi
