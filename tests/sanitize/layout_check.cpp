// Host-side check of the synapse layout builder (layout.cpp), built with g++
// under AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_layout_sanitized.py.  It builds the pull layout (with and
// without delay phases), the slice partitions and the push layout of awkward
// nets and checks the invariants the kernels rely on:
//   - group offsets increase, every group and every section (delay phases,
//     delay-1 part) is a multiple of 64 records;
//   - every input synapse appears exactly once, with its weight (-0 stored
//     as +0), pre-neuron, delay and post-neuron; fillers carry -0.0 and
//     source -1;
//   - a record sits in lane (offset within its group) mod 64, and a record
//     in a lane-owned row belongs to that lane's post; overflow records follow
//     the rows of their section;
//   - the delays of a section lie in its phase (part B: delay 1);
//   - the compact records (batch kernel) decode to each record's ring
//     offset, source bit, post and weight;
//   - the lane-only layout holds every synapse once in its post's lane, and
//     its lane records decode to the LDS offset and bit of the source in the
//     phase's staged rows and to the weight;
//   - slices of a partition are contiguous and cover all groups;
//   - the push layout lists every synapse once under its pre-neuron.
// Prints "ok <cases>" and exits 0, or names the first violated invariant.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "../../paper_2305_02510_amd/csrc/sn_internal.h"

using namespace snmi;

static int g_fail = 0;
#define CHECK(cond, ...)                          \
  do {                                            \
    if (!(cond)) {                                \
      std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
      std::printf(__VA_ARGS__);                   \
      std::printf("\n");                          \
      g_fail = 1;                                 \
      return;                                     \
    }                                             \
  } while (0)

struct Net {
  int32_t n = 1, D = 1;
  std::vector<int32_t> pre, post;
  std::vector<float> w;
  std::vector<uint8_t> d;
};

static bool is_neg_zero(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  return u == 0x80000000u;
}

static void check_layout(const Net& net, int32_t phase_rows) {
  const int64_t nnz = static_cast<int64_t>(net.pre.size());
  HostLayout L = build_layout(net.n, nnz, net.pre.data(), net.post.data(), net.w.data(), net.d.data(), net.D,
                              phase_rows);
  CHECK(!L.too_large, "unexpected too_large");
  const int32_t G = (net.n + kGroup - 1) / kGroup;
  const int32_t P = L.phases;
  CHECK(static_cast<int32_t>(L.gptr.size()) == G + 1 && static_cast<int32_t>(L.gsplit.size()) == G, "table sizes");
  CHECK(L.recs.size() == L.src.size(), "src size");
  CHECK(L.gptr[0] == 0 && L.gptr[G] == static_cast<int64_t>(L.recs.size()), "gptr ends");
  CHECK(P >= 1 && static_cast<int64_t>(L.wsec.size()) == static_cast<int64_t>(G) * P, "wsec size");
  std::vector<int> seen(static_cast<size_t>(nnz), 0);
  for (int32_t g = 0; g < G; ++g) {
    const int32_t a = L.gptr[g], e = L.gptr[g + 1], sp = L.gsplit[g];
    CHECK(a <= sp && sp <= e, "group %d: split outside", g);
    CHECK((sp - a) % kGroup == 0 && (e - sp) % kGroup == 0, "group %d: parts not multiples of 64", g);
    CHECK(e - a <= L.max_group_records, "group %d: max_group_records", g);
    // section bounds: phases P-1 .. 0 of part A, then part B
    std::vector<int32_t> bound;
    for (int32_t p = P - 1; p >= 0; --p) bound.push_back(L.wsec[static_cast<size_t>(g) * P + p]);
    bound.push_back(sp);
    bound.push_back(e);
    CHECK(bound[0] == a, "group %d: first section does not start the group", g);
    for (size_t q = 0; q + 1 < bound.size(); ++q) {
      CHECK(bound[q] <= bound[q + 1] && (bound[q + 1] - bound[q]) % kGroup == 0, "group %d: section %zu", g, q);
      const bool partB = q + 1 == bound.size() - 1;
      const int32_t ph = partB ? 0 : P - 1 - static_cast<int32_t>(q);
      int32_t dlo = 2, dhi = 64;
      if (partB) dlo = dhi = 1;
      else if (P > 1) {
        dlo = std::max(2, ph * L.phase_rows + 1);
        dhi = (ph + 1) * L.phase_rows;
      }
      bool overflow = false;  // once a record leaves its lane, the rest of the section is overflow
      for (int32_t i = bound[q]; i < bound[q + 1]; ++i) {
        const Rec& r = L.recs[i];
        const uint32_t pre = r.meta & 0xFFFFFu, del = ((r.meta >> 20) & 63u) + 1, pl = r.meta >> 26;
        const int lane = (i - a) % kGroup;
        CHECK(static_cast<int32_t>(del) >= dlo && static_cast<int32_t>(del) <= dhi,
              "group %d rec %d: delay %u outside [%d, %d]", g, i, del, dlo, dhi);
        const int32_t k = L.src[i];
        if (k < 0) {
          CHECK(k == -1 && is_neg_zero(r.w), "filler %d: weight or source", i);
          CHECK(static_cast<int>(pl) == lane, "filler %d not on its lane", i);
          continue;
        }
        CHECK(k < nnz, "record %d: source %d", i, k);
        ++seen[k];
        const float wk = net.w[k] == 0.f ? 0.f : net.w[k];
        CHECK(std::memcmp(&wk, &r.w, 4) == 0, "record %d: weight", i);
        CHECK(static_cast<int32_t>(pre) == net.pre[k] && static_cast<int32_t>(del) == net.d[k], "record %d: pre/delay", i);
        CHECK(g * kGroup + static_cast<int32_t>(pl) == net.post[k], "record %d: post", i);
        if (static_cast<int>(pl) != lane) overflow = true;
        (void)overflow;
      }
    }
  }
  for (int64_t k = 0; k < nnz; ++k) CHECK(seen[k] == 1, "synapse %lld seen %d times", (long long)k, seen[k]);
  // compact records of the batch kernel: offset of the source word from the
  // current ring row ((D + 1 - delay) * 2G + pre / 32), source bit, post
  // (relative to the record's lane) and numerator, whenever the ring fits the
  // offset field
  {
    float scale = 0.f;
    const std::vector<uint32_t> C = compact_records(L, net.n, net.D, &scale);
    const uint32_t W32 = 2u * static_cast<uint32_t>(G), Dr = static_cast<uint32_t>(net.D) + 1u;
    const bool fits = static_cast<uint64_t>(Dr) * W32 <= kCompactMaxRing;
    CHECK(C.empty() == (L.recs.empty() || !fits), "compact records: built %d, ring fits %d", (int)!C.empty(), (int)fits);
    for (size_t i = 0; i < C.size(); ++i) {
      const uint32_t c = C[i];
      const Rec& r = L.recs[i];
      const uint32_t pre = r.meta & 0xFFFFFu, d = ((r.meta >> 20) & 63u) + 1u;
      CHECK(((c >> 5) & (kCompactMaxRing - 1u)) == (Dr - d) * W32 + (pre >> 5), "compact %zu: offset", i);
      CHECK((c & 31u) == (pre & 31u) && ((((c >> 18) + i) & 63u) == (r.meta >> 26)), "compact %zu: bit or post", i);
      const float wk = static_cast<float>(static_cast<int8_t>(c >> 24)) * scale;
      CHECK(wk == r.w, "compact %zu: weight", i);
    }
  }
  // slice partitions
  for (int32_t slices : {1, 2, 7, 256}) {
    SlicePlan p = partition_groups(L, G, slices, 128);
    CHECK(p.P >= 1 && p.wg_group.front() == 0 && p.wg_group.back() == G, "partition ends");
    for (int32_t s = 0; s < p.P; ++s) CHECK(p.wg_group[s] < p.wg_group[s + 1], "empty slice %d", s);
  }
  // push layout
  const int32_t npad = G * kGroup;
  HostPush H = build_push_layout(net.n, npad, nnz, net.pre.data(), net.post.data(), net.w.data(), net.d.data());
  CHECK(static_cast<int32_t>(H.optr.size()) == npad + 1 && H.optr[npad] == nnz, "push offsets");
  for (int32_t i = 0; i < npad; ++i) CHECK(H.optr[i] <= H.optr[i + 1], "push offsets not monotone at %d", i);
  for (int32_t i = 0; i < net.n; ++i) {
    for (int32_t q = H.optr[i]; q < H.optr[i + 1]; ++q) {
      const uint32_t post = H.orecs[q].meta & 0xFFFFFu;
      CHECK(static_cast<int32_t>(post) < net.n, "push record %d: post", q);
    }
  }
}

// The lane-only layout of the wide kernel for blocks of `block` steps and its
// 4-byte lane records: every section whole rows (the phases of the delays >=
// block, then one section per delay block - 1 .. 1), every record in its
// post's lane, and each lane record naming the LDS word and bit of its source
// in the phase's staged rows, with its weight's numerator (fillers: k = 0).
static void check_lane_layout(const Net& net, int32_t phase_rows, int32_t block) {
  const int64_t nnz = static_cast<int64_t>(net.pre.size());
  HostLayout L = build_layout(net.n, nnz, net.pre.data(), net.post.data(), net.w.data(), net.d.data(), net.D,
                              phase_rows, true, block);
  CHECK(!L.too_large, "lane layout: unexpected too_large");
  const int32_t G = (net.n + kGroup - 1) / kGroup;
  const int32_t P = L.phases;
  float scale = 0.f;
  const std::vector<uint32_t> LR = lane_records(L, G, &scale);
  if (nnz == 0) return;
  CHECK(LR.size() == L.recs.size(), "lane records missing (%zu of %zu)", LR.size(), L.recs.size());
  const int64_t row = kGroup;
  std::vector<int> seen(static_cast<size_t>(nnz), 0);
  for (int32_t g = 0; g < G; ++g) {
    // sections: phases P-1 .. 0 of the delay >= block records, then delays block - 1 .. 1
    std::vector<int32_t> bound;
    for (int32_t p = P - 1; p >= 0; --p) bound.push_back(L.wsec[static_cast<size_t>(g) * P + p]);
    for (int32_t d = block - 1; d >= 1; --d) bound.push_back(L.ssec[static_cast<size_t>(g) * (block - 1) + d - 1]);
    CHECK(L.gsplit[g] == bound.back(), "lane group %d: delay-1 section", g);
    bound.push_back(L.gptr[g + 1]);
    CHECK(bound[0] == L.gptr[g], "lane group %d: first section", g);
    for (size_t q = 0; q + 1 < bound.size(); ++q)
      CHECK(bound[q] <= bound[q + 1] && (bound[q + 1] - bound[q]) % row == 0, "lane group %d: section %zu", g, q);
    for (int32_t i = L.gptr[g]; i < L.gptr[g + 1]; ++i) {
      const uint32_t c = LR[i];
      const int32_t k = L.src[i];
      const uint32_t off = (c >> 5) & (kLaneMaxOffset - 1u);
      CHECK(static_cast<int32_t>(L.recs[i].meta >> 26) == (i - L.gptr[g]) % kGroup, "lane record %d off its lane", i);
      // every record, filler or not, names a word of staged row block - 1 or
      // below (the kernels of a block read up to block - 1 rows higher)
      CHECK(off >= static_cast<uint32_t>(block - 1) * 2u * G * 4u, "lane record %d: offset above row %d", i,
            block - 1);
      if (k < 0) {
        CHECK((c >> 24) == 0, "filler %d: k", i);
        continue;
      }
      ++seen[k];
      const int32_t pre = net.pre[k], d = net.d[k];
      // a short delay in its own section, delays >= block of phase p in phase p's
      size_t sec = 0;
      while (bound[sec + 1] <= i) ++sec;
      if (static_cast<int32_t>(sec) >= P) {
        const int32_t ds = P + block - 1 - static_cast<int32_t>(sec);
        CHECK(d == ds, "lane record %d: delay %d in the section of delay %d", i, d, ds);
      } else {
        const int32_t ph = P - 1 - static_cast<int32_t>(sec);
        CHECK(d >= block && (P == 1 || (d - 1) / phase_rows == ph), "lane record %d: delay %d in phase %d", i, d, ph);
      }
      const uint32_t row = (P > 1 ? static_cast<uint32_t>((d - 1) % phase_rows) : static_cast<uint32_t>(d - 1)) +
                           static_cast<uint32_t>(block - 1);
      CHECK(off % 4 == 0 && off / 4 == row * 2u * G + static_cast<uint32_t>(pre) / 32u, "lane record %d: offset", i);
      CHECK((c & 31u) == static_cast<uint32_t>(pre) % 32u, "lane record %d: bit", i);
      const float wk = static_cast<float>(static_cast<int8_t>(c >> 24)) * scale;
      CHECK(wk == net.w[k], "lane record %d: weight", i);
    }
  }
  for (int64_t k = 0; k < nnz; ++k) CHECK(seen[k] == 1, "lane layout: synapse %lld seen %d times", (long long)k, seen[k]);
}

static Net random_net(uint32_t seed, int32_t n, double p, int32_t D, bool dups_and_loops) {
  std::mt19937 rng(seed);
  Net net;
  net.n = n;
  net.D = D;
  const int64_t m = static_cast<int64_t>(p * n * n);
  std::uniform_int_distribution<int32_t> node(0, n - 1), del(1, D), kw(-64, 64);
  for (int64_t i = 0; i < m; ++i) {
    int32_t a = node(rng), b = node(rng);
    if (!dups_and_loops && a == b) continue;
    net.pre.push_back(a);
    net.post.push_back(b);
    net.w.push_back(kw(rng) / 64.f);
    net.d.push_back(static_cast<uint8_t>(del(rng)));
    if (dups_and_loops && i % 17 == 0) {  // a duplicate of this synapse
      net.pre.push_back(a);
      net.post.push_back(b);
      net.w.push_back(-0.f);  // a stored zero weight of either sign reads as +0
      net.d.push_back(static_cast<uint8_t>(del(rng)));
    }
  }
  return net;
}

int main() {
  int cases = 0;
  auto run = [&](const Net& net) {
    for (int32_t pr : {0, 1, 3, 7, 31}) {
      check_layout(net, pr);
      if (g_fail) return;
      ++cases;
      for (int32_t block : {2, 4}) {
        if (pr > 0 && pr < block - 1) continue;  // a later phase must start at a delay >= block
        check_lane_layout(net, pr, block);
        if (g_fail) return;
        ++cases;
      }
    }
  };
  {  // empty nets
    Net e;
    run(e);
    e.n = 130;
    e.D = 64;
    run(e);
  }
  run(random_net(1, 300, 0.05, 16, true));   // duplicates, self-loops, -0 weights
  run(random_net(2, 1000, 0.01, 64, false)); // every delay up to 64
  {                                          // hubs: two posts with thousands of inputs
    Net h = random_net(3, 700, 0.004, 9, false);
    std::mt19937 rng(4);
    for (int32_t j : {5, 600})
      for (int i = 0; i < 3000; ++i) {
        h.pre.push_back(static_cast<int32_t>(rng() % 700));
        h.post.push_back(j);
        h.w.push_back(static_cast<float>(static_cast<int>(rng() % 129) - 64) / 64.f);
        h.d.push_back(static_cast<uint8_t>(1 + rng() % 9));
      }
    run(h);
  }
  {  // the largest index range: 2^20 neurons, a few synapses at the edges
    Net big;
    big.n = 1 << 20;
    big.D = 64;
    const int32_t ends[] = {0, 1, 63, 64, (1 << 20) - 65, (1 << 20) - 2, (1 << 20) - 1};
    for (int32_t a : ends)
      for (int32_t b : ends) {
        big.pre.push_back(a);
        big.post.push_back(b);
        big.w.push_back(0.5f);
        big.d.push_back(static_cast<uint8_t>(1 + (a + b) % 64));
      }
    check_layout(big, 0);
    if (!g_fail) check_layout(big, 16);
    cases += 2;
  }
  if (g_fail) return 1;
  std::printf("ok %d\n", cases);
  return 0;
}
