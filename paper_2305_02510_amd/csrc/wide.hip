// Per-step pull delivery for nets whose spike history does not fit in LDS
// (N = 100,000 with delays up to 16: 16 rows of 100,000 bits = 200 KB), the
// synaptic input of §2.1's update summed over the pull records of every
// post-neuron group, followed by the fused neuron update.
//
// One launch per step, or two per step pair (see MODE below: records of
// delay >= 2 read once for two steps).  Workgroup (w, b) owns the contiguous groups
// [g0, g1) of trial b.  The delays are cut into phases of Dl delays (Dl =
// as many history rows as fit in LDS beside the sums); the layout orders the
// delay >= 2 records of every group by phase (phases P-1 .. 1, then phase 0
// running on into the delay-1 records).  For each phase the workgroup copies
// the raster rows of that phase's delays into LDS once, then streams the
// phase's records of all its groups, finding every source bit in LDS.
// Looking each bit up in the raster in memory instead costs one scattered L2
// request per record, which caps the record stream near 2 TB/s.  Without
// phases (more than kWideMaxPhases would be needed) delays above Dl read the
// raster in memory.
//
// Streaming: in a phase every wave walks its own records with no barrier:
// with at least 16 groups wave w owns groups g0 + w, g0 + w + 16, ...; with
// fewer the 16 waves are spread over the groups as teams of m (16 / ng
// rounded up or down), member i taking batches i, i + m, ... of its group
// (a batch is 512 records, 8 per lane).  Three record buffers
// in rotation keep two batches in flight while one is delivered.  Lane-owned
// rows put every record of post l in lane l, so a lane sums its post's input
// in a register; overflow records of other posts are added into the group's
// LDS row atomically.  An owner adds its sums into the group's row; a team's
// members leave theirs in LDS slots that one member adds after the phase's
// barrier.  After the last phase wave w updates groups g0 + w, g0 + w + 16,
// ... and writes their spike words.
//
// LANE: when every delay is staged (phases cover D) the net may also hold a
// lane-only copy of its layout (no overflow: every record in its post's lane;
// the delay-1 records in a section of their own after the phases)
// as 4-byte lane records that carry the LDS offset of their source word, the
// source's bit and an int8 weight numerator, every section whole rows of
// 64.  The kernel then streams those, half the bytes of the
// 8-byte records, with no atomic, no bounds mask and no address arithmetic
// beyond two bit-field extractions per record; a lane sums its numerators as
// an integer and scales the sum once.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sn_device.h"
#include "sn_internal.h"

namespace snmi {

constexpr int kWideThreads = 1024;
constexpr int kWideWaves = kWideThreads / 64;
constexpr int kWideU = 8;                              // 8-byte records per lane in one batch
constexpr int kWideNpw = 4;                            // groups updated per wave, at most
constexpr int kWideStage = 8;                          // history words per thread in flight while staging
constexpr size_t kWidePartLds = kWideWaves * kGroup * sizeof(float);  // a team's per-wave sums of one step
constexpr size_t kWideStaticLds = 64;
constexpr size_t kWideLdsLimit = 160 * 1024;
constexpr size_t kStepRingLimitWide = 64 * 1024;  // below this the per-group kernel stages every row

// Loads are unconditional, from an index clamped into [0, end) (the records
// array always holds at least one record's worth of memory), so all of them
// stay in flight together; records past `end` are masked when delivered.
__device__ __forceinline__ void wide_load(const DevNet& n, int base, int end, int lane, Rec (&r)[kWideU]) {
#pragma unroll
  for (int u = 0; u < kWideU; ++u) r[u] = n.recs[max(0, min(base + u * 64 + lane, end - 1))];
}

// Records of group g in phase p: phase p >= 1 is the section [wsec[p],
// wsec[p - 1]); phase 0 runs from wsec[0] to the group's end (delay-1 part
// included).  Without phases: all records of the group.  LANE: the offsets of
// the lane-record layout, and `sec` picks part of it: 0 the whole phase as
// above, 1 the phase's records of delay >= 2 (phase 0 ends where the group's
// delay-1 records begin), 2 the group's delay-1 records.
template <bool LANE>
__device__ __forceinline__ void wide_range(const DevNet& n, int g, int p, int sec, int& beg, int& end) {
  const int32_t* gp = LANE ? n.lgptr : n.gptr;
  if (LANE && sec == 2) {
    beg = n.lgsplit[g];
    end = gp[g + 1];
    return;
  }
  const int32_t last = LANE && sec == 1 ? n.lgsplit[g] : gp[g + 1];  // end of phase 0
  if (n.phases <= 1) {
    beg = gp[g];
    end = last;
    return;
  }
  const int32_t* ws = (LANE ? n.lwsec : n.wsec) + static_cast<size_t>(g) * n.phases;
  beg = ws[p];
  end = p == 0 ? last : ws[p - 1];
}

// A wave's walk over the records of one phase.  With ng >= 16 groups wave w
// owns groups g0 + w, g0 + w + 16, ... and walks all their batches; with
// fewer, a team of m waves shares one group, member i taking batches i,
// i + m, ...  A batch is 512 records of one group (8 per lane).
struct WidePair {
  int g, k, beg, end, nb;
  bool valid;
};

__device__ __forceinline__ void wide_enter(const DevNet& n, WidePair& s, int p) {
  constexpr int batch = 64 * kWideU;
  wide_range<false>(n, s.g, p, 0, s.beg, s.end);
  s.nb = max(1, (s.end - s.beg + batch - 1) / batch);
}

__device__ __forceinline__ WidePair wide_start(const DevNet& n, int p, int g0, int g1, bool own, int team,
                                               int member) {
  WidePair s{};
  s.g = g0 + team;  // own: team == wave
  s.k = own ? 0 : member;
  s.valid = s.g < g1;
  if (s.valid) {
    wide_enter(n, s, p);
    s.valid = s.k < s.nb;
  }
  return s;
}

__device__ __forceinline__ WidePair wide_next(const DevNet& n, const WidePair& s, int p, int g1, int m, bool own) {
  WidePair r = s;
  if (!s.valid) return r;
  r.k = s.k + m;
  if (r.k >= s.nb) {
    r.valid = false;
    if (own) {  // the wave's next owned group
      r.g = s.g + kWideWaves;
      r.k = 0;
      r.valid = r.g < g1;
      if (r.valid) wide_enter(n, r, p);
    }
  }
  return r;
}

__device__ __forceinline__ int wide_first(const WidePair& s) { return s.beg + s.k * (64 * kWideU); }

// A pair past the wave's last one loads (and never delivers) that last
// pair's records again.
__device__ __forceinline__ void wide_load_pair(const DevNet& n, const WidePair& s, int lane, Rec (&r)[kWideU]) {
  wide_load(n, wide_first(s), s.end, lane, r);
}

// Lane-record walk: a pair is (group, batch) as above; sections are whole
// rows, so a batch that runs past its section's end skips the rows beyond it
// (a uniform test per row, no per-record mask), and empty sections are
// skipped.  Loads past a section's end stay inside the array's slack.
constexpr int kLaneU = kLaneBatchRows;  // records per lane in one batch
struct LanePair {
  int g, k, beg, end, nb;
  bool valid;
};

__device__ __forceinline__ void lane_enter(const DevNet& n, LanePair& s, int p, int sec) {
  wide_range<true>(n, s.g, p, sec, s.beg, s.end);
  s.nb = (s.end - s.beg + 64 * kLaneU - 1) / (64 * kLaneU);
}

// From s.g: an owning wave moves on to its first group (every 16th) with a
// non-empty section; a team member keeps its group if its batch exists.
__device__ __forceinline__ void lane_settle(const DevNet& n, LanePair& s, int p, int sec, int g1, bool own) {
  s.valid = s.g < g1;
  if (!s.valid) return;
  lane_enter(n, s, p, sec);
  if (own) {
    while (s.nb == 0) {
      s.g += kWideWaves;
      if (s.g >= g1) {
        s.valid = false;
        return;
      }
      lane_enter(n, s, p, sec);
    }
  }
  s.valid = s.k < s.nb;
}

__device__ __forceinline__ LanePair lane_start(const DevNet& n, int p, int sec, int g0, int g1, bool own, int team,
                                               int member) {
  LanePair s{};
  s.g = g0 + team;
  s.k = own ? 0 : member;
  lane_settle(n, s, p, sec, g1, own);
  return s;
}

__device__ __forceinline__ LanePair lane_next(const DevNet& n, const LanePair& s, int p, int sec, int g1, int m,
                                              bool own) {
  LanePair r = s;
  if (!s.valid) return r;
  r.k = s.k + m;
  if (r.k >= s.nb) {
    r.valid = false;
    if (own) {
      r.g = s.g + kWideWaves;
      r.k = 0;
      lane_settle(n, r, p, sec, g1, true);
    }
  }
  return r;
}

// A pair past the wave's last one loads the array's first batch (never
// delivered); the array holds at least one batch (its slack).
__device__ __forceinline__ void lane_load(const DevNet& n, const LanePair& s, int lane, uint32_t (&r)[kLaneU]) {
  const uint32_t* src = n.lrecs + (s.valid ? s.beg + s.k * (64 * kLaneU) : 0) + lane;
#pragma unroll
  for (int u = 0; u < kLaneU; ++u) r[u] = src[u * 64];
}

// One wave's walk over the lane records of section `sec` of phase p (see
// wide_range): no barrier, three record buffers in rotation keep two batches
// in flight while one is delivered (no buffer is copied: a copy would wait
// for its load).  A lane sums the weight numerators k of its active records
// as an integer; DUAL (records of delay >= 2 in the first kernel of a step
// pair) also sums, into isum2, the records whose source spiked one step
// later: the word one staged row below.  An owned group's sums go to its
// LDS rows (gacc, gacc2) when the walk leaves it; a team member keeps its
// share in isum / isum2.
template <bool DUAL>
__device__ __forceinline__ void lane_walk(const DevNet& n, int p, int sec, int g0, int g1, bool own, int team,
                                          int member, int m, int lane, const char* ring_bytes, uint32_t row_bytes,
                                          float* gacc, float* gacc2, int& isum, int& isum2) {
  LanePair s0 = lane_start(n, p, sec, g0, g1, own, team, member);
  LanePair s1 = lane_next(n, s0, p, sec, g1, m, own), s2 = lane_next(n, s1, p, sec, g1, m, own);
  uint32_t b0[kLaneU], b1[kLaneU], b2[kLaneU];
  lane_load(n, s0, lane, b0);
  lane_load(n, s1, lane, b1);
  lane_load(n, s2, lane, b2);
  auto body = [&](const LanePair& sc, const uint32_t (&cur)[kLaneU], const LanePair& sn) -> bool {
    if (!sc.valid) return false;
    auto deliver = [&](uint32_t c) {
      const uint32_t off = (c >> 5) & (kLaneMaxOffset - 1u);
      const int k = static_cast<int>(c) >> 24;
      const uint32_t word = *reinterpret_cast<const uint32_t*>(ring_bytes + off);
      // all ones when the source spiked (the bit sign-extended), else 0
      // (v_bfe reads only the offset's low 5 bits: the source's bit)
      isum += __builtin_amdgcn_sbfe(static_cast<int>(word), c, 1u) & k;
      if constexpr (DUAL) {  // every record here lies in row 1 or below: off >= row_bytes
        const uint32_t word2 = *reinterpret_cast<const uint32_t*>(ring_bytes + (off - row_bytes));
        isum2 += __builtin_amdgcn_sbfe(static_cast<int>(word2), c, 1u) & k;
      }
    };
    const int rows_left = (sc.end - sc.beg) / 64 - sc.k * kLaneU;  // uniform
    if (rows_left >= kLaneU) {
#pragma unroll
      for (int u = 0; u < kLaneU; ++u) deliver(cur[u]);
    } else {  // the section's last batch
#pragma unroll
      for (int u = 0; u < kLaneU; ++u)
        if (u < rows_left) deliver(cur[u]);
    }
    if (own && (!sn.valid || sn.g != sc.g)) {  // an owned group: this wave is its only contributor
      gacc[(sc.g - g0) * kGroup + lane] += static_cast<float>(isum) * n.lscale;
      isum = 0;
      if constexpr (DUAL) {
        gacc2[(sc.g - g0) * kGroup + lane] += static_cast<float>(isum2) * n.lscale;
        isum2 = 0;
      }
    }
    return sn.valid;
  };
  for (;;) {
    if (!body(s0, b0, s1)) break;
    const LanePair s3 = lane_next(n, s2, p, sec, g1, m, own);
    lane_load(n, s3, lane, b0);
    if (!body(s1, b1, s2)) break;
    const LanePair s4 = lane_next(n, s3, p, sec, g1, m, own);
    lane_load(n, s4, lane, b1);
    if (!body(s2, b2, s3)) break;
    const LanePair s5 = lane_next(n, s4, p, sec, g1, m, own);
    lane_load(n, s5, lane, b2);
    s0 = s3;
    s1 = s4;
    s2 = s5;
  }
}

// FALLBACK: no delay phases and more delays than staged rows; delays above
// the staged rows read the raster in memory.
// NPW: groups one wave updates at most (1 when a workgroup has <= 16).
// LANE: lane records (n.lrecs, n.lgptr, n.lwsec); never with FALLBACK.
// MODE 0: step t.  MODE 1 and 2 (LANE only): steps t and t + 1 of a step
// pair.  MODE 1 delivers step t and, from the same records of delay >= 2
// (their sources' words one staged row below), the input of step t + 1 from
// those delays, which it leaves in n.held; MODE 2, launched for step t + 1,
// adds the delay-1 records to n.held and updates.  A record of delay d >= 2
// is then read once for the two steps.
// Row q of a phase (first delay dbase + 1) holds the history of step
// t - dbase - q, at LDS row q - 1 + shift: rows q = 1 .. rows always, q = 0
// for MODE 1 in phases p >= 1.  shift = 1 (whenever lane records exist) also
// keeps the second step's sums and team slots; shift = 0 only when they and
// a second row do not fit (then LDS holds one step's sums).
template <bool FALLBACK, int NPW, bool LANE, int MODE>
__global__ __launch_bounds__(kWideThreads) void k_step_wide(const DevNet n, int t, int Dl, int P, int shift) {
  constexpr int U = kWideU;
  static_assert(MODE == 0 || (LANE && !FALLBACK), "step pairs run on lane records");
  extern __shared__ __align__(16) uint32_t smem[];
  const int b = blockIdx.y;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: the walk state lives in scalars
  const int W32 = 2 * n.G;
  const size_t rstride = static_cast<size_t>(n.B) * n.G;
  const uint64_t* hist = n.raster + static_cast<size_t>(b) * n.G;
  const int g0 = static_cast<int>(static_cast<int64_t>(n.G) * blockIdx.x / gridDim.x);
  const int g1 = static_cast<int>(static_cast<int64_t>(n.G) * (blockIdx.x + 1) / gridDim.x);
  const int ng = g1 - g0;
  // with fewer groups than waves, group q gets waves ceil(16q/ng) ..
  // ceil(16(q+1)/ng) - 1 (2 or 3 waves for 7 groups); else every wave owns
  const bool own = ng >= kWideWaves;
  const int team = own ? wave : wave * ng / kWideWaves;
  const int tfirst = own ? wave : (team * kWideWaves + ng - 1) / ng;
  const int m = own ? 1 : (team + 1 == ng ? kWideWaves : ((team + 1) * kWideWaves + ng - 1) / ng) - tfirst;
  const int member = wave - tfirst;
  // LDS: the staged rows first (a lane record's offset is an LDS address),
  // then the groups' sums of the two steps and the team slots (with shift =
  // 0, one step's: the second step's names alias the first's, unused)
  uint32_t* ring = smem;                                                                   // [Dl + shift][W32]
  float* gacc = reinterpret_cast<float*>(smem + static_cast<size_t>(Dl + shift) * W32);   // [g1 - g0][64]
  float* gacc2 = gacc + static_cast<size_t>(shift) * ng * kGroup;                          // [g1 - g0][64]
  float(*part)[kGroup] = reinterpret_cast<float(*)[kGroup]>(gacc2 + static_cast<size_t>(ng) * kGroup);  // [16][64]
  float(*part2)[kGroup] = part + shift * kWideWaves;                                                  // [16][64]

  // neuron state of the groups this wave updates, loaded now, used last
  float V[NPW], th[NPW], lam[NPW], rs[NPW], amp[NPW];
  int ref[NPW], R[NPW];
  uint64_t ew[NPW];
#pragma unroll
  for (int i = 0; i < NPW; ++i) {
    const int g = g0 + wave + i * kWideWaves;
    V[i] = th[i] = lam[i] = rs[i] = amp[i] = 0.f;
    ref[i] = R[i] = 0;
    ew[i] = 0;
    if (g < g1) {
      const int j = g * kGroup + lane;
      const size_t sj = static_cast<size_t>(b) * n.Npad + j;
      V[i] = n.V[sj];
      ref[i] = n.ref[sj];
      th[i] = n.theta[j];
      lam[i] = n.leak[j];
      rs[i] = n.reset[j];
      amp[i] = n.amp[j];
      R[i] = n.refr[j];
      ew[i] = n.ext[row_word(n, t, b, g)];
    }
  }
  for (int i = tid; i < ng * kGroup; i += kWideThreads) {
    if constexpr (MODE == 2)  // the input of this step gathered by the pair's first kernel
      gacc[i] = n.held[static_cast<size_t>(b) * n.Npad + static_cast<size_t>(g0) * kGroup + i];
    else
      gacc[i] = 0.f;
    if constexpr (MODE == 1) gacc2[i] = 0.f;
  }

  const int phases = MODE == 2 ? 1 : P;  // MODE 2: the delay-1 records of phase 0 only
  for (int p = 0; p < phases; ++p) {
    const int dbase = p * Dl;  // the phase's delays are dbase + 1 .. dbase + Dl
    const int rows = MODE == 2 ? 1 : min(Dl, n.D - dbase);
    const int q0 = MODE == 1 && p > 0 ? 0 : 1;  // first staged row
    // stage the phase's rows: every load of a round is issued before its
    // stores, so a round costs one memory latency, not one per word.  Word
    // i of the phase is (row q0 + i / G, word i mod G); one division per
    // round, then the next word of the thread (1024 further) by adding and
    // carrying, and a word goes to LDS as one 8-byte store.
    uint64_t* ring64 = reinterpret_cast<uint64_t*>(ring);
    const int staged = (rows + 1 - q0) * n.G;  // words
    const int lds_end = (rows + 1) * n.G;
    const int lds_skip = (1 - shift) * n.G;  // row q at LDS word (q - 1 + shift) G; q >= 1 when shift = 0
    for (int base = 0; base < staged; base += kWideThreads * kWideStage) {
      uint64_t v[kWideStage];
      int r = (base + tid) / n.G, w = base + tid - r * n.G;
      int at[kWideStage];  // the word's index q G + w in the staged rows
#pragma unroll
      for (int q = 0; q < kWideStage; ++q) {
        if (q > 0) {
          w += kWideThreads;
          while (w >= n.G) {
            w -= n.G;
            ++r;
          }
        }
        const int row = q0 + r;
        const int ts = t - dbase - row;
        at[q] = row * n.G + w;
        v[q] = (at[q] < lds_end && ts >= 0) ? hist[static_cast<size_t>(ts) * rstride + w] : 0ull;
      }
#pragma unroll
      for (int q = 0; q < kWideStage; ++q)
        if (at[q] < lds_end) ring64[at[q] - lds_skip] = v[q];
    }
    __syncthreads();

    float tsum = 0.f, tsum2 = 0.f;  // a team member's share of its group's sums
    if constexpr (LANE) {
      const char* ring_bytes = reinterpret_cast<const char*>(ring);
      const uint32_t row_bytes = static_cast<uint32_t>(W32) * sizeof(uint32_t);
      int isum = 0, isum2 = 0;
      if constexpr (MODE == 0) {
        lane_walk<false>(n, p, 0, g0, g1, own, team, member, m, lane, ring_bytes, row_bytes, gacc, gacc2, isum, isum2);
      } else if constexpr (MODE == 1) {
        lane_walk<true>(n, p, 1, g0, g1, own, team, member, m, lane, ring_bytes, row_bytes, gacc, gacc2, isum, isum2);
        if (p == 0)  // the delay-1 records: step t only
          lane_walk<false>(n, 0, 2, g0, g1, own, team, member, m, lane, ring_bytes, row_bytes, gacc, gacc2, isum,
                           isum2);
      } else {
        lane_walk<false>(n, 0, 2, g0, g1, own, team, member, m, lane, ring_bytes, row_bytes, gacc, gacc2, isum, isum2);
      }
      tsum = static_cast<float>(isum) * n.lscale;
      tsum2 = static_cast<float>(isum2) * n.lscale;
    } else {
      const uint32_t* ring1 = ring + static_cast<size_t>(shift) * W32;  // row q = 1: the phase's first delay
      // this wave's (group, batch) walk: no barrier until the phase ends, three
      // record buffers in rotation keep two batches in flight while one is
      // delivered (no buffer is copied: a copy would wait for its load)
      WidePair s0 = wide_start(n, p, g0, g1, own, team, member);
      WidePair s1 = wide_next(n, s0, p, g1, m, own), s2 = wide_next(n, s1, p, g1, m, own);
      Rec b0[U], b1[U], b2[U];
      wide_load_pair(n, s0, lane, b0);
      wide_load_pair(n, s1, lane, b1);
      wide_load_pair(n, s2, lane, b2);
      float sum = 0.f;
      // delivers the batch of pair sc; an owned group's sum is added to its
      // row when the walk leaves it; false when sc was the wave's last pair
      auto body = [&](const WidePair& sc, const Rec (&cur)[U], const WidePair& sn) -> bool {
        if (!sc.valid) return false;
        float* acc_g = gacc + (sc.g - g0) * kGroup;
        const int first = wide_first(sc) + lane;
        uint32_t bit[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int d = static_cast<int>((cur[u].meta >> 20) & 63u) + 1;
          const uint32_t pre = cur[u].meta & 0xFFFFFu;
          const bool valid = first + u * 64 < sc.end;
          const int r = d - dbase - 1;  // row of the phase's staged rows, from row 1
          if (!FALLBACK) {
            // every record of the phase lies in its rows; a masked one may not
            const uint32_t rc = static_cast<uint32_t>(min(max(r, 0), rows - 1));
            bit[u] = (ring1[__umul24(rc, static_cast<uint32_t>(W32)) + (pre >> 5)] >> (pre & 31u)) &
                     static_cast<uint32_t>(valid);
          } else if (r < rows) {
            bit[u] = (ring1[__umul24(static_cast<uint32_t>(r), static_cast<uint32_t>(W32)) + (pre >> 5)] >> (pre & 31u)) &
                     static_cast<uint32_t>(valid);
          } else {  // a delay beyond the staged rows
            bit[u] = valid && t - d >= 0
                         ? static_cast<uint32_t>(hist[static_cast<size_t>(t - d) * rstride + (pre >> 6)] >> (pre & 63u)) & 1u
                         : 0u;
          }
        }
        bool other = false;  // an active overflow record of another lane's post
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t post = cur[u].meta >> 26;
          sum += (bit[u] && post == static_cast<uint32_t>(lane)) ? cur[u].w : 0.f;
          other |= bit[u] && post != static_cast<uint32_t>(lane);
        }
        if (other) {  // rare: overflow records follow the lane-owned rows
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const uint32_t post = cur[u].meta >> 26;
            if (bit[u] && post != static_cast<uint32_t>(lane)) atomicAdd(&acc_g[post], cur[u].w);
          }
        }
        if (own && (!sn.valid || sn.g != sc.g)) {  // an owned group: this wave is its only contributor
          acc_g[lane] += sum;
          sum = 0.f;
        }
        return sn.valid;
      };
      for (;;) {
        if (!body(s0, b0, s1)) break;
        const WidePair s3 = wide_next(n, s2, p, g1, m, own);
        wide_load_pair(n, s3, lane, b0);
        if (!body(s1, b1, s2)) break;
        const WidePair s4 = wide_next(n, s3, p, g1, m, own);
        wide_load_pair(n, s4, lane, b1);
        if (!body(s2, b2, s3)) break;
        const WidePair s5 = wide_next(n, s4, p, g1, m, own);
        wide_load_pair(n, s5, lane, b2);
        s0 = s3;
        s1 = s4;
        s2 = s5;
      }
      tsum = sum;
    }
    if (!own) {  // a team of m waves per group: the sums meet in LDS
      part[wave][lane] = tsum;
      if (MODE == 1) part2[wave][lane] = tsum2;
      __syncthreads();
      if (member == 0) {
        float a = gacc[team * kGroup + lane];
        for (int i = 0; i < m; ++i) a += part[tfirst + i][lane];
        gacc[team * kGroup + lane] = a;
        if (MODE == 1) {
          float a2 = gacc2[team * kGroup + lane];
          for (int i = 0; i < m; ++i) a2 += part2[tfirst + i][lane];
          gacc2[team * kGroup + lane] = a2;
        }
      }
    }
    __syncthreads();  // every lookup of this phase done, every group row complete
  }

#pragma unroll
  for (int i = 0; i < NPW; ++i) {
    const int g = g0 + wave + i * kWideWaves;
    if (g < g1) {  // uniform per wave
      const float syn = gacc[(g - g0) * kGroup + lane];
      const bool s = lif_update(V[i], ref[i], syn, (ew[i] >> lane) & 1ull, th[i], lam[i], rs[i], amp[i], R[i]);
      const uint64_t sw = __ballot(s);
      const int j = g * kGroup + lane;
      const size_t sj = static_cast<size_t>(b) * n.Npad + j;
      n.V[sj] = V[i];
      n.ref[sj] = static_cast<uint8_t>(ref[i]);
      if (lane == 0) n.raster[row_word(n, t, b, g)] = sw;
      if (MODE == 1) n.held[sj] = gacc2[(g - g0) * kGroup + lane];
    }
  }
}

bool wide_net(const DevNet& n) {
  return static_cast<size_t>(n.D) * 2 * n.G * sizeof(uint32_t) > kStepRingLimitWide;
}

WidePlan wide_plan(const DevNet& n, int cus) {
  WidePlan w;
  w.grid = std::max(1, std::min(cus, n.G));
  w.gpw = (n.G + w.grid - 1) / w.grid;
  if (w.gpw > kWideNpw * kWideWaves) {  // more groups than the waves can update: more workgroups
    w.gpw = kWideNpw * kWideWaves;
    w.grid = (n.G + w.gpw - 1) / w.gpw;
  }
  const size_t row = static_cast<size_t>(2 * n.G) * sizeof(uint32_t);
  const size_t sums = static_cast<size_t>(w.gpw) * kGroup * sizeof(float);
  // step pairs: two steps' sums and team slots and one row beside the
  // phase's Dl for the row of one step later, when two rows fit with them;
  // else one step's sums
  const size_t dual = (kWideLdsLimit - kWideStaticLds - 2 * (kWidePartLds + sums)) / row;
  const size_t single = (kWideLdsLimit - kWideStaticLds - kWidePartLds - sums) / row;
  w.shift = dual >= 2 ? 1 : 0;
  w.Dl = static_cast<int>(std::min<size_t>(w.shift ? dual - 1 : single, static_cast<size_t>(n.D)));
  w.P = w.Dl > 0 ? (n.D + w.Dl - 1) / w.Dl : 0;
  if (w.P > kWideMaxPhases) w.P = 1;  // too many phases: delays above Dl read memory
  return w;
}

static size_t wide_lds(const DevNet& n, const WidePlan& w, int Dl) {
  return static_cast<size_t>(Dl + w.shift) * 2 * n.G * sizeof(uint32_t) +
         (1 + w.shift) * (static_cast<size_t>(w.gpw) * kGroup * sizeof(float) + kWidePartLds);
}

// Phases come from the layout (n.phases, n.phase_rows); a layout without
// phases runs with as many rows as fit.
static int wide_rows_of(const DevNet& n, const WidePlan& w) { return n.phases > 1 ? n.phase_rows : w.Dl; }

hipError_t prepare_wide_kernel(const DevNet& n, int cus) {
  const WidePlan w = wide_plan(n, cus);
  const int Dl = wide_rows_of(n, w);
  if (Dl < 1 || wide_lds(n, w, Dl) + kWideStaticLds > kWideLdsLimit) return hipErrorInvalidValue;
  const int bytes = static_cast<int>(wide_lds(n, w, Dl));
  const void* fns[] = {reinterpret_cast<const void*>(&k_step_wide<false, 1, false, 0>),
                       reinterpret_cast<const void*>(&k_step_wide<true, 1, false, 0>),
                       reinterpret_cast<const void*>(&k_step_wide<false, kWideNpw, false, 0>),
                       reinterpret_cast<const void*>(&k_step_wide<true, kWideNpw, false, 0>),
                       reinterpret_cast<const void*>(&k_step_wide<false, 1, true, 0>),
                       reinterpret_cast<const void*>(&k_step_wide<false, kWideNpw, true, 0>),
                       reinterpret_cast<const void*>(&k_step_wide<false, 1, true, 1>),
                       reinterpret_cast<const void*>(&k_step_wide<false, kWideNpw, true, 1>),
                       reinterpret_cast<const void*>(&k_step_wide<false, 1, true, 2>),
                       reinterpret_cast<const void*>(&k_step_wide<false, kWideNpw, true, 2>)};
  for (const void* f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_step_wide(const DevNet& n, int32_t t, int cus, hipStream_t s) {
  const WidePlan w = wide_plan(n, cus);
  const int Dl = wide_rows_of(n, w);
  const int P = n.phases > 1 ? n.phases : 1;
  if (Dl < 1 || wide_lds(n, w, Dl) + kWideStaticLds > kWideLdsLimit) return hipErrorInvalidValue;
  if (P > 1 && Dl * P < n.D) return hipErrorInvalidValue;  // phases must cover every delay
  const bool fallback = P == 1 && Dl < n.D;
  const dim3 grid(w.grid, n.B), block(kWideThreads);
  const size_t lds = wide_lds(n, w, Dl);
  // lane records address the staged rows: only when every delay is staged
  // (from LDS row 1)
  const bool lane = n.lrecs != nullptr && !fallback && w.shift == 1;
#define SN_WIDE(FB, NPW, LN) \
  hipLaunchKernelGGL((k_step_wide<FB, NPW, LN, 0>), grid, block, lds, s, n, t, Dl, P, w.shift)
  const int key = (fallback ? 1 : 0) + (w.gpw <= kWideWaves ? 0 : 2) + (lane ? 4 : 0);
  switch (key) {
    case 0: SN_WIDE(false, 1, false); break;
    case 1: SN_WIDE(true, 1, false); break;
    case 2: SN_WIDE(false, kWideNpw, false); break;
    case 3: SN_WIDE(true, kWideNpw, false); break;
    case 4: SN_WIDE(false, 1, true); break;
    default: SN_WIDE(false, kWideNpw, true); break;
  }
#undef SN_WIDE
  return hipGetLastError();
}

bool wide_pairs(const DevNet& n, int cus) {
  if (!n.lrecs || !n.lgsplit || !n.held) return false;
  const WidePlan w = wide_plan(n, cus);
  const int Dl = wide_rows_of(n, w);
  const int P = n.phases > 1 ? n.phases : 1;
  return Dl >= 1 && w.shift == 1 && !(P == 1 && Dl < n.D) && wide_lds(n, w, Dl) + kWideStaticLds <= kWideLdsLimit;
}

hipError_t launch_pair_wide(const DevNet& n, int32_t t, int cus, hipStream_t s) {
  if (!wide_pairs(n, cus)) return hipErrorInvalidValue;
  const WidePlan w = wide_plan(n, cus);
  const int Dl = wide_rows_of(n, w);
  const int P = n.phases > 1 ? n.phases : 1;
  if (P > 1 && Dl * P < n.D) return hipErrorInvalidValue;  // phases must cover every delay
  const dim3 grid(w.grid, n.B), block(kWideThreads);
  const size_t lds = wide_lds(n, w, Dl);
  if (w.gpw <= kWideWaves) {
    hipLaunchKernelGGL((k_step_wide<false, 1, true, 1>), grid, block, lds, s, n, t, Dl, P, 1);
    hipLaunchKernelGGL((k_step_wide<false, 1, true, 2>), grid, block, lds, s, n, t + 1, Dl, P, 1);
  } else {
    hipLaunchKernelGGL((k_step_wide<false, kWideNpw, true, 1>), grid, block, lds, s, n, t, Dl, P, 1);
    hipLaunchKernelGGL((k_step_wide<false, kWideNpw, true, 2>), grid, block, lds, s, n, t + 1, Dl, P, 1);
  }
  return hipGetLastError();
}

static hipError_t device_cus_wide(int& cus) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return e;
}

// the per-step path of a net runs this kernel exactly when wide_net holds
bool step_pairs(const DevNet& n) {
  if (!wide_net(n)) return false;
  int cus = 0;
  if (device_cus_wide(cus) != hipSuccess) return false;
  return wide_pairs(n, cus);
}

hipError_t launch_step_pair(const DevNet& n, int32_t t, hipStream_t s) {
  int cus = 0;
  const hipError_t e = device_cus_wide(cus);
  return e != hipSuccess ? e : launch_pair_wide(n, t, cus, s);
}

}  // namespace snmi
