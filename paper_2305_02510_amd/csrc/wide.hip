// Per-step pull delivery for nets whose spike history does not fit in LDS
// (N = 100,000 with delays up to 16: 16 rows of 100,000 bits = 200 KB), the
// synaptic input of §2.1's update summed over the pull records of every
// post-neuron group, followed by the fused neuron update.
//
// One launch per step, or K launches per block of K steps (see MODE below:
// records of delay >= K read once for K steps).  Workgroup (w, b) owns the
// contiguous groups
// [g0, g1) of trial b.  The delays are cut into phases of Dl delays (Dl =
// as many history rows as fit in LDS beside the sums); the layout orders the
// delay >= 2 records of every group by phase (phases P-1 .. 1, then phase 0
// running on into the delay-1 records; lane layouts: the delays >= K, then a
// section for each delay K - 1 .. 1).  For each phase the workgroup copies
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
// the short delays in sections of their own after the phases)
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
// wsec[p - 1]); phase 0 runs from wsec[0] to the group's end (the short
// sections included).  Without phases: all records of the group.  LANE: the
// offsets of the lane-record layout, and the section kind: kSecPhase as
// above; kSecLong phase p's delays >= block (phase 0 ends where the short
// sections begin); kSecShort the section of delay d < block; kSecFrom the
// sections of delays d .. 1 (from the section of delay d to the group's end).
constexpr int kSecPhase = 0, kSecLong = 1, kSecShort = 2, kSecFrom = 3;
template <bool LANE>
__device__ __forceinline__ void wide_range(const DevNet& n, int g, int p, int kind, int d, int& beg, int& end) {
  if (!LANE) {
    if (n.phases <= 1) {
      beg = n.gptr[g];
      end = n.gptr[g + 1];
      return;
    }
    const int32_t* ws = n.wsec + static_cast<size_t>(g) * n.phases;
    beg = ws[p];
    end = p == 0 ? n.gptr[g + 1] : ws[p - 1];
    return;
  }
  const int32_t* lg = n.lgptr;
  const int32_t* ss = n.lsec + static_cast<size_t>(g) * (n.lblock - 1);  // ss[d - 1]: section of delay d
  if (kind == kSecShort || kind == kSecFrom) {
    beg = ss[d - 1];
    end = kind == kSecFrom || d == 1 ? lg[g + 1] : ss[d - 2];
    return;
  }
  const int32_t last = kind == kSecLong ? ss[n.lblock - 2] : lg[g + 1];  // end of phase 0
  if (n.phases <= 1) {
    beg = lg[g];
    end = last;
    return;
  }
  const int32_t* ws = n.lwsec + static_cast<size_t>(g) * n.phases;
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
  wide_range<false>(n, s.g, p, kSecPhase, 0, s.beg, s.end);
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

// sec = kind * 64 + d (see wide_range)
__device__ __forceinline__ void lane_enter(const DevNet& n, LanePair& s, int p, int sec) {
  wide_range<true>(n, s.g, p, sec >> 6, sec & 63, s.beg, s.end);
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
// lane_enter): no barrier, three record buffers in rotation keep two batches
// in flight while one is delivered (no buffer is copied: a copy would wait
// for its load).  A lane sums the weight numerators k of its active records
// as integers: for C steps of a block at once (the first kernel of a block,
// records of delay >= C), sum j from the source word j staged rows below the
// record's word, j = 0 .. C - 1, after skipping `skip` bytes of rows (the
// later kernels of a block).  An owned group's sums go to its LDS rows (sum
// j at gacc + j * gstride) when the walk leaves it; a team member keeps its
// share in isum.
template <int C, int NS>
__device__ __forceinline__ void lane_walk(const DevNet& n, int p, int sec, int g0, int g1, bool own, int team,
                                          int member, int m, int lane, const char* ring_bytes, uint32_t row_bytes,
                                          uint32_t skip, float* gacc, int gstride, int (&isum)[NS]) {
  static_assert(C <= NS, "one sum per step");
  LanePair s0 = lane_start(n, p, sec, g0, g1, own, team, member);
  LanePair s1 = lane_next(n, s0, p, sec, g1, m, own), s2 = lane_next(n, s1, p, sec, g1, m, own);
  uint32_t b0[kLaneU], b1[kLaneU], b2[kLaneU];
  lane_load(n, s0, lane, b0);
  lane_load(n, s1, lane, b1);
  lane_load(n, s2, lane, b2);
  auto body = [&](const LanePair& sc, const uint32_t (&cur)[kLaneU], const LanePair& sn) -> bool {
    if (!sc.valid) return false;
    auto deliver = [&](uint32_t c) {
      // every record of these sections lies at least skip + (C - 1) rows
      // below row 0 (its row is (d - 1) mod Dl + block - 1)
      const uint32_t off = ((c >> 5) & (kLaneMaxOffset - 1u)) - skip;
      const int k = static_cast<int>(c) >> 24;
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const uint32_t word = *reinterpret_cast<const uint32_t*>(ring_bytes + (off - j * row_bytes));
        // all ones when the source spiked (the bit sign-extended), else 0
        // (v_bfe reads only the offset's low 5 bits: the source's bit)
        isum[j] += __builtin_amdgcn_sbfe(static_cast<int>(word), c, 1u) & k;
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
#pragma unroll
      for (int j = 0; j < C; ++j) {
        gacc[j * gstride + (sc.g - g0) * kGroup + lane] += static_cast<float>(isum[j]) * n.lscale;
        isum[j] = 0;
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
// LANE: lane records (n.lrecs, n.lgptr, n.lwsec, n.lsec); never with FALLBACK.
// MODE 0: step t.  MODE 1 and 2 (LANE only): a block of KT = n.lblock steps
// t .. t + KT - 1.  The input of step t + i through a synapse of delay d > i
// depends only on spikes up to step t - 1.  MODE 1 streams every record once:
// a record of delay d adds into the sums of steps t .. t + min(d, KT) - 1
// (its source words 0 .. min(d, KT) - 1 staged rows below its word); it
// updates step t and leaves the sums of steps t + 1 .. in n.held.  MODE 2,
// launched for i = 1 .. KT - 1 in turn, adds the records of delays 1 .. i to
// step t + i's held sum and updates step t + i.
// LDS row r of a phase (first delay dbase + 1) holds the history of step
// t - dbase - r + shift - 1 (shift = block - 1 extra rows, 0 when a single
// history row fills the LDS): MODE 0 stages the rows of steps t - dbase - 1
// .. t - dbase - rows; MODE 1 in phases p >= 1 also the shift later ones
// (all before step t while Dl >= block - 1); MODE 2 (phase 0) the rows of
// steps t .. t + i - 1.  After the rows: the sums of the block's steps
// [shift + 1][g1 - g0][64], then the team slots [shift + 1][16][64].
template <bool FALLBACK, int NPW, bool LANE, int MODE, int KT>
__global__ __launch_bounds__(kWideThreads) void k_step_wide(const DevNet n, int t, int Dl, int P, int shift, int ib) {
  constexpr int U = kWideU;
  constexpr int NS = MODE == 1 ? KT : 1;  // sums per lane
  static_assert(MODE == 0 || (LANE && !FALLBACK), "blocks of steps run on lane records");
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
  const int tu = MODE == 2 ? t + ib : t;  // the step this kernel updates
  // with fewer groups than waves, group q gets waves ceil(16q/ng) ..
  // ceil(16(q+1)/ng) - 1 (2 or 3 waves for 7 groups); else every wave owns
  const bool own = ng >= kWideWaves;
  const int team = own ? wave : wave * ng / kWideWaves;
  const int tfirst = own ? wave : (team * kWideWaves + ng - 1) / ng;
  const int m = own ? 1 : (team + 1 == ng ? kWideWaves : ((team + 1) * kWideWaves + ng - 1) / ng) - tfirst;
  const int member = wave - tfirst;
  // LDS: the staged rows first (a lane record's offset is an LDS address)
  uint32_t* ring = smem;                                                                   // [Dl + shift][W32]
  float* gacc = reinterpret_cast<float*>(smem + static_cast<size_t>(Dl + shift) * W32);   // [shift + 1][ng][64]
  const int gstride = ng * kGroup;
  float* part = gacc + static_cast<size_t>(shift + 1) * gstride;                           // [shift + 1][16][64]
  constexpr int pstride = kWideWaves * kGroup;

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
      ew[i] = n.ext[row_word(n, tu, b, g)];
    }
  }
  const size_t hstride = static_cast<size_t>(n.B) * n.Npad;  // held sums of one step
  const size_t hbase = static_cast<size_t>(b) * n.Npad + static_cast<size_t>(g0) * kGroup;
  for (int i = tid; i < gstride; i += kWideThreads) {
    if constexpr (MODE == 2)  // the input of this step gathered by the block's first kernel
      gacc[i] = n.held[(ib - 1) * hstride + hbase + i];
    else
      gacc[i] = 0.f;
    if constexpr (MODE == 1) {
#pragma unroll
      for (int j = 1; j < KT; ++j) gacc[j * gstride + i] = 0.f;
    }
  }

  const int phases = MODE == 2 ? 1 : P;  // MODE 2: the short delays of phase 0 only
  for (int p = 0; p < phases; ++p) {
    const int dbase = p * Dl;  // the phase's delays are dbase + 1 .. dbase + Dl
    // rows q0 .. qhi, row q holding step t - dbase - q at LDS row q + shift - 1
    const int q0 = MODE == 2 ? 1 - ib : MODE == 1 && p > 0 ? 1 - shift : 1;
    const int qhi = MODE == 2 ? 0 : min(Dl, n.D - dbase);
    const int rows = qhi;  // the phase's delays staged (8-byte path)
    // stage the phase's rows: every load of a round is issued before its
    // stores, so a round costs one memory latency, not one per word.  Word
    // i of the phase is (row q0 + i / G, word i mod G); one division per
    // round, then the next word of the thread (1024 further) by adding and
    // carrying, and a word goes to LDS as one 8-byte store.
    uint64_t* ring64 = reinterpret_cast<uint64_t*>(ring);
    const int nrows = qhi - q0 + 1;
    const int nwords = nrows * n.G;
    const int at0 = (q0 + shift - 1) * n.G;  // LDS word of row q0 (>= 0)
    for (int base = 0; base < nwords; base += kWideThreads * kWideStage) {
      uint64_t v[kWideStage];
      int r = (base + tid) / n.G, w = base + tid - r * n.G;
#pragma unroll
      for (int q = 0; q < kWideStage; ++q) {
        if (q > 0) {
          w += kWideThreads;
          while (w >= n.G) {
            w -= n.G;
            ++r;
          }
        }
        const int ts = t - dbase - (q0 + r);
        v[q] = (r < nrows && ts >= 0) ? hist[static_cast<size_t>(ts) * rstride + w] : 0ull;
      }
#pragma unroll
      for (int q = 0; q < kWideStage; ++q) {
        const int i = base + tid + q * kWideThreads;
        if (i < nwords) ring64[at0 + i] = v[q];
      }
    }
    __syncthreads();

    float tsum[NS];  // a team member's share of its group's sums
#pragma unroll
    for (int j = 0; j < NS; ++j) tsum[j] = 0.f;
    if constexpr (LANE) {
      const char* ring_bytes = reinterpret_cast<const char*>(ring);
      const uint32_t row_bytes = static_cast<uint32_t>(W32) * sizeof(uint32_t);
      int isum[NS];
#pragma unroll
      for (int j = 0; j < NS; ++j) isum[j] = 0;
      constexpr int kPhase = kSecPhase << 6, kLong = kSecLong << 6, kShort = kSecShort << 6, kFrom = kSecFrom << 6;
      if constexpr (MODE == 0) {
        lane_walk<1>(n, p, kPhase, g0, g1, own, team, member, m, lane, ring_bytes, row_bytes, 0u, gacc, gstride, isum);
      } else if constexpr (MODE == 1) {
        lane_walk<KT>(n, p, kLong, g0, g1, own, team, member, m, lane, ring_bytes, row_bytes, 0u, gacc, gstride, isum);
        if (p == 0) {  // the short delays d < KT: steps t .. t + d - 1
          if constexpr (KT > 3)
            lane_walk<3>(n, 0, kShort | 3, g0, g1, own, team, member, m, lane, ring_bytes, row_bytes, 0u, gacc, gstride,
                         isum);
          if constexpr (KT > 2)
            lane_walk<2>(n, 0, kShort | 2, g0, g1, own, team, member, m, lane, ring_bytes, row_bytes, 0u, gacc, gstride,
                         isum);
          lane_walk<1>(n, 0, kShort | 1, g0, g1, own, team, member, m, lane, ring_bytes, row_bytes, 0u, gacc, gstride,
                       isum);
        }
      } else {  // delays 1 .. ib for step t + ib: their words ib rows up
        lane_walk<1>(n, 0, kFrom | ib, g0, g1, own, team, member, m, lane, ring_bytes, row_bytes,
                     static_cast<uint32_t>(ib) * row_bytes, gacc, gstride, isum);
      }
#pragma unroll
      for (int j = 0; j < NS; ++j) tsum[j] = static_cast<float>(isum[j]) * n.lscale;
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
          const int r = d - dbase - 1;  // row of the phase's staged rows, from row q = 1
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
      tsum[0] = sum;
    }
    if (!own) {  // a team of m waves per group: the sums meet in LDS
#pragma unroll
      for (int j = 0; j < NS; ++j) part[j * pstride + wave * kGroup + lane] = tsum[j];
      __syncthreads();
      if (member == 0) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
          float a = gacc[j * gstride + team * kGroup + lane];
          for (int i = 0; i < m; ++i) a += part[j * pstride + (tfirst + i) * kGroup + lane];
          gacc[j * gstride + team * kGroup + lane] = a;
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
      if (lane == 0) n.raster[row_word(n, tu, b, g)] = sw;
      if constexpr (MODE == 1) {
#pragma unroll
        for (int q = 1; q < KT; ++q) n.held[(q - 1) * hstride + sj] = gacc[q * gstride + (g - g0) * kGroup + lane];
      }
    }
  }
}

bool wide_net(const DevNet& n) {
  return static_cast<size_t>(n.D) * 2 * n.G * sizeof(uint32_t) > kStepRingLimitWide;
}

// Steps per block of the lane layout: the largest of 4, 2 whose block - 1
// extra rows and block sets of sums and team slots fit beside Dl >= 1 staged
// rows, where the phases (if any) are at most kWideMaxPhases and at least
// block - 1 delays each (a later phase's rows of steps t .. t + block - 2 must
// all lie before step t); else 1 (no extra rows, no lane records).
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
  for (int blk : {4, 2, 1}) {
    const size_t fixed = kWideStaticLds + static_cast<size_t>(blk) * (kWidePartLds + sums);
    const size_t fit = fixed < kWideLdsLimit ? (kWideLdsLimit - fixed) / row : 0;
    const int Dl = static_cast<int>(std::min<size_t>(fit >= static_cast<size_t>(blk) ? fit - (blk - 1) : 0,
                                                     static_cast<size_t>(n.D)));
    const int P = Dl > 0 ? (n.D + Dl - 1) / Dl : 0;
    const bool ok = blk == 1 || (Dl >= 1 && P <= kWideMaxPhases && (P == 1 || Dl >= blk - 1));
    if (!ok) continue;
    w.block = blk;
    w.shift = blk - 1;
    w.Dl = Dl;
    w.P = P > kWideMaxPhases ? 1 : P;  // too many phases: delays above Dl read memory
    break;
  }
  return w;
}

static size_t wide_lds(const DevNet& n, const WidePlan& w, int Dl) {
  return static_cast<size_t>(Dl + w.shift) * 2 * n.G * sizeof(uint32_t) +
         static_cast<size_t>(w.block) * (static_cast<size_t>(w.gpw) * kGroup * sizeof(float) + kWidePartLds);
}

// Phases come from the layout (n.phases, n.phase_rows); a layout without
// phases runs with as many rows as fit.
static int wide_rows_of(const DevNet& n, const WidePlan& w) { return n.phases > 1 ? n.phase_rows : w.Dl; }

hipError_t prepare_wide_kernel(const DevNet& n, int cus) {
  const WidePlan w = wide_plan(n, cus);
  const int Dl = wide_rows_of(n, w);
  if (Dl < 1 || wide_lds(n, w, Dl) + kWideStaticLds > kWideLdsLimit) return hipErrorInvalidValue;
  const int bytes = static_cast<int>(wide_lds(n, w, Dl));
  const void* fns[] = {reinterpret_cast<const void*>(&k_step_wide<false, 1, false, 0, 1>),
                       reinterpret_cast<const void*>(&k_step_wide<true, 1, false, 0, 1>),
                       reinterpret_cast<const void*>(&k_step_wide<false, kWideNpw, false, 0, 1>),
                       reinterpret_cast<const void*>(&k_step_wide<true, kWideNpw, false, 0, 1>),
                       reinterpret_cast<const void*>(&k_step_wide<false, 1, true, 0, 1>),
                       reinterpret_cast<const void*>(&k_step_wide<false, kWideNpw, true, 0, 1>),
                       reinterpret_cast<const void*>(&k_step_wide<false, 1, true, 1, 2>),
                       reinterpret_cast<const void*>(&k_step_wide<false, kWideNpw, true, 1, 2>),
                       reinterpret_cast<const void*>(&k_step_wide<false, 1, true, 1, 4>),
                       reinterpret_cast<const void*>(&k_step_wide<false, kWideNpw, true, 1, 4>),
                       reinterpret_cast<const void*>(&k_step_wide<false, 1, true, 2, 1>),
                       reinterpret_cast<const void*>(&k_step_wide<false, kWideNpw, true, 2, 1>)};
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
  // lane records address the staged rows: only when every delay is staged,
  // from the layout's block
  const bool lane = n.lrecs != nullptr && !fallback && w.block >= 2 && n.lblock == w.block;
#define SN_WIDE(FB, NPW, LN) \
  hipLaunchKernelGGL((k_step_wide<FB, NPW, LN, 0, 1>), grid, block, lds, s, n, t, Dl, P, w.shift, 0)
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

int wide_block(const DevNet& n, int cus) {
  if (!n.lrecs || !n.lsec || !n.held) return 1;
  const WidePlan w = wide_plan(n, cus);
  const int Dl = wide_rows_of(n, w);
  const int P = n.phases > 1 ? n.phases : 1;
  const bool ok = w.block >= 2 && n.lblock == w.block && Dl >= 1 && !(P == 1 && Dl < n.D) &&
                  (P == 1 || Dl >= w.block - 1) && wide_lds(n, w, Dl) + kWideStaticLds <= kWideLdsLimit;
  return ok ? w.block : 1;
}

hipError_t launch_block_wide(const DevNet& n, int32_t t, int cus, hipStream_t s) {
  const int blk = wide_block(n, cus);
  if (blk < 2) return hipErrorInvalidValue;
  const WidePlan w = wide_plan(n, cus);
  const int Dl = wide_rows_of(n, w);
  const int P = n.phases > 1 ? n.phases : 1;
  if (P > 1 && Dl * P < n.D) return hipErrorInvalidValue;  // phases must cover every delay
  const dim3 grid(w.grid, n.B), block(kWideThreads);
  const size_t lds = wide_lds(n, w, Dl);
  const bool one = w.gpw <= kWideWaves;
  if (blk == 4) {
    if (one) hipLaunchKernelGGL((k_step_wide<false, 1, true, 1, 4>), grid, block, lds, s, n, t, Dl, P, 3, 0);
    else hipLaunchKernelGGL((k_step_wide<false, kWideNpw, true, 1, 4>), grid, block, lds, s, n, t, Dl, P, 3, 0);
  } else {
    if (one) hipLaunchKernelGGL((k_step_wide<false, 1, true, 1, 2>), grid, block, lds, s, n, t, Dl, P, 1, 0);
    else hipLaunchKernelGGL((k_step_wide<false, kWideNpw, true, 1, 2>), grid, block, lds, s, n, t, Dl, P, 1, 0);
  }
  for (int i = 1; i < blk; ++i) {
    if (one) hipLaunchKernelGGL((k_step_wide<false, 1, true, 2, 1>), grid, block, lds, s, n, t, Dl, P, blk - 1, i);
    else hipLaunchKernelGGL((k_step_wide<false, kWideNpw, true, 2, 1>), grid, block, lds, s, n, t, Dl, P, blk - 1, i);
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
int step_block(const DevNet& n) {
  if (!wide_net(n)) return 1;
  int cus = 0;
  if (device_cus_wide(cus) != hipSuccess) return 1;
  return wide_block(n, cus);
}

hipError_t launch_step_block(const DevNet& n, int32_t t, hipStream_t s) {
  int cus = 0;
  const hipError_t e = device_cus_wide(cus);
  return e != hipSuccess ? e : launch_block_wide(n, t, cus, s);
}

}  // namespace snmi
