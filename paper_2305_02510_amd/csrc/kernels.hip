// HIP kernels for gfx950: pull delivery of delayed spikes and the fused
// leak / integrate / threshold / refractory / reset update of §2.1.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sn_device.h"
#include "sn_internal.h"

namespace snmi {

// ---------------------------------------------------------------------------
// Persistent kernel: runs `steps` time steps in one launch.
//
// Workgroup (w, b) owns the contiguous post-neuron groups [g0, g0 + ng) of
// slice w for trial b: their records (copied to LDS when they fit) and their
// neuron state (registers).  The spike history of the last D steps is a ring
// of D + 1 bit rows (slot t mod (D+1) holds step t; step t reads the slots of
// t - d, d = 1..D, never its own), in LDS when it fits.
//
// Delivery.  Records in lane-owned rows (lane l holds a synapse of post l)
// add into a register of their lane; only overflow records of high
// in-degree posts use LDS atomics.  How the waves share the groups is one of
// three modes (kModeSlot, kModeOwn, kModeRange) chosen per slice.
//
// Spike exchange.  Every step each workgroup also publishes its spike words,
// 32 spikes per 64-bit word tagged with the step: (t + 1) << 32 | bits, stored
// with one device-scope relaxed atomic in the mailbox ring [D+1][B][2G].
// Because tag and data share one atomic location, a reader that sees tag
// t + 1 sees that step's bits; no cache writeback or invalidate is needed.
// A workgroup first delivers its delay >= 2 synapses (history it already
// holds), then reads row t - 1, waiting on any word whose tag is not yet t,
// then delivers its delay-1 synapses.  A slice runs at most one step ahead
// of the slowest, so a slot is never rewritten before every reader is done
// with it.  Without an LDS ring the bits are read from the mailbox ring
// itself.  Every wait is bounded: after kSpinLimit polls the workgroup
// records a timeout in *status and all its waves exit; slices waiting on it
// then time out the same way.
//
// Thread tid owns the neurons of local groups wave + k * nwave (k < NPT), so
// the ballot of a wave is the spike word of one group.
// ---------------------------------------------------------------------------
constexpr uint32_t kSpinLimit = 1u << 22;
constexpr int kMaxWaves = 16;  // waves of the largest workgroup (1024 threads)

__device__ __forceinline__ uint64_t load_dev(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_dev(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Meta word of a record staged in LDS next to an LDS spike ring: bits 0-15
// the ring offset (Dr - d) * W32 + pre / 32 of the source word relative to
// the current row (row t - d = cur - d mod Dr), bits 16-20 the source bit
// pre % 32, bits 26-31 the post-neuron in its group (as in global records).
// A ring held in LDS has Dr * W32 < 2^16 words, so the offset fits.
__device__ __forceinline__ uint32_t lds_meta(uint32_t m, int Dr, int W32) {
  const uint32_t d = ((m >> 20) & 63u) + 1u;
  const uint32_t pre = m & 0xFFFFFu;
  return ((static_cast<uint32_t>(Dr) - d) * static_cast<uint32_t>(W32) + (pre >> 5)) | ((pre & 31u) << 16) |
         (m & 0xFC000000u);
}

// LDS accumulator rows per group: two buffers (by step parity) when several
// waves deliver into one group, so a fast wave of step t + 1 never adds into
// the row the updating wave is still reading for step t.
__host__ __device__ __forceinline__ int acc_rows(int ng_max, int nwave) {
  return ng_max < nwave ? 2 * ng_max : ng_max;
}

// Records [k, k + 4 * 64) of the calling lane's chunk (four, 64 apart);
// valid(u) is false past `end`.  Loads are issued unconditionally with the
// index clamped into the chunk (start < end), so the four are in flight
// together; deliver_chunk masks the invalid ones.  COMPACT reads the 4-byte
// copies of the records (n.crecs, see compact_record).
// A record as held between its load and its delivery: the 8-byte record,
// or with COMPACT its 4-byte copy.
template <bool COMPACT>
struct RecHeld {
  using type = Rec;
};
template <>
struct RecHeld<true> {
  using type = uint32_t;
};

// Which records of a held chunk are inside their section: a flag per
// record, or with COMPACT (sections of whole rows) the count of valid rows.
template <bool COMPACT, int U>
struct ChunkValid {
  bool v[U];
  __device__ __forceinline__ bool operator()(int u) const { return v[u]; }
};
template <int U>
struct ChunkValid<true, U> {
  int rows;
  __device__ __forceinline__ bool operator()(int u) const { return u < rows; }
};

template <bool RECS_LDS, bool COMPACT = false, int U = 4>
__device__ __forceinline__ void load_recs(const DevNet& n, const Rec* lrec, int start, int end, int lane, int r0,
                                          typename RecHeld<COMPACT>::type (&rc)[U], ChunkValid<COMPACT, U>& valid) {
  if constexpr (COMPACT) {
    // start and end are row boundaries: a row is valid or masked as a whole,
    // and a masked row's loads stay inside the array's slack (one chunk),
    // so the loads need no clamp and take their row from an immediate offset
    valid.rows = (end - start) >> 6;
    if constexpr (RECS_LDS) {  // the slice's records staged in LDS (4 bytes each)
      const uint32_t* src = reinterpret_cast<const uint32_t*>(lrec) + (start - r0) + lane;
#pragma unroll
      for (int u = 0; u < U; ++u) rc[u] = src[64 * u];
    } else {
      // (through the global address space: the pointer comes from device
      // memory, and a flat load would also hold back the waits for LDS reads)
      const __attribute__((address_space(1))) uint32_t* src =
          (const __attribute__((address_space(1))) uint32_t*)(n.crecs + start + lane);
#pragma unroll
      for (int u = 0; u < U; ++u) rc[u] = src[64 * u];
    }
  } else {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = start + lane + 64 * u;
      valid.v[u] = k < end;
      const int kc = k < end ? k : end - 1;
      if constexpr (RECS_LDS) {
        rc[u] = lrec[kc - r0];
      } else {
        rc[u] = n.recs[kc];
      }
    }
  }
}

// How the waves of a workgroup share the delivery of its ng groups:
//   kModeSlot   ng < nwave: team q of m = nwave / ng waves delivers group q,
//               member i the chunks i, i + m, ...; partial sums go to LDS
//               slots read by the updating wave;
//   kModeOwn    wave w delivers the groups w, w + nwave, ... (those it also
//               updates), used when that balances: ng a multiple of nwave or
//               at least 4 nwave;
//   kModeRange  otherwise: the groups' chunks are cut into nwave contiguous
//               ranges; a group inside one range is added to its accumulator
//               row directly, a group split between ranges atomically.
constexpr int kModeSlot = 0, kModeOwn = 1, kModeRange = 2;

// The U records of one chunk held by a lane: source bits from the ring
// (or the mailbox), own-post weights into *sum, other posts atomically.
template <bool RECS_LDS, bool RING_LDS, int U = 4>
__device__ __forceinline__ void deliver_chunk(const DevNet& n, const Rec (&rc)[U], const ChunkValid<false, U>& valid,
                                              const uint32_t* ring, const uint64_t* mring, float* acc_g, float& sum,
                                              int lane, int t, int cur, int Dr, int W32, uint32_t curW, uint32_t DrW) {
  uint32_t bit[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t mt = rc[u].meta;
    if (RING_LDS && RECS_LDS) {
      // staged records carry their ring offset (see lds_meta): the row of
      // step t - d is cur - d modulo Dr, i.e. one add and a wrap.  A clamped
      // record (past the end) is a valid record, so the read stays inside
      // the ring; masking arithmetically keeps the four reads unconditional
      // and in flight together.  Rows of steps before 0 are zero in the
      // ring, so no test of t - d is needed.
      uint32_t adr = curW + (mt & 0xFFFFu);
      adr = min(adr, adr - DrW);
      bit[u] = (ring[adr] >> ((mt >> 16) & 31u)) & static_cast<uint32_t>(valid(u));
      continue;
    }
    const int d = static_cast<int>((mt >> 20) & 63u) + 1;
    const uint32_t pre = mt & 0xFFFFFu;
    int slot = cur - d;
    if (slot < 0) slot += Dr;
    if (RING_LDS) {
      bit[u] = (ring[slot * W32 + (pre >> 5)] >> (pre & 31u)) & static_cast<uint32_t>(valid(u));
    } else {
      bit[u] = 0u;
      if (valid(u) && t - d >= 0) {
        const uint32_t word =
            static_cast<uint32_t>(load_dev(mring + static_cast<size_t>(slot) * n.B * W32 + (pre >> 5)));
        bit[u] = (word >> (pre & 31u)) & 1u;
      }
    }
  }
  bool other = false;  // an active overflow record of another lane's post (rare)
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t post = rc[u].meta >> 26;
    sum += (bit[u] && post == static_cast<uint32_t>(lane)) ? rc[u].w : 0.f;
    other |= bit[u] && post != static_cast<uint32_t>(lane);
  }
  if (other) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t post = rc[u].meta >> 26;
      if (bit[u] && post != static_cast<uint32_t>(lane)) atomicAdd(&acc_g[post], rc[u].w);
    }
  }
}

// The U compact records of one chunk held by a lane (batch kernel: ring in
// LDS, records streamed from memory).  A record carries its source word's
// offset from the current ring row, so the lookup is one add and a wrap,
// and its source bit, extracted sign-extended into an all-ones mask.  Every
// active record's numerator k is added to the lane's integer sum (exact;
// scaled once when the sum is flushed); a record of another lane's post (an
// overflow record: nonzero post field) is rare, so it is taken back out of
// the sum afterwards and its weight added to its post atomically.
// The ring of the batch kernel holds every row twice (rows r and r + Dr), so
// the row of step t - d, cur + Dr - d, needs no wrap.
template <int U>
__device__ __forceinline__ void deliver_compact(const uint32_t (&rc)[U], const ChunkValid<true, U>& valid,
                                                const uint32_t* ring, float* acc_g, int& isum, float scale, int lane,
                                                uint32_t curW) {
  constexpr uint32_t kPostField = 63u << 18;
  int act[U];
  uint32_t other = 0;  // nonzero: an active overflow record in the chunk
  // rows past the section's end hold records of the next section (or the
  // slack), whose ring offsets are in range: every read is issued, and the
  // masked rows' bits are cleared arithmetically (a chunk is full unless it
  // is its section's last)
  auto deliver = [&](int u, int mask) {
    const uint32_t c = rc[u];
    const uint32_t adr = curW + ((c >> 5) & (kCompactMaxRing - 1u));
    // (v_bfe reads only the offset's low 5 bits: the source's bit)
    act[u] = __builtin_amdgcn_sbfe(static_cast<int>(ring[adr]), c, 1u) & mask;
    isum += act[u] & (static_cast<int>(c) >> 24);
    other |= static_cast<uint32_t>(act[u]) & c & kPostField;
  };
  const int rows = __builtin_amdgcn_readfirstlane(valid.rows);  // uniform
  if (rows >= U) {
#pragma unroll
    for (int u = 0; u < U; ++u) deliver(u, -1);
  } else {
#pragma unroll
    for (int u = 0; u < U; ++u) deliver(u, u < rows ? -1 : 0);
  }
  if (other) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t c = rc[u];
      if (act[u] != 0 && (c & kPostField) != 0) {
        const int k = static_cast<int>(c) >> 24;
        isum -= k;
        atomicAdd(&acc_g[(lane + (c >> 18)) & 63], static_cast<float>(k) * scale);
      }
    }
  }
}

// Delivers one chunk held by a lane: 8-byte records through deliver_chunk,
// compact ones through deliver_compact.
template <bool RECS_LDS, bool RING_LDS, bool COMPACT, int U>
__device__ __forceinline__ void deliver_held(const DevNet& n, const typename RecHeld<COMPACT>::type (&rc)[U],
                                             const ChunkValid<COMPACT, U>& valid, const uint32_t* ring, const uint64_t* mring,
                                             float* acc_g, float& sum, int& isum, int lane, int t, int cur, int Dr,
                                             int W32, uint32_t curW, uint32_t DrW) {
  if constexpr (COMPACT) {
    static_assert(RING_LDS, "compact records address a ring in LDS");
    deliver_compact<U>(rc, valid, ring, acc_g, isum, n.cscale, lane, curW);
  } else {
    deliver_chunk<RECS_LDS, RING_LDS, U>(n, rc, valid, ring, mring, acc_g, sum, lane, t, cur, Dr, W32, curW, DrW);
  }
}

// The lane's own-post sum of a walk segment: the float sum, or with compact
// records the integer sum of numerators times the scale.
template <bool COMPACT>
__device__ __forceinline__ float take_sum(const DevNet& n, float& sum, int& isum) {
  const float s = COMPACT ? static_cast<float>(isum) * n.cscale : sum;
  sum = 0.f;
  isum = 0;
  return s;
}

// Slot mode: the chunks member, member + m, ... of the records [beg, end)
// of one group part.  Returns the lane's own-post sum.
template <bool RECS_LDS, bool RING_LDS, bool COMPACT = false, int U = 4>
__device__ __forceinline__ float deliver_group(const DevNet& n, const Rec* lrec, const uint32_t* ring,
                                               const uint64_t* mring, float* acc_g, int beg, int end, int member,
                                               int m, int lane, int r0, int t, int cur, int Dr, int W32) {
  float sum = 0.f;
  int isum = 0;
  int start = beg + member * (64 * U);
  if (start >= end) return sum;
  const uint32_t curW = static_cast<uint32_t>(cur * W32);
  const uint32_t DrW = static_cast<uint32_t>(Dr * W32);
  const int stride = m * (64 * U);
  using Held = typename RecHeld<COMPACT>::type;
  Held rc[U];
  ChunkValid<COMPACT, U> valid;
  load_recs<RECS_LDS, COMPACT, U>(n, lrec, start, end, lane, r0, rc, valid);
  for (; start < end; start += stride) {
    Held nx[U];
    ChunkValid<COMPACT, U> nvalid;
    if (!RECS_LDS && start + stride < end) load_recs<RECS_LDS, COMPACT, U>(n, lrec, start + stride, end, lane, r0, nx, nvalid);
    deliver_held<RECS_LDS, RING_LDS, COMPACT, U>(n, rc, valid, ring, mring, acc_g, sum, isum, lane, t, cur, Dr, W32,
                                                 curW, DrW);
    if (start + stride < end) {
      if (RECS_LDS) {
        load_recs<RECS_LDS, COMPACT, U>(n, lrec, start + stride, end, lane, r0, rc, valid);
      } else {
#pragma unroll
        for (int u = 0; u < U; ++u) rc[u] = nx[u];
        valid = nvalid;
      }
    }
  }
  return take_sum<COMPACT>(n, sum, isum);
}

// One part of the delivery (delay >= 2 or delay 1) as a walk over chunks.
// cs[lg] .. cs[lg + 1] are the part's chunks of group lg, bp[lg] / ep[lg]
// its first / past-last record.  The walk starts at chunk c of group lg and
// steps by cstride inside a group; at a group's end (or at chunk hi) it
// moves by gstep groups (0: stop).  A lane sums the records of its own post
// (lane-owned rows) in a register and flushes the sum when the group
// changes: Slot mode returns it, Own and Range modes add it into acc[lg]
// (Range: atomically unless the whole group lies in [lo, hi)).  Records of
// other posts (overflow) are added into acc[lg][post] atomically.  Records
// in global memory are prefetched one chunk ahead, across group changes.
template <bool RECS_LDS, bool RING_LDS, bool COMPACT = false, int U = 4>
__device__ __forceinline__ float deliver(const DevNet& n, const Rec* lrec, const uint32_t* ring,
                                         const uint64_t* mring, float* acc, const int* cs, const int* bp,
                                         const int* ep, int ng, int lg, int c, int cstride, int gstep, int lo, int hi,
                                         int mode, int lane, int r0, int t, int cur, int Dr, int W32) {
  float ret = 0.f;
  // the first item: skip to a group with chunks left
  auto item_end = [&](int g) { return mode == kModeRange ? min(cs[g + 1], hi) : cs[g + 1]; };
  if (mode == kModeRange ? c >= hi : c >= item_end(lg)) {
    if (mode != kModeOwn) return ret;
    while (lg < ng && cs[lg] == cs[lg + 1]) lg += gstep;
    if (lg >= ng) return ret;
    c = cs[lg];
  }
  const uint32_t curW = static_cast<uint32_t>(cur * W32);
  const uint32_t DrW = static_cast<uint32_t>(Dr * W32);
  // the current group's records, first chunk and chunk bound (re-read from
  // LDS only when the walk moves to another group)
  int beg = bp[lg], end = ep[lg], c0 = cs[lg], cend = item_end(lg);
  using Held = typename RecHeld<COMPACT>::type;
  Held rc[U];
  ChunkValid<COMPACT, U> valid;
  load_recs<RECS_LDS, COMPACT, U>(n, lrec, beg + (c - c0) * (64 * U), end, lane, r0, rc, valid);
  float sum = 0.f;
  int isum = 0;
  for (;;) {
    // the next item
    int nlg = lg, nc = c + cstride;
    bool more = true;
    if (nc >= cend) {
      if (mode == kModeSlot) {
        more = false;
      } else if (mode == kModeRange) {
        more = nc < hi;
        nlg = lg + 1;
        while (more && cs[nlg + 1] <= nc) ++nlg;  // skip groups without chunks
      } else {
        nlg = lg + gstep;
        while (nlg < ng && cs[nlg] == cs[nlg + 1]) nlg += gstep;
        more = nlg < ng;
        nc = more ? cs[nlg] : nc;
      }
    }
    int nbeg = beg, nend = end, nc0 = c0, ncend = cend;
    if (nlg != lg && more) {
      nbeg = bp[nlg];
      nend = ep[nlg];
      nc0 = cs[nlg];
      ncend = item_end(nlg);
    }
    Held nx[U];
    ChunkValid<COMPACT, U> nvalid;
    if (!RECS_LDS && more) load_recs<RECS_LDS, COMPACT, U>(n, lrec, nbeg + (nc - nc0) * (64 * U), nend, lane, r0, nx, nvalid);
    float* acc_g = acc + lg * kGroup;
    deliver_held<RECS_LDS, RING_LDS, COMPACT, U>(n, rc, valid, ring, mring, acc_g, sum, isum, lane, t, cur, Dr, W32,
                                                 curW, DrW);
    if (!more || nlg != lg) {  // flush the group's register sum (uniform)
      const float gsum = take_sum<COMPACT>(n, sum, isum);
      if (mode == kModeSlot) {
        ret = gsum;
      } else if (mode == kModeOwn || (cs[lg] >= lo && cs[lg + 1] <= hi)) {
        acc_g[lane] += gsum;  // this wave is the group's only contributor in this part
      } else {
        atomicAdd(&acc_g[lane], gsum);
      }
    }
    if (!more) break;
    if (RECS_LDS) {
      load_recs<RECS_LDS, COMPACT, U>(n, lrec, nbeg + (nc - nc0) * (64 * U), nend, lane, r0, rc, valid);
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) rc[u] = nx[u];
      valid = nvalid;
    }
    lg = nlg;
    c = nc;
    beg = nbeg;
    end = nend;
    c0 = nc0;
    cend = ncend;
  }
  return ret;
}

// PARAMS_LDS: neuron parameters live in LDS instead of registers (the batch
// kernel, whose occupancy is bound by registers, not LDS).
template <int NPT, bool RECS_LDS, bool RING_LDS, bool MULTI, bool PARAMS_LDS = false, bool COMPACT = false, int U = 4>
__device__ __forceinline__ bool sim_body(const SimArgs& a, int w, int b, int t0, int steps, unsigned char* smem,
                                         int& abort_flag) {
  const DevNet& n = a.n;
  const int nthr = blockDim.x;
  const int nwave = nthr >> 6;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int Dr = n.D + 1;
  const int W32 = 2 * n.G;
  const int g0 = a.wg_group[w];
  const int ng = a.wg_group[w + 1] - g0;
  const int r0 = n.gptr[g0];
  const int nrec = n.gptr[g0 + ng] - r0;
  const bool use_mail = MULTI || !RING_LDS;
  // delivery mode (see kModeSlot) and accumulator buffers
  const int m = ng < nwave ? nwave / ng : 1;
  const int team = wave / m;
  const int member = wave - team * m;
  const int mode = (ng < nwave && 4 * m * ng >= 3 * nwave) ? kModeSlot
                   : (ng >= nwave && (ng % nwave == 0 || ng >= 4 * nwave)) ? kModeOwn : kModeRange;
  const int nacc = acc_rows(a.ng_max, nwave) > a.ng_max ? 2 : 1;
  // another wave may add into a group's row while its updater reads it, so
  // the step ends with a barrier unless the rows alternate by step parity
  const bool end_barrier = mode != kModeOwn && nacc == 1;
  // mailbox ring of this trial: slot s at mring + s * B * W32
  uint64_t* mring = a.mailbox + static_cast<size_t>(b) * W32;

  uint32_t* ring = reinterpret_cast<uint32_t*>(smem);
  // with COMPACT the ring holds every row twice (see deliver_compact)
  constexpr int kRingCopies = COMPACT ? 2 : 1;
  const int ring_second = COMPACT ? Dr * W32 : 0;  // offset of the second copy
  float* acc = reinterpret_cast<float*>(ring + (RING_LDS ? kRingCopies * Dr * W32 : 0));  // [nacc][ng_max][64]
  float* part = acc + acc_rows(a.ng_max, nwave) * kGroup;                    // [kMaxWaves][64]
  int* gsp = reinterpret_cast<int*>(part + kMaxWaves * kGroup);  // [ng + 1] starts, [ng] splits
  int* csA = gsp + 2 * a.ng_max + 1;                              // [ng + 1] chunk offsets, delay >= 2
  int* csB = csA + a.ng_max + 1;                                  // [ng + 1] chunk offsets, delay 1
  float* prm = reinterpret_cast<float*>(csB + a.ng_max + 2);      // PARAMS_LDS: [5][ng_max][64]
  Rec* lrec = reinterpret_cast<Rec*>(prm + (PARAMS_LDS ? 5 * a.ng_max * kGroup : 0));  // 8-byte aligned

  if (tid == 0) abort_flag = 0;
  __syncthreads();
  if (RING_LDS) {
    for (int i = tid; i < kRingCopies * Dr * W32; i += nthr) ring[i] = 0u;
  }
  for (int i = tid; i < acc_rows(a.ng_max, nwave) * kGroup; i += nthr) acc[i] = 0.f;
  for (int i = tid; i <= ng; i += nthr) gsp[i] = n.gptr[g0 + i];
  for (int i = tid; i < ng; i += nthr) gsp[ng + 1 + i] = n.gsplit[g0 + i];
  if (tid == 0) {  // chunk offsets of both parts (after the loads above land)
    int ca = 0, cb = 0;
    for (int i = 0; i < ng; ++i) {
      const int s0 = n.gptr[g0 + i], s1 = n.gsplit[g0 + i], s2 = n.gptr[g0 + i + 1];
      csA[i] = ca;
      csB[i] = cb;
      ca += (s1 - s0 + (64 * U) - 1) / (64 * U);
      cb += (s2 - s1 + (64 * U) - 1) / (64 * U);
    }
    csA[ng] = ca;
    csB[ng] = cb;
  }
  if (RECS_LDS && COMPACT) {  // 4-byte records as they are, then one chunk of zero slack
    uint32_t* l32 = reinterpret_cast<uint32_t*>(lrec);
    for (int i = tid; i < nrec + 64 * U; i += nthr) l32[i] = i < nrec ? n.crecs[r0 + i] : 0u;
  } else if (RECS_LDS) {
    for (int i = tid; i < nrec; i += nthr) {
      Rec r = n.recs[r0 + i];
      if (RING_LDS) r.meta = lds_meta(r.meta, Dr, W32);
      lrec[i] = r;
    }
  }
  __syncthreads();
  if (RING_LDS) {  // history of the steps before t0 (rows < 0 stay zero)
    const size_t rstride = static_cast<size_t>(n.B) * n.G;
    const uint64_t* hist = n.raster + static_cast<size_t>(b) * n.G;
    for (int d = 1; d <= n.D; ++d) {
      const int ts = t0 - d;
      if (ts < 0) break;
      const int slot = ts % Dr;
      for (int i = tid; i < n.G; i += nthr) {
        const uint64_t wv = hist[static_cast<size_t>(ts) * rstride + i];
        ring[slot * W32 + 2 * i] = static_cast<uint32_t>(wv);
        ring[slot * W32 + 2 * i + 1] = static_cast<uint32_t>(wv >> 32);
        if (COMPACT) {
          ring[ring_second + slot * W32 + 2 * i] = static_cast<uint32_t>(wv);
          ring[ring_second + slot * W32 + 2 * i + 1] = static_cast<uint32_t>(wv >> 32);
        }
      }
    }
  }

  // where this wave's walk over each part starts (see deliver)
  int wlg[2], wc[2], wlo[2], whi[2];
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const int* cs = x == 0 ? csA : csB;
    const int q = cs[ng];
    wlo[x] = 0;
    whi[x] = q;
    if (mode == kModeSlot) {
      wlg[x] = team < ng ? team : ng;
      wc[x] = team < ng ? cs[team] + member : q;
    } else if (mode == kModeOwn) {
      wlg[x] = wave;
      wc[x] = wave < ng ? cs[wave] : q;
    } else {
      wlo[x] = static_cast<int>(static_cast<int64_t>(q) * wave / nwave);
      whi[x] = static_cast<int>(static_cast<int64_t>(q) * (wave + 1) / nwave);
      int g = 0;
      while (g < ng && cs[g + 1] <= wlo[x]) ++g;
      wlg[x] = g;
      wc[x] = wlo[x];
    }
  }
  constexpr int NP = PARAMS_LDS ? 1 : NPT;  // parameter registers
  float V[NPT], th[NP], lam[NP], rs[NP], amp[NP];
  int ref[NPT], R[NP];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int lg = wave + k * nwave;
    V[k] = 0.f; ref[k] = 0;
    if (!PARAMS_LDS) { th[k % NP] = 0.f; lam[k % NP] = 0.f; rs[k % NP] = 0.f; amp[k % NP] = 0.f; R[k % NP] = 0; }
    if (lg < ng) {
      const int j = (g0 + lg) * kGroup + lane;
      V[k] = n.V[static_cast<size_t>(b) * n.Npad + j];
      ref[k] = n.ref[static_cast<size_t>(b) * n.Npad + j];
      if (PARAMS_LDS) {
        const int i = lg * kGroup + lane, s5 = a.ng_max * kGroup;
        prm[i] = n.theta[j];
        prm[s5 + i] = n.leak[j];
        prm[2 * s5 + i] = n.reset[j];
        prm[3 * s5 + i] = n.amp[j];
        prm[4 * s5 + i] = __int_as_float(static_cast<int>(n.refr[j]));
      } else {
        th[k % NP] = n.theta[j];
        lam[k % NP] = n.leak[j];
        rs[k % NP] = n.reset[j];
        amp[k % NP] = n.amp[j];
        R[k % NP] = n.refr[j];
      }
    }
  }
  __syncthreads();

  for (int t = t0; t < t0 + steps; ++t) {
    // external spike words of this step, issued first and consumed by the
    // update (a value carried across iterations would make every wave wait
    // for its stores at the end of the step)
    // (the 32-bit half of the group's word that holds this lane's bit)
    uint32_t ew[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int lg = wave + k * nwave;
      ew[k] = lg < ng ? reinterpret_cast<const uint32_t*>(n.ext + row_word(n, t, b, g0 + lg))[lane >> 5] : 0u;
    }
    const int cur = t % Dr;
    float* accb = acc + (nacc == 2 ? (t & 1) * a.ng_max * kGroup : 0);
    // receive row t - 1: every word carries its step tag.  The first read of
    // this thread's word is issued before the delay >= 2 delivery, which
    // hides its latency; a word whose tag is not yet t is read again.
    const int prev = (t > 0 ? t - 1 : 0) % Dr;
    const bool receive = MULTI && t > t0;
    uint64_t early = 0;
    if (receive && tid < W32) early = load_dev(mring + static_cast<size_t>(prev) * n.B * W32 + tid);
    // delay >= 2: every needed row is already held
    const int cstride = mode == kModeSlot ? m : 1;
    const int gstep = mode == kModeOwn ? nwave : 1;
    float sum = 0.f;
    if (mode == kModeSlot) {  // uniform per wave
      if (team < ng)
        sum = deliver_group<RECS_LDS, RING_LDS, COMPACT, U>(n, lrec, ring, mring, accb + team * kGroup, gsp[team],
                                                gsp[ng + 1 + team], member, m, lane, r0, t, cur, Dr, W32);
    } else if (wlg[0] < ng) {
      deliver<RECS_LDS, RING_LDS, COMPACT, U>(n, lrec, ring, mring, accb, csA, gsp, gsp + ng + 1, ng, wlg[0], wc[0], cstride,
                                  gstep, wlo[0], whi[0], mode, lane, r0, t, cur, Dr, W32);
    }
    if (receive) {
      const uint64_t tag = static_cast<uint64_t>(t);
      for (int i = tid; i < W32; i += nthr) {
        const uint64_t* p = mring + static_cast<size_t>(prev) * n.B * W32 + i;
        uint64_t v = i == tid ? early : load_dev(p);
        uint32_t spins = 0;
        while ((v >> 32) != tag) {
          if (++spins > kSpinLimit) {
            abort_flag = 1;
            __hip_atomic_store(a.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          v = load_dev(p);
        }
        if (RING_LDS) ring[prev * W32 + i] = static_cast<uint32_t>(v);
        if (RING_LDS && COMPACT) ring[ring_second + prev * W32 + i] = static_cast<uint32_t>(v);
      }
    }
    __syncthreads();
    if (MULTI && abort_flag) return false;  // uniform: read after the barrier
    // delay 1
    if (mode == kModeSlot) {
      if (team < ng)
        sum += deliver_group<RECS_LDS, RING_LDS, COMPACT, U>(n, lrec, ring, mring, accb + team * kGroup, gsp[ng + 1 + team],
                                                 gsp[team + 1], member, m, lane, r0, t, cur, Dr, W32);
    } else if (wlg[1] < ng) {
      deliver<RECS_LDS, RING_LDS, COMPACT, U>(n, lrec, ring, mring, accb, csB, gsp + ng + 1, gsp + 1, ng, wlg[1], wc[1], cstride,
                                  gstep, wlo[1], whi[1], mode, lane, r0, t, cur, Dr, W32);
    }
    if (mode == kModeSlot) part[wave * kGroup + lane] = sum;  // partial sums for the updating wave
    if (mode != kModeOwn) __syncthreads();
    // fused neuron update; the ballot of a wave is the spike word of its group
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int lg = wave + k * nwave;
      if (lg < ng) {  // uniform per wave
        float syn = accb[lg * kGroup + lane];
        accb[lg * kGroup + lane] = 0.f;
        if (mode == kModeSlot) {
          for (int i = 0; i < m; ++i) syn += part[(lg * m + i) * kGroup + lane];
        }
        bool s;
        if (PARAMS_LDS) {
          const int i = lg * kGroup + lane, s5 = a.ng_max * kGroup;
          s = lif_update(V[k], ref[k], syn, (ew[k] >> (lane & 31)) & 1u, prm[i], prm[s5 + i], prm[2 * s5 + i],
                         prm[3 * s5 + i], __float_as_int(prm[4 * s5 + i]));
        } else {
          s = lif_update(V[k], ref[k], syn, (ew[k] >> (lane & 31)) & 1u, th[k % NP], lam[k % NP], rs[k % NP],
                         amp[k % NP], R[k % NP]);
        }
        const uint64_t sw = __ballot(s);
        const int g = g0 + lg;
        if (lane == 0) n.raster[row_word(n, t, b, g)] = sw;
        if (RING_LDS && lane < 2) {
          ring[cur * W32 + 2 * g + lane] = static_cast<uint32_t>(sw >> (32 * lane));
          if (COMPACT) ring[ring_second + cur * W32 + 2 * g + lane] = static_cast<uint32_t>(sw >> (32 * lane));
        }
        if (use_mail && lane < 2) {
          const uint64_t tagged = (static_cast<uint64_t>(t + 1) << 32) | ((sw >> (32 * lane)) & 0xFFFFFFFFull);
          store_dev(mring + static_cast<size_t>(cur) * n.B * W32 + 2 * g + lane, tagged);
        }
      }
    }
    // Otherwise no barrier closes the step: the next step's delay >= 2
    // delivery reads rows up to t - 1 only, its accumulator rows are the
    // other buffer or this wave's own, and everything that reads row t, the
    // partial sums or the received words comes after its first barrier.
    if (end_barrier) __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int lg = wave + k * nwave;
    if (lg < ng) {
      const int j = (g0 + lg) * kGroup + lane;
      n.V[static_cast<size_t>(b) * n.Npad + j] = V[k];
      n.ref[static_cast<size_t>(b) * n.Npad + j] = static_cast<uint8_t>(ref[k]);
    }
  }
  __syncthreads();  // the shared memory may be reused by the caller
  return true;
}

// COMPACT: the slice's compact records (n.crecs) staged in LDS, 4 bytes each,
// against a doubled ring (records and ring both in LDS).
template <int NPT, bool RECS_LDS, bool RING_LDS, bool MULTI, bool COMPACT = false>
__global__ __launch_bounds__(1024) void k_sim(const SimArgs a, int t0, int steps) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int abort_flag;
  const int w = MULTI ? static_cast<int>(blockIdx.x) : 0;
  const int b = MULTI ? static_cast<int>(blockIdx.y) : static_cast<int>(blockIdx.x);
  sim_body<NPT, RECS_LDS, RING_LDS, MULTI, false, COMPACT>(a, w, b, t0, steps, smem, abort_flag);
}

// Mailbox before a launch starting at t0: slot of row r (t0 - D <= r < t0,
// r >= 0) holds row r of the raster tagged r + 1; every other slot is zero
// (tag 0 is never awaited), so no word left by an earlier launch can match a
// tag this launch waits for.
__global__ void k_prefill_mailbox(const SimArgs a, int t0) {
  const DevNet& n = a.n;
  const int W32 = 2 * n.G;
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int Dr = n.D + 1;
  const size_t total = static_cast<size_t>(Dr) * n.B * W32;
  if (i >= total) return;
  const int word = static_cast<int>(i % W32);
  const int b = static_cast<int>((i / W32) % n.B);
  const int slot = static_cast<int>(i / (static_cast<size_t>(W32) * n.B));
  // the row r in [t0 - D, t0] with r mod Dr == slot
  int r = t0 - ((t0 - slot) % Dr + Dr) % Dr;
  uint64_t v = 0;
  if (r < t0 && r >= 0) {
    const uint64_t wv = n.raster[row_word(n, r, b, word >> 1)];
    v = (static_cast<uint64_t>(r + 1) << 32) | ((wv >> (32 * (word & 1))) & 0xFFFFFFFFull);
  }
  a.mailbox[i] = v;
}

hipError_t launch_prefill_mailbox(const SimArgs& a, int32_t t0, hipStream_t s) {
  const size_t total = static_cast<size_t>(a.n.D + 1) * a.n.B * 2 * a.n.G;
  hipLaunchKernelGGL(k_prefill_mailbox, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s, a, t0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched persistent kernel (see BatchArgs): workgroups 0 .. n_team - 1 first
// run their team slice, then every workgroup takes queue entries until the
// queue is empty.  Team slices wait only on slices of the same network, all
// of which are resident (cooperative launch) and start with their team task.
// ---------------------------------------------------------------------------
// Records per lane in one chunk of the batch kernel's record stream: 12 with
// 4-byte records (three times the bytes in flight per wave; measured on the
// 512-net batch: 8 -> 115 ms, 12 -> 109 ms, 16 -> 119 ms per 500-step run),
// else 4.
template <bool COMPACT>
constexpr int kBatchU = COMPACT ? kCompactChunkRows : 4;

// COMPACT: every network of the batch has 4-byte record copies (n.crecs).
template <bool COMPACT>
__global__ __launch_bounds__(kBatchThreads, 4) void k_batch(const BatchArgs ba, int steps) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int abort_flag;
  __shared__ int next;
  if (static_cast<int>(blockIdx.x) < ba.n_team) {
    const int4 tt = ba.team[blockIdx.x];
    const SimArgs a = ba.nets[tt.x].team;
    if (!sim_body<kBatchMaxGroups / (kBatchThreads / 64), false, true, true, true, COMPACT, kBatchU<COMPACT>>(
            a, tt.y, tt.z, tt.w, steps, smem,
                                                                                   abort_flag))
      return;
  }
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(ba.queue_head, 1);
    __syncthreads();
    const int i = next;
    __syncthreads();
    if (i >= ba.n_queue) return;
    const int4 qt = ba.queue[i];
    const SimArgs a = ba.nets[qt.x].single;
    sim_body<kBatchMaxGroups / (kBatchThreads / 64), false, true, false, true, COMPACT, kBatchU<COMPACT>>(
        a, 0, qt.y, qt.z, steps, smem,
                                                                               abort_flag);
  }
}

constexpr size_t kLdsLimit = 160 * 1024;
constexpr int kMaxNpt = 8;

// LDS of sim_body: [ring][accumulators][partial sums][group offsets][records]
// (compact: 4-byte records plus one 4-row chunk of slack, two ring copies)
size_t sim_lds_bytes(const DevNet& n, int ng_max, int64_t max_recs, int nwave, bool recs_lds, bool ring_lds,
                     bool compact) {
  size_t bytes = static_cast<size_t>(acc_rows(ng_max, nwave)) * kGroup * sizeof(float);
  bytes += static_cast<size_t>(kMaxWaves) * kGroup * sizeof(float);
  bytes += static_cast<size_t>(4 * ng_max + 4) * sizeof(int);
  if (ring_lds) bytes += static_cast<size_t>(compact ? 2 : 1) * (n.D + 1) * 2 * n.G * sizeof(uint32_t);
  if (recs_lds)
    bytes += compact ? static_cast<size_t>(max_recs + 4 * 64) * sizeof(uint32_t) : static_cast<size_t>(max_recs) * sizeof(Rec);
  return bytes + 64;  // static LDS of the kernel
}

// (a net with compact records may run in a batch that keeps two copies of
// its ring)
size_t batch_lds_bytes(const DevNet& n, int ng_max) {
  return sim_lds_bytes(n, ng_max, 0, kBatchThreads / 64, false, true) - 64 +
         static_cast<size_t>(5) * ng_max * kGroup * sizeof(float) +
         (n.crecs ? static_cast<size_t>(n.D + 1) * 2 * n.G * sizeof(uint32_t) : 0);
}

int batch_blocks_per_cu(size_t lds, bool compact) {
  int blocks = 0;
  const void* fn = compact ? reinterpret_cast<const void*>(&k_batch<true>) : reinterpret_cast<const void*>(&k_batch<false>);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
    return 0;
  const hipError_t e = compact ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<true>, kBatchThreads, lds)
                               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<false>, kBatchThreads, lds);
  return e == hipSuccess ? blocks : 0;
}

hipError_t launch_batch(const BatchArgs& a, int grid, size_t lds, int32_t steps, bool compact, hipStream_t s) {
  const void* fn = compact ? reinterpret_cast<const void*>(&k_batch<true>) : reinterpret_cast<const void*>(&k_batch<false>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e != hipSuccess) return e;
  void* args[] = {const_cast<BatchArgs*>(&a), &steps};
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kBatchThreads), args, static_cast<unsigned>(lds), s);
}

__global__ void k_zero_i32(int32_t* p) { *p = 0; }

hipError_t launch_zero_i32(int32_t* p, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, s, p);
  return hipGetLastError();
}

size_t lds_limit() { return kLdsLimit; }

// Threads of a slice's workgroup: at least one wave per group (the update),
// and enough waves that delivery has ~8 records per lane, up to 1024.
int sim_threads(int ng_max, int64_t max_recs) {
  int64_t thr = std::max<int64_t>(static_cast<int64_t>(ng_max) * kGroup, (max_recs / 8 + 63) / 64 * 64);
  return static_cast<int>(std::min<int64_t>(thr, 1024));
}

int sim_npt(int ng_max, int64_t max_recs) {
  const int nw = sim_threads(ng_max, max_recs) / kGroup;
  return (ng_max + nw - 1) / nw;
}

template <int NPT, bool RL, bool GL, bool MULTI, bool COMPACT = false>
static hipError_t launch_sim_t(const SimArgs& a, int32_t t0, int32_t steps, hipStream_t s, size_t lds) {
  const void* fn = reinterpret_cast<const void*>(&k_sim<NPT, RL, GL, MULTI, COMPACT>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(kLdsLimit - 64));
  if (e != hipSuccess) return e;
  const dim3 block(sim_threads(a.ng_max, a.max_recs));
  if (MULTI) {
    const dim3 grid(a.P, a.n.B);
    void* args[] = {const_cast<SimArgs*>(&a), &t0, &steps};
    return hipLaunchCooperativeKernel(fn, grid, block, args, static_cast<unsigned>(lds), s);
  }
  hipLaunchKernelGGL((k_sim<NPT, RL, GL, MULTI, COMPACT>), dim3(a.n.B), block, lds, s, a, t0, steps);
  return hipGetLastError();
}

template <bool MULTI>
static hipError_t launch_sim_m(const SimArgs& a, bool rl, bool gl, bool compact, int32_t t0, int32_t steps,
                               hipStream_t s, size_t lds) {
  const int npt = sim_npt(a.ng_max, a.max_recs);
  const int np2 = npt <= 1 ? 1 : npt <= 2 ? 2 : npt <= 4 ? 4 : 8;
  if (compact) {  // records and ring in LDS
    switch (np2) {
      case 1: return launch_sim_t<1, true, true, MULTI, true>(a, t0, steps, s, lds);
      case 2: return launch_sim_t<2, true, true, MULTI, true>(a, t0, steps, s, lds);
      case 4: return launch_sim_t<4, true, true, MULTI, true>(a, t0, steps, s, lds);
      default: return launch_sim_t<8, true, true, MULTI, true>(a, t0, steps, s, lds);
    }
  }
  const int key = np2 * 4 + (rl ? 2 : 0) + (gl ? 1 : 0);
  switch (key) {
#define SN_CASE(NP)                                                                  \
  case NP * 4 + 0: return launch_sim_t<NP, false, false, MULTI>(a, t0, steps, s, lds); \
  case NP * 4 + 1: return launch_sim_t<NP, false, true, MULTI>(a, t0, steps, s, lds);  \
  case NP * 4 + 2: return launch_sim_t<NP, true, false, MULTI>(a, t0, steps, s, lds);  \
  case NP * 4 + 3: return launch_sim_t<NP, true, true, MULTI>(a, t0, steps, s, lds);
    SN_CASE(1)
    SN_CASE(2)
    SN_CASE(4)
    SN_CASE(8)
#undef SN_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sim(const SimArgs& a, bool recs_lds, bool ring_lds, int32_t t0, int32_t steps, hipStream_t s) {
  if (sim_npt(a.ng_max, a.max_recs) > kMaxNpt) return hipErrorInvalidValue;
  const int nwave = sim_threads(a.ng_max, a.max_recs) / kGroup;
  size_t lds = sim_lds_bytes(a.n, a.ng_max, a.max_recs, nwave, recs_lds, ring_lds) - 64;
  if (lds + 64 > kLdsLimit) return hipErrorInvalidValue;
  // records and ring in LDS: the compact records when the net has them and
  // they fit (half the record bytes, a doubled ring)
  bool compact = false;
  if (recs_lds && ring_lds && a.n.crecs) {
    const size_t lc = sim_lds_bytes(a.n, a.ng_max, a.max_recs, nwave, true, true, true) - 64;
    if (lc + 64 <= kLdsLimit) {
      compact = true;
      lds = lc;
    }
  }
  if (a.P > 1 || !ring_lds) {
    const hipError_t e = launch_prefill_mailbox(a, t0, s);
    if (e != hipSuccess) return e;
  }
  if (a.P > 1) return launch_sim_m<true>(a, recs_lds, ring_lds, compact, t0, steps, s, lds);
  return launch_sim_m<false>(a, recs_lds, ring_lds, compact, t0, steps, s, lds);
}


// ---------------------------------------------------------------------------
// Per-step pull kernel: workgroup (g, b) accumulates, for trial b, the
// delayed input of the 64 posts of group g.  It loads the group's records
// (coalesced 8-byte loads, U per lane in flight) and, at the same time, the D
// previous raster rows into LDS when they fit (RING), so each record costs
// one global round trip; the source bit of row t - d is then an LDS read and
// w is added into an LDS accumulator.  Wave 0 applies the neuron update and
// writes the group's spike word.
// STDP (one trial, plasticity on): with `apply`, the rule of step t - 1 (the
// rule of k_stdp with T = t - 1, from the history words H_{t-1}) is applied
// to every loaded record before its delivery, which then uses the new
// weight; wave 0 writes H_t of its 64 neurons.  The rule of the last step of
// a run is applied by k_stdp.
// ---------------------------------------------------------------------------
template <int WAVES, int U, bool RING, bool STDP>
__global__ __launch_bounds__(WAVES * 64) void k_step(const DevNet n, int t, const StdpArgs sa, int apply) {
  __shared__ float acc[kGroup];
  __shared__ float part[WAVES][kGroup];
  __shared__ uint64_t hq_s[STDP ? kGroup : 1];  // H_{t-1} of this group's neurons
  __shared__ float tab_s[STDP ? 32 : 1];         // the rule's tables: ltp [0, 16), ltd [16, 32)
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t* ring = reinterpret_cast<uint32_t*>(smem);  // [D][2G]: row t - d at (d - 1)
  const int g = blockIdx.x;
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int j = g * kGroup + lane;
  const int W32 = 2 * n.G;
  const size_t rstride = static_cast<size_t>(n.B) * n.G;
  const uint64_t* hist = n.raster + static_cast<size_t>(b) * n.G;

  float V = 0.f, th = 0.f, lam = 0.f, rs = 0.f, amp = 0.f;
  int ref = 0, R = 0;
  uint64_t ew = 0;
  if (wave == 0) {
    acc[lane] = 0.f;
    const size_t sj = static_cast<size_t>(b) * n.Npad + j;
    V = n.V[sj];
    ref = n.ref[sj];
    th = n.theta[j];
    lam = n.leak[j];
    rs = n.reset[j];
    amp = n.amp[j];
    R = n.refr[j];
    ew = n.ext[row_word(n, t, b, g)];
    if (STDP) hq_s[lane] = sa.hist[static_cast<size_t>((t - 1) & 1) * n.Npad + j];
    // the tables in LDS: an amplitude is then an LDS read, not a load from
    // the kernel arguments in memory with a per-lane index
    if (STDP && lane < 32) tab_s[lane] = lane < 16 ? sa.ltp[lane] : sa.ltd[lane - 16];
  }
  const int beg = n.gptr[g];
  const int end = n.gptr[g + 1];
  // first batch of records, issued before the history rows
  Rec rr[U];
  bool ok[U];
  int base = beg + wave * 64 * U;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = base + u * 64 + lane;
    ok[u] = k < end;
    rr[u] = ok[u] ? n.recs[k] : Rec{0.f, 0u};
  }
  if (RING) {
    for (int i = threadIdx.x; i < n.D * n.G; i += WAVES * 64) {
      const int d = i / n.G + 1, w = i - (d - 1) * n.G;
      const int ts = t - d;
      const uint64_t v = ts >= 0 ? hist[static_cast<size_t>(ts) * rstride + w] : 0ull;
      ring[(d - 1) * W32 + 2 * w] = static_cast<uint32_t>(v);
      ring[(d - 1) * W32 + 2 * w + 1] = static_cast<uint32_t>(v >> 32);
    }
  }
  __syncthreads();
  float sum = 0.f;  // lane-owned records (record k of the group is in lane k mod 64)
  const uint32_t wmask = STDP ? (1u << sa.window) - 1u : 0u;
  for (;;) {
    if (STDP && apply) {  // rule of step T = t - 1 on the loaded records
      const int T = t - 1;
      const uint64_t* hprev = sa.hist + static_cast<size_t>(T & 1) * n.Npad;
      // the pre-neuron's history word is read only where the rule can need
      // it: potentiation (the post spiked at T) or a delay whose pre spike of
      // step T - d is not in the staged rows (depression otherwise reads
      // that bit from the ring: row T - d = t - (d + 1))
      uint64_t hp[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool live = ok[u] && __float_as_uint(rr[u].w) != 0x80000000u;  // fillers keep -0.0
        const int d = static_cast<int>((rr[u].meta >> 20) & 63u) + 1;
        const bool need = (hq_s[rr[u].meta >> 26] & 1ull) || !RING || d >= n.D;
        hp[u] = live && need ? hprev[rr[u].meta & 0xFFFFFu] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (!ok[u] || __float_as_uint(rr[u].w) == 0x80000000u) continue;
        const uint32_t m = rr[u].meta;
        const uint32_t pre = m & 0xFFFFFu;
        const int d = static_cast<int>((m >> 20) & 63u) + 1;
        const uint32_t pl = m >> 26;
        const uint64_t hq = hq_s[pl];
        float change = 0.f;
        if (d + sa.window <= 64) {
          if (hq & 1ull) {
            const uint32_t x = static_cast<uint32_t>(hp[u] >> d) & wmask;
            if (x) change += tab_s[__builtin_ctz(x)];
          }
          const uint32_t pre_at = RING && d < n.D ? (ring[d * W32 + (pre >> 5)] >> (pre & 31u)) & 1u
                                                  : static_cast<uint32_t>(hp[u] >> d) & 1u;
          if (pre_at) {
            const uint32_t x = static_cast<uint32_t>(hq >> 1) & wmask;
            if (x) change -= tab_s[16 + __builtin_ctz(x)];
          }
        } else {  // the window leaves the history words: raster rows
          auto rbit = [&](int tau, uint32_t neuron) -> uint32_t {
            return static_cast<uint32_t>(n.raster[row_word(n, tau, 0, static_cast<int>(neuron >> 6))] >>
                                         (neuron & 63u)) & 1u;
          };
          const uint32_t post = static_cast<uint32_t>(g) * kGroup + pl;
          if (hq & 1ull) {
            for (int lag = 0; lag < sa.window; ++lag) {
              const int tau = T - lag - d;
              if (tau < 0) break;
              if (rbit(tau, pre)) {
                change += tab_s[lag];
                break;
              }
            }
          }
          if (T - d >= 0 && rbit(T - d, pre)) {
            for (int lag = 1; lag <= sa.window; ++lag) {
              if (T - lag < 0) break;
              if (rbit(T - lag, post)) {
                change -= tab_s[16 + lag - 1];
                break;
              }
            }
          }
        }
        const float w = fminf(fmaxf(rr[u].w + change, sa.w_min), sa.w_max);
        if (__float_as_uint(w) != __float_as_uint(rr[u].w)) {
          sa.recs[base + u * 64 + lane].w = w;
          rr[u].w = w;
        }
      }
    }
    uint32_t bit[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t m = rr[u].meta;
      const int d = static_cast<int>((m >> 20) & 63u) + 1;
      const uint32_t pre = m & 0xFFFFFu;
      bit[u] = 0u;
      if (ok[u] && t - d >= 0) {
        if (RING) {
          bit[u] = (ring[(d - 1) * W32 + (pre >> 5)] >> (pre & 31u)) & 1u;
        } else {
          bit[u] = static_cast<uint32_t>(hist[static_cast<size_t>(t - d) * rstride + (pre >> 6)] >> (pre & 63u)) & 1u;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t post = rr[u].meta >> 26;
      sum += (bit[u] && post == static_cast<uint32_t>(lane)) ? rr[u].w : 0.f;
      if (bit[u] && post != static_cast<uint32_t>(lane)) atomicAdd(&acc[post], rr[u].w);
    }
    base += WAVES * 64 * U;
    if (base >= end) break;  // uniform per wave
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = base + u * 64 + lane;
      ok[u] = k < end;
      rr[u] = ok[u] ? n.recs[k] : Rec{0.f, 0u};
    }
  }
  if (WAVES > 1) part[wave][lane] = sum;
  __syncthreads();
  if (wave == 0) {
    float syn = acc[lane] + sum;
#pragma unroll
    for (int i = 1; i < WAVES; ++i) syn += part[i][lane];
    const bool s = lif_update(V, ref, syn, (ew >> lane) & 1ull, th, lam, rs, amp, R);
    const uint64_t sw = __ballot(s);
    const size_t sj = static_cast<size_t>(b) * n.Npad + j;
    n.V[sj] = V;
    n.ref[sj] = static_cast<uint8_t>(ref);
    if (lane == 0) n.raster[row_word(n, t, b, g)] = sw;
    if (STDP) sa.hist[static_cast<size_t>(t & 1) * n.Npad + j] = (hq_s[lane] << 1) | (s ? 1ull : 0ull);
  }
}

// ---------------------------------------------------------------------------
// Plasticity after the update of step t (one trial; the rule of
// sn_set_stdp): workgroup g visits the records of group g.  For a record
// i -> j of delay d: if j spiked at t, the latest arrival of i at j within
// the window (i spiked at t - d - lag, lag < W) adds ltp[lag]; if a spike of
// i arrives at t (i spiked at t - d), the latest spike of j at t - lag,
// 1 <= lag <= W, subtracts ltd[lag - 1]; then the weight is clipped to
// [w_min, w_max].  Spike bits come from the raster rows (written by earlier
// launches); fillers (weight -0.0) are left alone.  Every change is a
// function of spike times only, so records are independent.
// ---------------------------------------------------------------------------
// Spike times come from per-neuron history words: hist[p][i] bit k = spike
// of neuron i at step T - k, where T = t - 1 for the buffer p = (t - 1) & 1
// the kernel of step t reads.  H_t(i) = (H_{t-1}(i) << 1) | s_i(t), with
// s_i(t) from the raster row t staged in LDS.  Then
//   potentiation: the arrivals within the window are bits d .. d + W - 1 of
//     H_t(pre); the latest is the lowest set bit;
//   depression: an arrival at t is bit d of H_t(pre); the post spikes at
//     t - 1 .. t - W are bits 1 .. W of H_t(post).
// A record with d + W > 64 (its window leaves the 64-bit history) reads
// the raster rows instead.  Workgroup (g, c) visits the records
// c * chunk .. of group g; workgroups (g, 0) write H_t of the group's 64
// neurons to the other buffer, for step t + 1.

__global__ __launch_bounds__(kStdpThreads) void k_stdp(const StdpArgs a, int t) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t* row_t = reinterpret_cast<uint64_t*>(smem);  // raster row t, G words
  __shared__ uint64_t hpost[kGroup];                    // H_t of this group's neurons
  const DevNet& n = a.n;
  const int g = blockIdx.x;
  const int gbeg = n.gptr[g], gend = n.gptr[g + 1];
  const int beg = min(gend, gbeg + static_cast<int>(blockIdx.y) * a.chunk);
  const int end = min(gend, beg + a.chunk);
  const uint64_t* hprev = a.hist + static_cast<size_t>((t - 1) & 1) * n.Npad;
  uint64_t* hcur = a.hist + static_cast<size_t>(t & 1) * n.Npad;
  for (int w = threadIdx.x; w < n.G; w += blockDim.x) row_t[w] = n.raster[row_word(n, t, 0, w)];
  __syncthreads();
  if (threadIdx.x < kGroup) {
    const uint32_t j = static_cast<uint32_t>(g) * kGroup + threadIdx.x;
    const uint64_t h = (hprev[j] << 1) | ((row_t[g] >> threadIdx.x) & 1ull);
    hpost[threadIdx.x] = h;
    if (blockIdx.y == 0) hcur[j] = h;
  }
  __syncthreads();
  const uint32_t wmask = (1u << a.window) - 1u;
  auto hist_t = [&](uint32_t i) -> uint64_t {
    return (hprev[i] << 1) | ((row_t[i >> 6] >> (i & 63u)) & 1ull);
  };
  auto bit = [&](int tau, uint32_t neuron) -> uint32_t {  // raster bit, for windows beyond the history
    return static_cast<uint32_t>(n.raster[row_word(n, tau, 0, static_cast<int>(neuron >> 6))] >> (neuron & 63u)) & 1u;
  };
  for (int k0 = beg + static_cast<int>(threadIdx.x); k0 < end; k0 += kStdpUnroll * kStdpThreads) {
    Rec rr[kStdpUnroll];
#pragma unroll
    for (int u = 0; u < kStdpUnroll; ++u) {
      const int k = k0 + u * kStdpThreads;
      rr[u] = k < end ? a.recs[k] : Rec{-0.f, 0u};
    }
    uint64_t hp[kStdpUnroll];
#pragma unroll
    for (int u = 0; u < kStdpUnroll; ++u) {
      const int k = k0 + u * kStdpThreads;
      const bool live = k < end && __float_as_uint(rr[u].w) != 0x80000000u;  // past the group, or a filler
      hp[u] = live ? hist_t(rr[u].meta & 0xFFFFFu) : 0ull;
    }
#pragma unroll
    for (int u = 0; u < kStdpUnroll; ++u) {
      const int k = k0 + u * kStdpThreads;
      const Rec r = rr[u];
      if (k >= end || __float_as_uint(r.w) == 0x80000000u) continue;
      const uint32_t pre = r.meta & 0xFFFFFu;
      const int d = static_cast<int>((r.meta >> 20) & 63u) + 1;
      const uint32_t pl = r.meta >> 26;
      const uint64_t hq = hpost[pl];
      float change = 0.f;
      if (d + a.window <= 64) {
        if (hq & 1ull) {
          const uint32_t m = static_cast<uint32_t>(hp[u] >> d) & wmask;
          if (m) change += a.ltp[__builtin_ctz(m)];
        }
        if ((hp[u] >> d) & 1ull) {
          const uint32_t m = static_cast<uint32_t>(hq >> 1) & wmask;
          if (m) change -= a.ltd[__builtin_ctz(m)];
        }
      } else {
        const uint32_t post = static_cast<uint32_t>(g) * kGroup + pl;
        if (hq & 1ull) {
          for (int lag = 0; lag < a.window; ++lag) {
            const int tau = t - lag - d;
            if (tau < 0) break;
            if (bit(tau, pre)) {
              change += a.ltp[lag];
              break;
            }
          }
        }
        if (t - d >= 0 && bit(t - d, pre)) {
          for (int lag = 1; lag <= a.window; ++lag) {
            if (t - lag < 0) break;
            if (bit(t - lag, post)) {
              change -= a.ltd[lag - 1];
              break;
            }
          }
        }
      }
      const float w = fminf(fmaxf(r.w + change, a.w_min), a.w_max);
      if (__float_as_uint(w) != __float_as_uint(r.w)) a.recs[k].w = w;
    }
  }
}

// History words before step t0: buffer (t0 - 1) & 1 gets, for every neuron,
// bit k = spike at t0 - 1 - k (zero before step 0), from the raster.
__global__ void k_hist_build(const StdpArgs a, int t0) {
  const DevNet& n = a.n;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n.Npad) return;
  uint64_t h = 0ull;
  for (int k = 0; k < 64; ++k) {
    const int tau = t0 - 1 - k;
    if (tau < 0) break;
    h |= ((n.raster[row_word(n, tau, 0, i >> 6)] >> (i & 63)) & 1ull) << k;
  }
  a.hist[static_cast<size_t>((t0 - 1) & 1) * n.Npad + i] = h;
}

constexpr size_t kStdpRowLimit = 128 * 1024;  // raster row of 2^20 neurons

hipError_t launch_stdp(const StdpArgs& a, int32_t t, hipStream_t s) {
  const size_t lds = static_cast<size_t>(a.n.G) * sizeof(uint64_t);
  if (lds > kStdpRowLimit || !a.hist || a.chunk < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_stdp, dim3(a.n.G, a.chunks), dim3(kStdpThreads), lds, s, a, t);
  return hipGetLastError();
}

hipError_t launch_hist_build(const StdpArgs& a, int32_t t0, hipStream_t s) {
  hipLaunchKernelGGL(k_hist_build, dim3((a.n.Npad + 255) / 256), dim3(256), 0, s, a, t0);
  return hipGetLastError();
}

hipError_t prepare_stdp_kernel() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stdp), hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(kStdpRowLimit));
}

constexpr size_t kStepRingLimit = 64 * 1024;

static size_t step_ring_bytes(const DevNet& n) { return static_cast<size_t>(n.D) * 2 * n.G * sizeof(uint32_t); }

template <int WAVES, int U, bool STDP>
static hipError_t launch_step_t(const DevNet& n, int32_t t, const StdpArgs& sa, int apply, hipStream_t s) {
  const size_t ring = step_ring_bytes(n);
  if (ring <= kStepRingLimit) {
    hipLaunchKernelGGL((k_step<WAVES, U, true, STDP>), dim3(n.G, n.B), dim3(WAVES * 64), ring, s, n, t, sa, apply);
  } else {
    hipLaunchKernelGGL((k_step<WAVES, U, false, STDP>), dim3(n.G, n.B), dim3(WAVES * 64), 0, s, n, t, sa, apply);
  }
  return hipGetLastError();
}

static hipError_t device_cus(int& cus) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return e;
}

hipError_t prepare_step_kernel(const DevNet& n) {
  const size_t ring = step_ring_bytes(n);
  if (ring > kStepRingLimit) {
    int cus = 0;
    const hipError_t e = device_cus(cus);
    return e != hipSuccess ? e : prepare_wide_kernel(n, cus);
  }
  const void* fns[] = {reinterpret_cast<const void*>(&k_step<16, 8, true, false>),
                       reinterpret_cast<const void*>(&k_step<4, 8, true, false>),
                       reinterpret_cast<const void*>(&k_step<1, 4, true, false>),
                       reinterpret_cast<const void*>(&k_step<16, 8, true, true>),
                       reinterpret_cast<const void*>(&k_step<4, 8, true, true>),
                       reinterpret_cast<const void*>(&k_step<1, 4, true, true>)};
  for (const void* f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(ring));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_step(const DevNet& n, int32_t t, hipStream_t s) {
  if (step_ring_bytes(n) > kStepRingLimit) {
    // the history rows do not fit one group's workgroup: workgroups of
    // several groups stage them phase by phase (wide.hip), one per CU
    int cus = 0;
    const hipError_t e = device_cus(cus);
    return e != hipSuccess ? e : launch_step_wide(n, t, cus, s);
  }
  // enough waves per group that every lane has its U records in one pass
  const int per_group = n.G > 0 ? (static_cast<int>(n.nnz / n.G) + 1) : 1;
  const StdpArgs none{};
  if (per_group > 4 * 64 * 8) return launch_step_t<16, 8, false>(n, t, none, 0, s);
  if (per_group > 64 * 4) return launch_step_t<4, 8, false>(n, t, none, 0, s);
  return launch_step_t<1, 4, false>(n, t, none, 0, s);
}

hipError_t launch_step_stdp(const StdpArgs& a, int32_t t, int apply, hipStream_t s) {
  const DevNet& n = a.n;
  if (n.B != 1 || !a.hist) return hipErrorInvalidValue;
  const int per_group = n.G > 0 ? (static_cast<int>(n.nnz / n.G) + 1) : 1;
  if (per_group > 4 * 64 * 8) return launch_step_t<16, 8, true>(n, t, a, apply, s);
  if (per_group > 64 * 4) return launch_step_t<4, 8, true>(n, t, a, apply, s);
  return launch_step_t<1, 4, true>(n, t, a, apply, s);
}

// ---------------------------------------------------------------------------
// State reset: V = r, refractory counters 0, for every trial.
// ---------------------------------------------------------------------------
__global__ void k_reset_state(const DevNet n) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t total = static_cast<size_t>(n.B) * n.Npad;
  if (i < total) {
    n.V[i] = n.reset[i % n.Npad];
    n.ref[i] = 0;
  }
}

hipError_t launch_reset_state(const DevNet& n, hipStream_t s) {
  const size_t total = static_cast<size_t>(n.B) * n.Npad;
  const unsigned blocks = static_cast<unsigned>((total + 255) / 256);
  hipLaunchKernelGGL(k_reset_state, dim3(blocks), dim3(256), 0, s, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Input repack: device bits [B][steps][ceil(N/32)] u32 -> ext rows
// [t0 + i][b][G] u64 (bits of neurons >= N cleared).
// ---------------------------------------------------------------------------
__global__ void k_repack_input(const DevNet n, int t0, int steps, const uint32_t* __restrict__ bits, uint64_t* ext) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t total = static_cast<size_t>(n.B) * steps * n.G;
  if (i >= total) return;
  const int g = static_cast<int>(i % n.G);
  const size_t bt = i / n.G;
  const int tt = static_cast<int>(bt % steps);
  const int b = static_cast<int>(bt / steps);
  const int W32 = (n.N + 31) / 32;
  const uint32_t* src = bits + (static_cast<size_t>(b) * steps + tt) * W32;
  const uint32_t lo = (2 * g < W32) ? src[2 * g] : 0u;
  const uint32_t hi = (2 * g + 1 < W32) ? src[2 * g + 1] : 0u;
  uint64_t v = (static_cast<uint64_t>(hi) << 32) | lo;
  const int valid = n.N - g * kGroup;  // neurons of this group that exist
  if (valid < 64) v &= (valid <= 0) ? 0ull : ((1ull << valid) - 1ull);
  ext[row_word(n, t0 + tt, b, g)] = v;
}

hipError_t launch_repack_input(const DevNet& n, int32_t t0, int32_t steps, const uint32_t* bits, hipStream_t s) {
  const size_t total = static_cast<size_t>(n.B) * steps * n.G;
  if (total == 0) return hipSuccess;
  const unsigned blocks = static_cast<unsigned>((total + 255) / 256);
  hipLaunchKernelGGL(k_repack_input, dim3(blocks), dim3(256), 0, s, n, t0, steps, bits,
                     const_cast<uint64_t*>(n.ext));
  return hipGetLastError();
}

}  // namespace snmi
