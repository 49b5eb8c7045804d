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
// Spike exchange.  Every step each workgroup also publishes its spike words,
// 32 spikes per 64-bit word tagged with the step: (t + 1) << 32 | bits, stored
// with one device-scope relaxed atomic in the mailbox ring [D+1][B][2G].
// Because tag and data share one atomic location, a reader that sees tag
// t + 1 sees that step's bits; no cache writeback or invalidate is needed.
// A workgroup first delivers its delay >= 2 synapses (history it already
// holds), then reads row t - 1, waiting on any word whose tag is not yet
// t, then delivers its delay-1 synapses.  A slice runs at most one step ahead of the slowest,
// so a slot is never rewritten before every reader is done with it.  Without
// an LDS ring the bits are read from the mailbox ring itself.  Every wait is
// bounded: after kSpinLimit polls the workgroup records a timeout in *status
// and all its waves exit; slices waiting on it then time out the same way.
//
// Thread tid owns the neurons of local groups wave + k * nwave (k < NPT), so
// the ballot of a wave is the spike word of one group.
// ---------------------------------------------------------------------------
constexpr uint32_t kSpinLimit = 1u << 22;

__device__ __forceinline__ uint64_t load_dev(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_dev(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Delivers the chunks [c, c_end) of the calling wave's share (every nwave-th
// chunk): four independent record / bit / accumulate chains per lane.  When
// records stream from global memory, the next chunk's records are loaded
// while the current one is processed.
// Header of chunk c: from LDS (lhdr[c - hoff]) when staged there, else global.
struct Hdr {
  const uint2* lhdr;
  int hoff;
  bool in_lds;
};

template <bool RECS_LDS>
__device__ __forceinline__ void load_chunk(const DevNet& n, const Rec* lrec, const Hdr& hdr, int c, int lane, int r0,
                                           Rec (&rc)[4], int& lg_g, int& cnt) {
  const uint2 ch = hdr.in_lds ? hdr.lhdr[c - hdr.hoff] : n.chunks[c];
  const int start = static_cast<int>(ch.x);
  lg_g = static_cast<int>(ch.y & 0xFFFFFu);
  cnt = static_cast<int>(ch.y >> 20);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = lane + 64 * u;
    rc[u] = Rec{0.f, 0u};
    if (i < cnt) rc[u] = RECS_LDS ? lrec[start - r0 + i] : n.recs[start + i];
  }
}

// Chunk headers come from LDS when the slice's headers were staged there, so
// a record load never waits on a dependent global load.
template <bool RECS_LDS, bool RING_LDS>
__device__ __forceinline__ void deliver(const DevNet& n, const Rec* lrec, const Hdr& hdr, const uint32_t* ring,
                                        const uint64_t* mring, float* acc, int c, int c_end, int nwave,
                                        int lane, int g0, int r0, int t, int cur, int Dr, int W32) {
  if (c >= c_end) return;
  Rec rc[4];
  int g = 0, cnt = 0;
  load_chunk<RECS_LDS>(n, lrec, hdr, c, lane, r0, rc, g, cnt);
  for (; c < c_end; c += nwave) {
    Rec nx[4];
    int ng = 0, ncnt = 0;
    if (!RECS_LDS && c + nwave < c_end) load_chunk<RECS_LDS>(n, lrec, hdr, c + nwave, lane, r0, nx, ng, ncnt);
    uint32_t bit[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t m = rc[u].meta;
      const int d = static_cast<int>((m >> 20) & 63u) + 1;
      const uint32_t pre = m & 0xFFFFFu;
      bit[u] = 0u;
      if (lane + 64 * u < cnt && t - d >= 0) {
        int slot = cur - d;
        if (slot < 0) slot += Dr;
        const uint32_t word = RING_LDS ? ring[slot * W32 + (pre >> 5)]
                                       : static_cast<uint32_t>(load_dev(mring + static_cast<size_t>(slot) * n.B * W32 + (pre >> 5)));
        bit[u] = (word >> (pre & 31u)) & 1u;
      }
    }
    const int lg = g - g0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (bit[u]) atomicAdd(&acc[lg * kGroup + (rc[u].meta >> 26)], rc[u].w);
    }
    if (c + nwave < c_end) {
      if (RECS_LDS) {
        load_chunk<RECS_LDS>(n, lrec, hdr, c + nwave, lane, r0, rc, g, cnt);
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) rc[u] = nx[u];
        g = ng;
        cnt = ncnt;
      }
    }
  }
}

template <int NPT, bool RECS_LDS, bool RING_LDS, bool MULTI>
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
  const int cA0 = a.wg_chunk[w], cA1 = a.wg_chunk[w + 1];
  const int cB0 = a.wg_chunk[a.P + 1 + w], cB1 = a.wg_chunk[a.P + 1 + w + 1];
  const int r0 = n.gptr[g0];
  const int nrec = n.gptr[g0 + ng] - r0;
  const bool use_mail = MULTI || !RING_LDS;
  // mailbox ring of this trial: slot s at mring + s * B * W32
  uint64_t* mring = a.mailbox + static_cast<size_t>(b) * W32;

  uint32_t* ring = reinterpret_cast<uint32_t*>(smem);
  float* acc = reinterpret_cast<float*>(ring + (RING_LDS ? Dr * W32 : 0));
  uint2* lhdr = reinterpret_cast<uint2*>(acc + a.ng_max * kGroup);  // offsets are multiples of 8 bytes
  Rec* lrec = reinterpret_cast<Rec*>(lhdr + (a.hdr_lds ? a.max_chunks : 0));
  // chunk headers of both parts: part A at lhdr[0 .. nA), part B after it
  const int nA = cA1 - cA0;
  const Hdr hA{lhdr, cA0, a.hdr_lds != 0};
  const Hdr hB{lhdr + nA, cB0, a.hdr_lds != 0};

  if (tid == 0) abort_flag = 0;
  __syncthreads();
  if (RING_LDS) {
    for (int i = tid; i < Dr * W32; i += nthr) ring[i] = 0u;
  }
  for (int i = tid; i < ng * kGroup; i += nthr) acc[i] = 0.f;
  if (RECS_LDS) {
    for (int i = tid; i < nrec; i += nthr) lrec[i] = n.recs[r0 + i];
  }
  if (a.hdr_lds) {
    for (int i = tid; i < nA; i += nthr) lhdr[i] = n.chunks[cA0 + i];
    for (int i = tid; i < cB1 - cB0; i += nthr) lhdr[nA + i] = n.chunks[cB0 + i];
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
      }
    }
  }

  float V[NPT], th[NPT], lam[NPT], rs[NPT], amp[NPT];
  int ref[NPT], R[NPT];
  uint64_t ew[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int lg = wave + k * nwave;
    V[k] = 0.f; ref[k] = 0; th[k] = 0.f; lam[k] = 0.f; rs[k] = 0.f; amp[k] = 0.f; R[k] = 0; ew[k] = 0ull;
    if (lg < ng) {
      const int j = (g0 + lg) * kGroup + lane;
      V[k] = n.V[static_cast<size_t>(b) * n.Npad + j];
      ref[k] = n.ref[static_cast<size_t>(b) * n.Npad + j];
      th[k] = n.theta[j];
      lam[k] = n.leak[j];
      rs[k] = n.reset[j];
      amp[k] = n.amp[j];
      R[k] = n.refr[j];
      if (steps > 0) ew[k] = n.ext[row_word(n, t0, b, g0 + lg)];
    }
  }
  __syncthreads();

  for (int t = t0; t < t0 + steps; ++t) {
    uint64_t ew_next[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int lg = wave + k * nwave;
      ew_next[k] = (lg < ng && t + 1 < t0 + steps) ? n.ext[row_word(n, t + 1, b, g0 + lg)] : 0ull;
    }
    const int cur = t % Dr;
    // receive row t - 1: every word carries its step tag.  The first read of
    // this thread's word is issued before the delay >= 2 delivery, which
    // hides its latency; a word whose tag is not yet t is read again.
    const int prev = (t > 0 ? t - 1 : 0) % Dr;
    const bool receive = MULTI && t > t0;
    uint64_t early = 0;
    if (receive && tid < W32) early = load_dev(mring + static_cast<size_t>(prev) * n.B * W32 + tid);
    // delay >= 2: every needed row is already held
    deliver<RECS_LDS, RING_LDS>(n, lrec, hA, ring, mring, acc, cA0 + wave, cA1, nwave, lane, g0, r0, t, cur, Dr, W32);
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
      }
    }
    __syncthreads();
    if (MULTI && abort_flag) return false;  // uniform: read after the barrier
    // delay 1
    deliver<RECS_LDS, RING_LDS>(n, lrec, hB, ring, mring, acc, cB0 + wave, cB1, nwave, lane, g0, r0, t, cur, Dr, W32);
    __syncthreads();
    // fused neuron update; the ballot of a wave is the spike word of its group
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int lg = wave + k * nwave;
      if (lg < ng) {  // uniform per wave
        const float syn = acc[lg * kGroup + lane];
        acc[lg * kGroup + lane] = 0.f;
        const bool s = lif_update(V[k], ref[k], syn, (ew[k] >> lane) & 1ull, th[k], lam[k], rs[k], amp[k], R[k]);
        const uint64_t sw = __ballot(s);
        const int g = g0 + lg;
        if (lane == 0) n.raster[row_word(n, t, b, g)] = sw;
        if (RING_LDS && lane < 2) ring[cur * W32 + 2 * g + lane] = static_cast<uint32_t>(sw >> (32 * lane));
        if (use_mail && lane < 2) {
          const uint64_t tagged = (static_cast<uint64_t>(t + 1) << 32) | ((sw >> (32 * lane)) & 0xFFFFFFFFull);
          store_dev(mring + static_cast<size_t>(cur) * n.B * W32 + 2 * g + lane, tagged);
        }
      }
      ew[k] = ew_next[k];
    }
    __syncthreads();
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

template <int NPT, bool RECS_LDS, bool RING_LDS, bool MULTI>
__global__ __launch_bounds__(1024) void k_sim(const SimArgs a, int t0, int steps) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int abort_flag;
  const int w = MULTI ? static_cast<int>(blockIdx.x) : 0;
  const int b = MULTI ? static_cast<int>(blockIdx.y) : static_cast<int>(blockIdx.x);
  sim_body<NPT, RECS_LDS, RING_LDS, MULTI>(a, w, b, t0, steps, smem, abort_flag);
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
__global__ __launch_bounds__(kBatchThreads, 4) void k_batch(const BatchArgs ba, int steps) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int abort_flag;
  __shared__ int next;
  if (static_cast<int>(blockIdx.x) < ba.n_team) {
    const int4 tt = ba.team[blockIdx.x];
    const SimArgs a = ba.nets[tt.x].team;
    if (!sim_body<kBatchMaxGroups / (kBatchThreads / 64), false, true, true>(a, tt.y, tt.z, tt.w, steps, smem,
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
    sim_body<kBatchMaxGroups / (kBatchThreads / 64), false, true, false>(a, 0, qt.y, qt.z, steps, smem, abort_flag);
  }
}

size_t batch_lds_bytes(const DevNet& n, int ng_max, int max_chunks) {
  return static_cast<size_t>(n.D + 1) * 2 * n.G * sizeof(uint32_t) + static_cast<size_t>(ng_max) * kGroup * sizeof(float) +
         static_cast<size_t>(max_chunks) * sizeof(uint2);
}

int batch_blocks_per_cu(size_t lds) {
  int blocks = 0;
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch), hipFuncAttributeMaxDynamicSharedMemorySize,
                          static_cast<int>(lds)) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch, kBatchThreads, lds) != hipSuccess) return 0;
  return blocks;
}

hipError_t launch_batch(const BatchArgs& a, int grid, size_t lds, int32_t steps, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch), hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(lds));
  if (e != hipSuccess) return e;
  void* args[] = {const_cast<BatchArgs*>(&a), &steps};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_batch), dim3(grid), dim3(kBatchThreads), args,
                                    static_cast<unsigned>(lds), s);
}

__global__ void k_zero_i32(int32_t* p) { *p = 0; }

hipError_t launch_zero_i32(int32_t* p, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, s, p);
  return hipGetLastError();
}

constexpr size_t kLdsLimit = 160 * 1024;
constexpr int kMaxNpt = 8;

size_t sim_lds_bytes(const DevNet& n, int ng_max, int64_t max_recs, int max_chunks, bool recs_lds, bool ring_lds,
                     bool hdr_lds) {
  size_t bytes = static_cast<size_t>(ng_max) * kGroup * sizeof(float);
  if (hdr_lds) bytes += static_cast<size_t>(max_chunks) * sizeof(uint2);
  if (ring_lds) bytes += static_cast<size_t>(n.D + 1) * 2 * n.G * sizeof(uint32_t);
  if (recs_lds) bytes += static_cast<size_t>(max_recs) * sizeof(Rec);
  return bytes + 64;  // static LDS of the kernel
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

template <int NPT, bool RL, bool GL, bool MULTI>
static hipError_t launch_sim_t(const SimArgs& a, int32_t t0, int32_t steps, hipStream_t s, size_t lds) {
  const void* fn = reinterpret_cast<const void*>(&k_sim<NPT, RL, GL, MULTI>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(kLdsLimit - 64));
  if (e != hipSuccess) return e;
  const dim3 block(sim_threads(a.ng_max, a.max_recs));
  if (MULTI) {
    const dim3 grid(a.P, a.n.B);
    void* args[] = {const_cast<SimArgs*>(&a), &t0, &steps};
    return hipLaunchCooperativeKernel(fn, grid, block, args, static_cast<unsigned>(lds), s);
  }
  hipLaunchKernelGGL((k_sim<NPT, RL, GL, MULTI>), dim3(a.n.B), block, lds, s, a, t0, steps);
  return hipGetLastError();
}

template <bool MULTI>
static hipError_t launch_sim_m(const SimArgs& a, bool rl, bool gl, int32_t t0, int32_t steps, hipStream_t s,
                               size_t lds) {
  const int npt = sim_npt(a.ng_max, a.max_recs);
  const int np2 = npt <= 1 ? 1 : npt <= 2 ? 2 : npt <= 4 ? 4 : 8;
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
  const size_t lds = sim_lds_bytes(a.n, a.ng_max, a.max_recs, a.max_chunks, recs_lds, ring_lds, a.hdr_lds != 0) - 64;
  if (lds + 64 > kLdsLimit) return hipErrorInvalidValue;
  if (a.P > 1 || !ring_lds) {
    const hipError_t e = launch_prefill_mailbox(a, t0, s);
    if (e != hipSuccess) return e;
  }
  if (a.P > 1) return launch_sim_m<true>(a, recs_lds, ring_lds, t0, steps, s, lds);
  return launch_sim_m<false>(a, recs_lds, ring_lds, t0, steps, s, lds);
}


// ---------------------------------------------------------------------------
// Per-step pull kernel: workgroup (g, b) accumulates, for trial b, the
// delayed input of the 64 posts of group g.  It loads the group's records
// (coalesced 8-byte loads, U per lane in flight) and, at the same time, the D
// previous raster rows into LDS when they fit (RING), so each record costs
// one global round trip; the source bit of row t - d is then an LDS read and
// w is added into an LDS accumulator.  Wave 0 applies the neuron update and
// writes the group's spike word.
// ---------------------------------------------------------------------------
template <int WAVES, int U, bool RING>
__global__ __launch_bounds__(WAVES * 64) void k_step(const DevNet n, int t) {
  __shared__ float acc[kGroup];
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
  for (;;) {
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
      if (bit[u]) atomicAdd(&acc[rr[u].meta >> 26], rr[u].w);
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
  __syncthreads();
  if (wave == 0) {
    const bool s = lif_update(V, ref, acc[lane], (ew >> lane) & 1ull, th, lam, rs, amp, R);
    const uint64_t sw = __ballot(s);
    const size_t sj = static_cast<size_t>(b) * n.Npad + j;
    n.V[sj] = V;
    n.ref[sj] = static_cast<uint8_t>(ref);
    if (lane == 0) n.raster[row_word(n, t, b, g)] = sw;
  }
}

constexpr size_t kStepRingLimit = 64 * 1024;

static size_t step_ring_bytes(const DevNet& n) { return static_cast<size_t>(n.D) * 2 * n.G * sizeof(uint32_t); }

template <int WAVES, int U>
static hipError_t launch_step_t(const DevNet& n, int32_t t, hipStream_t s) {
  const size_t ring = step_ring_bytes(n);
  if (ring <= kStepRingLimit) {
    hipLaunchKernelGGL((k_step<WAVES, U, true>), dim3(n.G, n.B), dim3(WAVES * 64), ring, s, n, t);
  } else {
    hipLaunchKernelGGL((k_step<WAVES, U, false>), dim3(n.G, n.B), dim3(WAVES * 64), 0, s, n, t);
  }
  return hipGetLastError();
}

hipError_t prepare_step_kernel(const DevNet& n) {
  const size_t ring = step_ring_bytes(n);
  if (ring > kStepRingLimit) return hipSuccess;
  const void* fns[] = {reinterpret_cast<const void*>(&k_step<16, 8, true>),
                       reinterpret_cast<const void*>(&k_step<4, 8, true>),
                       reinterpret_cast<const void*>(&k_step<1, 4, true>)};
  for (const void* f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(ring));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_step(const DevNet& n, int32_t t, hipStream_t s) {
  // enough waves per group that every lane has its U records in one pass
  const int per_group = n.G > 0 ? (static_cast<int>(n.nnz / n.G) + 1) : 1;
  if (per_group > 4 * 64 * 8) return launch_step_t<16, 8>(n, t, s);
  if (per_group > 64 * 4) return launch_step_t<4, 8>(n, t, s);
  return launch_step_t<1, 4>(n, t, s);
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
