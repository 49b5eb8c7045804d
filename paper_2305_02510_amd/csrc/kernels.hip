// HIP kernels for gfx950: pull delivery of delayed spikes and the fused
// leak / integrate / threshold / refractory / reset update of §2.1.
#include <hip/hip_runtime.h>

#include "sn_internal.h"

namespace snmi {

// ---------------------------------------------------------------------------
// Neuron update (§2.1, steps 1 and 3-6; step 2's sum arrives in `syn`).
// All operands are binary32; with dyadic inputs every operation is exact.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float leak_toward(float v, float r, float lam) {
  if (v > r) return fmaxf(v - lam, r);
  if (v < r) return fminf(v + lam, r);
  return v;
}

__device__ __forceinline__ bool lif_update(float& V, int& ref, float syn, bool ext, float theta, float lam,
                                           float r, float amp, int R) {
  float U = leak_toward(V, r, lam);
  U = U + syn;
  if (ext) U = U + amp;
  const bool cand = U > theta;
  bool s;
  if (ref > 0) {
    s = false;
    ref = ref - 1;
  } else {
    s = cand;
  }
  if (s) {
    V = r;
    ref = R;
  } else {
    V = U;
  }
  return s;
}

__device__ __forceinline__ size_t row_word(const DevNet& n, int64_t t, int b, int g) {
  return (static_cast<size_t>(t) * n.B + b) * n.G + g;
}

// ---------------------------------------------------------------------------
// Persistent kernel: runs `steps` time steps in one launch.
//
// Workgroup (w, b) owns the contiguous post-neuron groups [g0, g1) of slice w
// for trial b: their records (copied to LDS when they fit) and their neuron
// state (registers).  The spike history of the last D steps is a ring of D+1
// bit rows in LDS when it fits (slot t mod (D+1) holds step t; step t reads
// the slots of t - d, d = 1..D, never its own), else it is read from the
// raster in global memory.
//
// With several slices (MULTI), the workgroups of a trial exchange each step's
// spike words through the raster: a workgroup writes its words, publishes
// `flags[b][w] = t + 1` with an agent-scope release, waits until every slice
// of its trial has published t + 1 (relaxed agent-scope polls, then an
// agent-scope acquire fence), and copies row t into its ring.  A slice can run
// at most one step ahead of the slowest one.  Every wait is bounded: after
// kSpinLimit polls the workgroup records a timeout in *status and all of its
// waves exit; the slices waiting on it then time out the same way.
//
// Thread tid owns the neurons of local groups wave + k * nwave (k < NPT), so
// the ballot of a wave is the spike word of one group.
// ---------------------------------------------------------------------------
constexpr uint32_t kSpinLimit = 1u << 22;

template <int NPT, bool RECS_LDS, bool RING_LDS, bool MULTI>
__global__ __launch_bounds__(1024) void k_sim(const SimArgs a, int t0, int steps) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int abort_flag;
  const DevNet& n = a.n;
  const int w = MULTI ? static_cast<int>(blockIdx.x) : 0;
  const int b = MULTI ? static_cast<int>(blockIdx.y) : static_cast<int>(blockIdx.x);
  const int nthr = blockDim.x;
  const int nwave = nthr >> 6;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int Dr = n.D + 1;
  const int W32 = 2 * n.G;
  const int g0 = a.wg_group[w];
  const int ng = a.wg_group[w + 1] - g0;
  const int c0 = a.wg_chunk[w];
  const int c1 = a.wg_chunk[w + 1];
  const int r0 = n.gptr[g0];
  const int nrec = n.gptr[g0 + ng] - r0;

  uint32_t* ring = reinterpret_cast<uint32_t*>(smem);
  float* acc = reinterpret_cast<float*>(ring + (RING_LDS ? Dr * W32 : 0));
  Rec* lrec = reinterpret_cast<Rec*>(acc + a.ng_max * kGroup);  // offsets are multiples of 8 bytes
  const size_t rstride = static_cast<size_t>(n.B) * n.G;
  const uint64_t* hist = n.raster + static_cast<size_t>(b) * n.G;

  if (tid == 0) abort_flag = 0;
  if (RING_LDS) {
    for (int i = tid; i < Dr * W32; i += nthr) ring[i] = 0u;
  }
  for (int i = tid; i < ng * kGroup; i += nthr) acc[i] = 0.f;
  if (RECS_LDS) {
    for (int i = tid; i < nrec; i += nthr) lrec[i] = n.recs[r0 + i];
  }
  __syncthreads();
  if (RING_LDS) {  // history of the steps before t0 (rows < 0 stay zero)
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
    // delivery: chunk c goes to wave (c - c0) mod nwave; a chunk holds at
    // most kChunk = 4 * 64 records, processed as four independent
    // record / bit / accumulate chains per lane
    for (int c = c0 + wave; c < c1; c += nwave) {
      const uint2 ch = n.chunks[c];
      const int start = static_cast<int>(ch.x);
      const int lg = static_cast<int>(ch.y & 0xFFFFFu) - g0;
      const int cnt = static_cast<int>(ch.y >> 20);
      Rec rc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = lane + 64 * u;
        rc[u] = Rec{0.f, 0u};
        if (i < cnt) rc[u] = RECS_LDS ? lrec[start - r0 + i] : n.recs[start + i];
      }
      uint32_t bit[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t m = rc[u].meta;
        const int d = static_cast<int>((m >> 20) & 63u) + 1;
        const uint32_t pre = m & 0xFFFFFu;
        bit[u] = 0u;
        if (lane + 64 * u < cnt && t - d >= 0) {
          if (RING_LDS) {
            int slot = cur - d;
            if (slot < 0) slot += Dr;
            bit[u] = (ring[slot * W32 + (pre >> 5)] >> (pre & 31u)) & 1u;
          } else {
            bit[u] = static_cast<uint32_t>(hist[static_cast<size_t>(t - d) * rstride + (pre >> 6)] >> (pre & 63u)) & 1u;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (bit[u]) atomicAdd(&acc[lg * kGroup + (rc[u].meta >> 26)], rc[u].w);
      }
    }
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
        if (lane == 0) {
          const int g = g0 + lg;
          n.raster[row_word(n, t, b, g)] = sw;
          if (RING_LDS) {
            ring[cur * W32 + 2 * g] = static_cast<uint32_t>(sw);
            ring[cur * W32 + 2 * g + 1] = static_cast<uint32_t>(sw >> 32);
          }
        }
      }
      ew[k] = ew_next[k];
    }
    if (MULTI) {
      __syncthreads();  // every spike word of this workgroup is written
      uint32_t* flags = a.flags + static_cast<size_t>(b) * a.P;
      if (tid == 0) __hip_atomic_store(&flags[w], static_cast<uint32_t>(t + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      for (int v = tid; v < a.P; v += nthr) {
        uint32_t spins = 0;
        while (__hip_atomic_load(&flags[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < static_cast<uint32_t>(t + 1)) {
          if (++spins > kSpinLimit) {
            abort_flag = 1;
            __hip_atomic_store(a.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
        }
      }
      __syncthreads();
      if (abort_flag) return;  // uniform: every thread sees the flag after the barrier
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (RING_LDS) {
        for (int i = tid; i < n.G; i += nthr) {
          const uint64_t wv = hist[static_cast<size_t>(t) * rstride + i];
          ring[cur * W32 + 2 * i] = static_cast<uint32_t>(wv);
          ring[cur * W32 + 2 * i + 1] = static_cast<uint32_t>(wv >> 32);
        }
      }
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
}

constexpr size_t kLdsLimit = 160 * 1024;
constexpr int kMaxNpt = 8;

size_t sim_lds_bytes(const DevNet& n, int ng_max, int64_t max_recs, bool recs_lds, bool ring_lds) {
  size_t bytes = static_cast<size_t>(ng_max) * kGroup * sizeof(float);
  if (ring_lds) bytes += static_cast<size_t>(n.D + 1) * 2 * n.G * sizeof(uint32_t);
  if (recs_lds) bytes += static_cast<size_t>(max_recs) * sizeof(Rec);
  return bytes + 64;  // static LDS of the kernel
}

size_t lds_limit() { return kLdsLimit; }

int sim_threads(int ng_max) { return ng_max * kGroup < 1024 ? ng_max * kGroup : 1024; }

int sim_npt(int ng_max) {
  const int nw = sim_threads(ng_max) / kGroup;
  return (ng_max + nw - 1) / nw;
}

template <int NPT, bool RL, bool GL, bool MULTI>
static hipError_t launch_sim_t(const SimArgs& a, int32_t t0, int32_t steps, hipStream_t s, size_t lds) {
  const void* fn = reinterpret_cast<const void*>(&k_sim<NPT, RL, GL, MULTI>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(kLdsLimit - 64));
  if (e != hipSuccess) return e;
  const dim3 block(sim_threads(a.ng_max));
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
  const int npt = sim_npt(a.ng_max);
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
  if (sim_npt(a.ng_max) > kMaxNpt) return hipErrorInvalidValue;
  const size_t lds = sim_lds_bytes(a.n, a.ng_max, a.max_recs, recs_lds, ring_lds) - 64;
  if (lds + 64 > kLdsLimit) return hipErrorInvalidValue;
  if (a.P > 1) return launch_sim_m<true>(a, recs_lds, ring_lds, t0, steps, s, lds);
  return launch_sim_m<false>(a, recs_lds, ring_lds, t0, steps, s, lds);
}

__global__ void k_clear_u32(uint32_t* p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0u;
}

hipError_t launch_clear_u32(uint32_t* p, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_clear_u32, dim3((count + 255) / 256), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-step pull kernel: workgroup (g, b) accumulates, for trial b, the
// delayed input of the 64 posts of group g by streaming the group's records
// (coalesced 8-byte loads, U records per lane in flight), testing the
// pre-neuron's bit in raster row t - d, and adding w into an LDS accumulator.
// Wave 0 then applies the neuron update and writes the group's spike word.
// ---------------------------------------------------------------------------
template <int WAVES, int U>
__global__ __launch_bounds__(WAVES * 64) void k_step(const DevNet n, int t) {
  __shared__ float acc[kGroup];
  const int g = blockIdx.x;
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int j = g * kGroup + lane;

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
  __syncthreads();

  const int beg = n.gptr[g];
  const int end = n.gptr[g + 1];
  const size_t rstride = static_cast<size_t>(n.B) * n.G;
  const uint64_t* hist = n.raster + static_cast<size_t>(b) * n.G;
  for (int base = beg + wave * 64 * U; base < end; base += WAVES * 64 * U) {
    Rec rr[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = base + u * 64 + lane;
      ok[u] = k < end;
      rr[u] = ok[u] ? n.recs[k] : Rec{0.f, 0u};
    }
    uint64_t word[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t m = rr[u].meta;
      const int ts = t - static_cast<int>((m >> 20) & 63u) - 1;
      ok[u] = ok[u] && ts >= 0;
      word[u] = ok[u] ? hist[static_cast<size_t>(ts) * rstride + ((m & 0xFFFFFu) >> 6)] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t m = rr[u].meta;
      if ((word[u] >> (m & 63u)) & 1ull) atomicAdd(&acc[m >> 26], rr[u].w);
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

hipError_t launch_step(const DevNet& n, int32_t t, hipStream_t s) {
  // enough waves per group to keep every lane busy with U = 4 records
  const int per_group = n.G > 0 ? (static_cast<int>(n.nnz / n.G) + 1) : 1;
  if (per_group > 8 * 64 * 4) {
    hipLaunchKernelGGL((k_step<16, 4>), dim3(n.G, n.B), dim3(1024), 0, s, n, t);
  } else if (per_group > 2 * 64 * 4) {
    hipLaunchKernelGGL((k_step<4, 4>), dim3(n.G, n.B), dim3(256), 0, s, n, t);
  } else {
    hipLaunchKernelGGL((k_step<1, 4>), dim3(n.G, n.B), dim3(64), 0, s, n, t);
  }
  return hipGetLastError();
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
