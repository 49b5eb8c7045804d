// Event-driven ("push") delivery for low firing rates.
//
// Instead of streaming every incoming synapse each step (pull), only the
// synapses of neurons that spiked are touched: a spike of neuron i at step t
// adds w into the accumulator row (t + d) mod (D+1) of the post-neuron, and
// at step t each neuron consumes (and clears) row t mod (D+1).  The same
// input sums as §2.1's s(t-d) x W are formed, in a different order; with the
// dyadic inputs every order gives the same binary32 value.
//
// k_push: one persistent workgroup per (slice, trial).  Per step it
//   1. updates its own neurons (input read from the accumulator row with
//      device-scope loads, then cleared),
//   2. compacts its spiking neurons into an LDS list (wave ballot + popcount
//      reserve slots, mbcnt gives each spiking lane its slot),
//   3. streams the out-going records of the listed neurons, one wave per
//      neuron, and adds every weight with a device-scope float atomic,
//   4. waits until its own stores and atomics are complete and publishes
//      flags[w] = t + 1; then waits until every slice of its trial has
//      published t + 1 (bounded: a timeout sets *status and ends the kernel).
// The accumulator rows a slice reads at t + 1 are therefore complete.
#include <hip/hip_runtime.h>

#include "sn_device.h"
#include "sn_internal.h"

namespace snmi {

constexpr uint32_t kPushSpinLimit = 1u << 22;

__device__ __forceinline__ float load_dev_f32(const float* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_dev_f32(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int NPT, bool MULTI>
__global__ __launch_bounds__(1024) void k_push(const PushArgs a, int t0, int steps) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int abort_flag;
  __shared__ int list_count;
  const DevNet& n = a.n;
  const int w = MULTI ? static_cast<int>(blockIdx.x) : 0;
  const int b = MULTI ? static_cast<int>(blockIdx.y) : static_cast<int>(blockIdx.x);
  const int nthr = blockDim.x;
  const int nwave = nthr >> 6;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int Dr = n.D + 1;
  const int g0 = a.wg_group[w];
  const int ng = a.wg_group[w + 1] - g0;
  int* list = reinterpret_cast<int*>(smem);  // [ng_max * 64] spiking neurons of this step
  const size_t rowstride = static_cast<size_t>(n.B) * n.Npad;
  float* acc_b = a.accum + static_cast<size_t>(b) * n.Npad;

  if (tid == 0) {
    abort_flag = 0;
    list_count = 0;
  }
  float V[NPT], th[NPT], lam[NPT], rs[NPT], amp[NPT];
  int ref[NPT], R[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int lg = wave + k * nwave;
    V[k] = 0.f; ref[k] = 0; th[k] = 0.f; lam[k] = 0.f; rs[k] = 0.f; amp[k] = 0.f; R[k] = 0;
    if (lg < ng) {
      const int j = (g0 + lg) * kGroup + lane;
      V[k] = n.V[static_cast<size_t>(b) * n.Npad + j];
      ref[k] = n.ref[static_cast<size_t>(b) * n.Npad + j];
      th[k] = n.theta[j];
      lam[k] = n.leak[j];
      rs[k] = n.reset[j];
      amp[k] = n.amp[j];
      R[k] = n.refr[j];
    }
  }
  __syncthreads();

  for (int t = t0; t < t0 + steps; ++t) {
    const int cur = t % Dr;
    // 1-2. update own neurons, compact the spiking ones
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int lg = wave + k * nwave;
      if (lg < ng) {  // uniform per wave
        const int g = g0 + lg;
        const int j = g * kGroup + lane;
        float* slot = acc_b + static_cast<size_t>(cur) * rowstride + j;
        const float syn = load_dev_f32(slot);
        store_dev_f32(slot, 0.f);
        const uint64_t ew = n.ext[row_word(n, t, b, g)];
        const bool s = lif_update(V[k], ref[k], syn, (ew >> lane) & 1ull, th[k], lam[k], rs[k], amp[k], R[k]);
        const uint64_t sw = __ballot(s);
        if (lane == 0) n.raster[row_word(n, t, b, g)] = sw;
        if (sw) {
          int base = 0;
          if (lane == 0) base = atomicAdd(&list_count, static_cast<int>(__popcll(sw)));
          base = __shfl(base, 0);
          const int rank = static_cast<int>(__builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(sw >> 32),
                                                                       __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(sw), 0u)));
          if (s) list[base + rank] = j;
        }
      }
    }
    __syncthreads();
    // 3. deliver: one wave per spiking neuron, lanes over its out-going records
    const int cnt = list_count;
    for (int i = wave; i < cnt; i += nwave) {
      const int pre = list[i];
      const int r1 = a.optr[pre + 1];
      for (int r = a.optr[pre] + lane; r < r1; r += 64) {
        const Rec rc = a.orecs[r];
        const int d = static_cast<int>((rc.meta >> 20) & 63u) + 1;
        const int post = static_cast<int>(rc.meta & 0xFFFFFu);
        int slot = cur + d;
        if (slot >= Dr) slot -= Dr;
        atomicAdd(acc_b + static_cast<size_t>(slot) * rowstride + post, rc.w);
      }
    }
    // every store and atomic of this wave has completed
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) list_count = 0;
    if (MULTI) {
      uint32_t* flags = a.flags + static_cast<size_t>(b) * a.P * 64;
      if (tid == 0) __hip_atomic_store(&flags[w * 64], static_cast<uint32_t>(t + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (int v = tid; v < a.P; v += nthr) {
        uint32_t spins = 0;
        while (__hip_atomic_load(&flags[v * 64], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < static_cast<uint32_t>(t + 1)) {
          if (++spins > kPushSpinLimit) {
            abort_flag = 1;
            __hip_atomic_store(a.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
        }
      }
    }
    __syncthreads();
    if (MULTI && abort_flag) return;  // uniform: read after the barrier
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

// Accumulator ring before a launch starting at t0: zero, plus the pending
// input of spikes emitted at t0 - D .. t0 - 1 that arrives at t0 or later.
// Workgroup (i, g, b): one spike word (step t0 - D + i, group g, trial b);
// one wave per spiking neuron of the word.
__global__ void k_push_zero(float* accum, size_t count) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) accum[i] = 0.f;
}

__global__ void k_push_pending(const PushArgs a, int t0) {
  const DevNet& n = a.n;
  const int ts = t0 - n.D + static_cast<int>(blockIdx.x);
  const int g = blockIdx.y;
  const int b = blockIdx.z;
  if (ts < 0) return;
  const int Dr = n.D + 1;
  const uint64_t word = n.raster[row_word(n, ts, b, g)];
  const int lane = threadIdx.x;
  const size_t rowstride = static_cast<size_t>(n.B) * n.Npad;
  float* acc_b = a.accum + static_cast<size_t>(b) * n.Npad;
  for (int l = 0; l < 64; ++l) {
    if (!((word >> l) & 1ull)) continue;
    const int pre = g * kGroup + l;
    for (int r = a.optr[pre] + lane; r < a.optr[pre + 1]; r += 64) {
      const Rec rc = a.orecs[r];
      const int d = static_cast<int>((rc.meta >> 20) & 63u) + 1;
      if (ts + d < t0) continue;  // already delivered
      const int slot = (ts + d) % Dr;
      atomicAdd(acc_b + static_cast<size_t>(slot) * rowstride + (rc.meta & 0xFFFFFu), rc.w);
    }
  }
}

// Threads of a slice: one wave per group for the update, at least 4 waves
// for the delivery of spiking neurons' out-going synapses.
static int push_threads(int ng_max) {
  const int thr = ng_max * kGroup < 256 ? 256 : ng_max * kGroup;
  return thr < 1024 ? thr : 1024;
}

template <int NPT, bool MULTI>
static hipError_t launch_push_t(const PushArgs& a, int32_t t0, int32_t steps, hipStream_t s) {
  const int nthr = push_threads(a.ng_max);
  const size_t lds = static_cast<size_t>(a.ng_max) * kGroup * sizeof(int);
  const void* fn = reinterpret_cast<const void*>(&k_push<NPT, MULTI>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e != hipSuccess) return e;
  if (MULTI) {
    void* args[] = {const_cast<PushArgs*>(&a), &t0, &steps};
    return hipLaunchCooperativeKernel(fn, dim3(a.P, a.n.B), dim3(nthr), args, static_cast<unsigned>(lds), s);
  }
  hipLaunchKernelGGL((k_push<NPT, MULTI>), dim3(a.n.B), dim3(nthr), lds, s, a, t0, steps);
  return hipGetLastError();
}

hipError_t launch_push(const PushArgs& a, int32_t t0, int32_t steps, hipStream_t s) {
  const int nthr = push_threads(a.ng_max);
  const int npt = (a.ng_max + nthr / kGroup - 1) / (nthr / kGroup);
  if (npt > 8 || a.P < 1) return hipErrorInvalidValue;
  const size_t count = static_cast<size_t>(a.n.D + 1) * a.n.B * a.n.Npad;
  hipLaunchKernelGGL(k_push_zero, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0, s, a.accum, count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // flags of an earlier launch must not satisfy this launch's waits (zero bits)
  const size_t nflags = static_cast<size_t>(a.n.B) * a.P * 64;
  hipLaunchKernelGGL(k_push_zero, dim3(static_cast<unsigned>((nflags + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<float*>(a.flags), nflags);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (t0 > 0) {
    hipLaunchKernelGGL(k_push_pending, dim3(a.n.D, a.n.G, a.n.B), dim3(64), 0, s, a, t0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int np2 = npt <= 1 ? 1 : npt <= 2 ? 2 : npt <= 4 ? 4 : 8;
  const bool multi = a.P > 1;
  switch (np2 * 2 + (multi ? 1 : 0)) {
    case 2: return launch_push_t<1, false>(a, t0, steps, s);
    case 3: return launch_push_t<1, true>(a, t0, steps, s);
    case 4: return launch_push_t<2, false>(a, t0, steps, s);
    case 5: return launch_push_t<2, true>(a, t0, steps, s);
    case 8: return launch_push_t<4, false>(a, t0, steps, s);
    case 9: return launch_push_t<4, true>(a, t0, steps, s);
    case 16: return launch_push_t<8, false>(a, t0, steps, s);
    case 17: return launch_push_t<8, true>(a, t0, steps, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace snmi
