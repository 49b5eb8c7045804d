// Dense many-trial step on the matrix cores (gfx950 MFMA).
//
// For delay-1 dense weights the delivery of §2.1 is literally the matrix
// product I[B x N] = S(t-1)[B x N] x W[N x N] of the previous step's spike
// vectors (0/1) with the weight matrix.  Spikes are exact in bfloat16, and so
// are the dyadic weights accepted by sn_load_dense_weights; products are exact
// and FP32 accumulation of dyadic partial sums below 2^17 is exact, so the
// result is the unique one regardless of the order the hardware adds in.
//
// Workgroup (c, tb): 16 post-neurons (columns 16c .. 16c+15) for 64 trials
// (tb * 64 ..).  Four waves split the contraction (pre-neurons) into quarters;
// each wave keeps four 16x16 accumulators (one per 16 trials) and issues
// v_mfma_f32_16x16x32_bf16 with the weight fragment shared by the four.  The
// spike operand comes from the bit raster: one 32-bit word of a trial's bits
// feeds four MFMA steps (see the K order in DenseArgs) and each byte is
// expanded to eight bfloat16 0/1 values through a 256-entry LDS table.  The
// four partial products are summed in LDS and the fused LIF update of §2.1
// writes V, the refractory counters and 16 spike bits per trial.
#include <hip/hip_runtime.h>

#include "sn_device.h"
#include "sn_internal.h"

namespace snmi {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef int i32x4 __attribute__((ext_vector_type(4)));

constexpr int kDenseTrials = 64;  // trials per workgroup

// Eight bfloat16 {0, 1} from the bits of one byte (element e = bit e), in
// registers: dword h holds elements 2h and 2h + 1, i.e. (b0 | b1 << 16) times
// 0x3F80 (bfloat16 1.0).  Four VALU operations per dword, no LDS traffic.
// Sixteen int8 {0, 1} from a 16-bit half of a spike word (byte i = bit i):
// four bits spread into the four bytes of a dword by one multiply,
// x * 0x00204081 = x + x << 7 + x << 14 + x << 21 (no carries for x < 16).
__device__ __forceinline__ i32x4 expand_bits_i8(uint32_t half) {
  i32x4 d;
#pragma unroll
  for (int h = 0; h < 4; ++h) d[h] = static_cast<int>((((half >> (4 * h)) & 0xFu) * 0x00204081u) & 0x01010101u);
  return d;
}

__device__ __forceinline__ bf16x8 expand_bits(uint32_t byte) {
  uint32_t d[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const uint32_t b0 = (byte >> (2 * h)) & 1u, b1 = (byte >> (2 * h + 1)) & 1u;
    d[h] = (b0 | (b1 << 16)) * 0x3F80u;
  }
  return __builtin_bit_cast(bf16x8, make_uint4(d[0], d[1], d[2], d[3]));
}
constexpr int kDenseThreads = 256;

__global__ __launch_bounds__(kDenseThreads) void k_dense_step(const DenseArgs a, int t) {
  const DevNet& n = a.n;
  const int c = blockIdx.x;   // column tile: posts 16c .. 16c + 15
  const int tb = blockIdx.y;  // trials tb * 64 ..
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int q = lane >> 4;    // lane group
  const int li = lane & 15;   // row (trial) / column index inside a 16 x 16 tile
  const int kw = a.kpad / 32; // 32-bit spike words per trial row
  const int sbw = kw + 1;     // LDS row stride (odd: rows fall in different banks)
  const int J = a.kpad / 128;

  extern __shared__ __align__(16) unsigned char smem[];
  uint4* tab = reinterpret_cast<uint4*>(smem);                      // [256] 8 x bf16 {0, 1}
  float* part = reinterpret_cast<float*>(tab + 256);                // [4 waves][64 trials][17]
  uint32_t* sb = reinterpret_cast<uint32_t*>(part + 4 * kDenseTrials * 17);  // [64][sbw]

  // expansion table: bit e of byte x -> bfloat16 1.0 (0x3F80) or 0 in element e
  {
    const uint32_t x = static_cast<uint32_t>(tid);
    uint32_t wv[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      wv[h] = (((x >> (2 * h)) & 1u) ? 0x3F80u : 0u) | (((x >> (2 * h + 1)) & 1u) ? 0x3F800000u : 0u);
    }
    tab[tid] = make_uint4(wv[0], wv[1], wv[2], wv[3]);
  }
  // spike bits of step t - 1 (raster row, 32-bit view), zero past N and for t = 0
  const uint32_t* r32 = reinterpret_cast<const uint32_t*>(n.raster);
  for (int i = tid; i < kDenseTrials * sbw; i += kDenseThreads) {
    const int bl = i / sbw, wi = i % sbw;
    const int b = tb * kDenseTrials + bl;
    uint32_t v = 0u;
    if (t >= 1 && b < n.B && wi < 2 * n.G) v = r32[row_word(n, t - 1, b, 0) * 2 + wi];
    sb[i] = v;
  }
  __syncthreads();

  f32x4 acc[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int j0 = wave * J / 4, j1 = (wave + 1) * J / 4;
  const uint4* wt = reinterpret_cast<const uint4*>(a.wt) + static_cast<size_t>(c) * J * 4 * 64;
  // weight fragments of block j + 1 are loaded while block j is multiplied
  uint4 bw[4], bn[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) bw[s] = j0 < j1 ? wt[(static_cast<size_t>(j0) * 4 + s) * 64 + lane] : make_uint4(0, 0, 0, 0);
  for (int j = j0; j < j1; ++j) {
    if (j + 1 < j1) {
#pragma unroll
      for (int s = 0; s < 4; ++s) bn[s] = wt[(static_cast<size_t>(j + 1) * 4 + s) * 64 + lane];
    }
    uint32_t sw[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) sw[m] = sb[(16 * m + li) * sbw + 4 * j + q];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bf16x8 bfrag = __builtin_bit_cast(bf16x8, bw[s]);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const bf16x8 afrag = __builtin_bit_cast(bf16x8, tab[(sw[m] >> (8 * s)) & 0xFFu]);
        acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afrag, bfrag, acc[m], 0, 0, 0);
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) bw[s] = bn[s];
  }
  // lane (q, li) holds rows 4q + r of each 16 x 16 tile, column li
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) part[(wave * kDenseTrials + 16 * m + 4 * q + r) * 17 + li] = acc[m][r];
  __syncthreads();

  // fused update: wave w handles trials 16w .. 16w + 15, four per pass;
  // lane (q, li) -> trial 16w + 4k + q, column li
  const int col = 16 * c + li;
  const float th = n.theta[col], lam = n.leak[col], rs = n.reset[col], amp = n.amp[col];
  const int R = n.refr[col];
  const uint16_t* e16 = reinterpret_cast<const uint16_t*>(n.ext);
  uint16_t* o16 = reinterpret_cast<uint16_t*>(n.raster);
  const int g = c >> 2, part16 = c & 3;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int tl = 16 * wave + 4 * k + q;
    const int b = tb * kDenseTrials + tl;
    bool s = false;
    if (b < n.B) {
      float syn = 0.f;
#pragma unroll
      for (int w = 0; w < 4; ++w) syn += part[(w * kDenseTrials + tl) * 17 + li];
      const size_t sj = static_cast<size_t>(b) * n.Npad + col;
      float V = n.V[sj];
      int ref = n.ref[sj];
      const bool ext = (e16[row_word(n, t, b, g) * 4 + part16] >> li) & 1u;
      s = lif_update(V, ref, syn, ext, th, lam, rs, amp, R);
      n.V[sj] = V;
      n.ref[sj] = static_cast<uint8_t>(ref);
    }
    const uint64_t bits = __ballot(s);
    if (li == 0 && b < n.B) o16[row_word(n, t, b, g) * 4 + part16] = static_cast<uint16_t>(bits >> (16 * q));
  }
}

// ---------------------------------------------------------------------------
// Persistent dense kernel: all requested steps in one cooperative launch.
// Workgroup (c, tb) owns 16 post-neurons (columns 16c ..) for 64 trials.
// Its 16-column slice of W (kpad x 16 bfloat16, 128 KB at N = 4096) is held
// in the registers of its four waves for the whole run, each wave the
// fragments of its quarter of K (144 registers per lane at most), so the
// weights are read from HBM once per launch and never from LDS; V and the
// refractory counters stay in registers.  Each step it
//   1. issues the loads of this step's external spike bits,
//   2. waits until every workgroup of its trial block has published step t-1
//      (one flag per workgroup, 256 bytes apart, device-scope loads),
//   3. copies the spike bits of step t-1 of its 64 trials from the raster
//      into LDS with coalesced device-scope 8-byte loads,
//   4. multiplies on the matrix cores, expanding spike bits to bfloat16 in
//      registers, and sums the four K quarters through LDS,
//   5. applies the fused LIF update and writes 16 spike bits per trial
//      (device-scope 16-bit stores), waits for its stores to complete, and
//      publishes flag = t + 1.
// Waits are bounded (a timeout sets *status and every wave exits; the other
// workgroups then time out the same way).
// ---------------------------------------------------------------------------
constexpr uint32_t kDenseSpinLimit = 1u << 22;
// K blocks of 128 per wave: J / 4 <= 9, i.e. kpad <= 4608 (N <= 4608).
constexpr int kMaxJPerWave = 9;
// 64-bit spike words a thread stages per step: 64 trials x kpad / 64 / 256
constexpr int kStageLoads = kDenseTrials * (4 * kMaxJPerWave * 128 / 64) / kDenseThreads;

// I8: int8 numerators on v_mfma_i32_16x16x64_i8 (see DenseArgs), else bfloat16.
template <bool I8>
__global__ __launch_bounds__(kDenseThreads) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_dense_persist(const DenseArgs a, uint32_t* flags, uint32_t* status, int t0, int steps) {
  const DevNet& n = a.n;
  const int c = blockIdx.x;
  const int tb = blockIdx.y;
  const int ncol = gridDim.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int q = lane >> 4;
  const int li = lane & 15;
  const int J = a.kpad / 128;
  const int kw = a.kpad / 32;  // 32-bit spike words per trial row
  const int sbw = kw + 4;      // LDS row stride: rows 4 banks apart

  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int abort_flag;
  float* part = reinterpret_cast<float*>(smem);                             // [4][64][17]
  uint32_t* sb = reinterpret_cast<uint32_t*>(part + 4 * kDenseTrials * 17);  // [64][sbw] spike words of t - 1

  // this wave's weight fragments: K blocks j0 .. j1 - 1, 4 steps each
  const int j0 = wave * J / 4, j1 = (wave + 1) * J / 4;
  constexpr int S = I8 ? 2 : 4;  // matrix-core steps per K block of 128
  const uint4* wsrc = I8 ? reinterpret_cast<const uint4*>(a.wt8) + static_cast<size_t>(c) * J * 2 * 64
                         : reinterpret_cast<const uint4*>(a.wt) + static_cast<size_t>(c) * J * 4 * 64;
  uint4 wreg[kMaxJPerWave][S];
#pragma unroll
  for (int jj = 0; jj < kMaxJPerWave; ++jj)
#pragma unroll
    for (int s = 0; s < S; ++s) wreg[jj][s] = j0 + jj < j1 ? wsrc[((j0 + jj) * S + s) * 64 + lane] : make_uint4(0, 0, 0, 0);
  const float scale = I8 ? a.scale8 : 1.f;
  if (tid == 0) abort_flag = 0;

  // neuron state: lane (q, li) of wave w, pass k -> trial 16w + 4k + q, column li
  const int col = 16 * c + li;
  const float th = n.theta[col], lam = n.leak[col], rs = n.reset[col], amp = n.amp[col];
  const int R = n.refr[col];
  float V[4];
  int ref[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int b = tb * kDenseTrials + 16 * wave + 4 * k + q;
    V[k] = 0.f;
    ref[k] = 0;
    if (b < n.B) {
      V[k] = n.V[static_cast<size_t>(b) * n.Npad + col];
      ref[k] = n.ref[static_cast<size_t>(b) * n.Npad + col];
    }
  }
  __syncthreads();

  const uint16_t* e16 = reinterpret_cast<const uint16_t*>(n.ext);
  uint16_t* o16 = reinterpret_cast<uint16_t*>(n.raster);
  uint32_t* myflags = flags + static_cast<size_t>(tb) * ncol * 64;
  const int g = c >> 2, part16 = c & 3;

  for (int t = t0; t < t0 + steps; ++t) {
    // this step's external spike bits, issued before the wait
    uint32_t ext16[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int b = tb * kDenseTrials + 16 * wave + 4 * k + q;
      ext16[k] = b < n.B ? e16[row_word(n, t, b, g) * 4 + part16] : 0u;
    }
    if (t > t0) {
      for (int v = tid; v < ncol; v += kDenseThreads) {
        uint32_t spins = 0;
        while (__hip_atomic_load(&myflags[v * 64], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < static_cast<uint32_t>(t)) {
          if (++spins > kDenseSpinLimit) {
            abort_flag = 1;
            __hip_atomic_store(status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
        }
      }
      __syncthreads();
      if (abort_flag) return;  // uniform: read after the barrier
    }
    f32x4 acc[4];
    i32x4 acc8[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
      acc8[m] = i32x4{0, 0, 0, 0};
    }
    if (t >= 1) {
      // spike words of step t - 1 of the 64 trials, 64-bit words coalesced;
      // all of a thread's loads are issued before the first LDS store
      const int nw64 = kw / 2;
      uint64_t v[kStageLoads];
#pragma unroll
      for (int e = 0; e < kStageLoads; ++e) {
        const int i = tid + kDenseThreads * e;
        const int tr = i / nw64, w = i - tr * nw64;
        const int b = tb * kDenseTrials + tr;
        v[e] = 0;
        if (i < kDenseTrials * nw64 && b < n.B && w < n.G)
          v[e] = __hip_atomic_load(&n.raster[row_word(n, t - 1, b, w)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
#pragma unroll
      for (int e = 0; e < kStageLoads; ++e) {
        const int i = tid + kDenseThreads * e;
        const int tr = i / nw64, w = i - tr * nw64;
        if (i < kDenseTrials * nw64) {
          sb[tr * sbw + 2 * w] = static_cast<uint32_t>(v[e]);
          sb[tr * sbw + 2 * w + 1] = static_cast<uint32_t>(v[e] >> 32);
        }
      }
      __syncthreads();
#pragma unroll
      for (int jj = 0; jj < kMaxJPerWave; ++jj) {
        const int j = j0 + jj;
        if (j >= j1) break;  // uniform
        uint32_t sw[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) sw[m] = sb[(16 * m + li) * sbw + 4 * j + q];
        if constexpr (I8) {
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const i32x4 bfrag = __builtin_bit_cast(i32x4, wreg[jj][s]);
#pragma unroll
            for (int m = 0; m < 4; ++m)
              acc8[m] = __builtin_amdgcn_mfma_i32_16x16x64_i8(expand_bits_i8((sw[m] >> (16 * s)) & 0xFFFFu), bfrag,
                                                              acc8[m], 0, 0, 0);
          }
        } else {
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const bf16x8 bfrag = __builtin_bit_cast(bf16x8, wreg[jj][s]);
#pragma unroll
            for (int m = 0; m < 4; ++m)
              acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(expand_bits((sw[m] >> (8 * s)) & 0xFFu), bfrag, acc[m],
                                                               0, 0, 0);
          }
        }
      }
    }
    // partial sums (int8 path: integers below 2^24, exact as floats)
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        part[(wave * kDenseTrials + 16 * m + 4 * q + r) * 17 + li] = I8 ? static_cast<float>(acc8[m][r]) : acc[m][r];
    __syncthreads();
    // the external bits, taken before this step's first store (a load
    // consumed after a store would wait for that store to complete)
    uint32_t em = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) em |= ((ext16[k] >> li) & 1u) << k;
    // all four updates first, then one store for the four words (a store
    // between updates would make the next one wait for it)
    uint32_t word16[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int tl = 16 * wave + 4 * k + q;
      const int b = tb * kDenseTrials + tl;
      bool s = false;
      if (b < n.B) {
        float syn = 0.f;
#pragma unroll
        for (int w = 0; w < 4; ++w) syn += part[(w * kDenseTrials + tl) * 17 + li];
        syn *= scale;  // a power of two: exact
        const bool ext = (em >> k) & 1u;
        s = lif_update(V[k], ref[k], syn, ext, th, lam, rs, amp, R);
      }
      word16[k] = static_cast<uint32_t>(__ballot(s) >> (16 * q)) & 0xFFFFu;
    }
    {  // one store instruction: lane (q, k) writes the word of trial 16 w + 4 k + q
      const uint32_t mine = li == 0 ? word16[0] : li == 1 ? word16[1] : li == 2 ? word16[2] : word16[3];
      const int b = tb * kDenseTrials + 16 * wave + 4 * li + q;
      if (li < 4 && b < n.B)
        __hip_atomic_store(&o16[row_word(n, t, b, g) * 4 + part16], static_cast<uint16_t>(mine), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    // publish step t once this workgroup's spike words are complete
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0)
      __hip_atomic_store(&myflags[c * 64], static_cast<uint32_t>(t + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int b = tb * kDenseTrials + 16 * wave + 4 * k + q;
    if (b < n.B) {
      n.V[static_cast<size_t>(b) * n.Npad + col] = V[k];
      n.ref[static_cast<size_t>(b) * n.Npad + col] = static_cast<uint8_t>(ref[k]);
    }
  }
}

size_t dense_persist_lds_bytes(int32_t kpad) {
  if (kpad / 128 > 4 * kMaxJPerWave) return static_cast<size_t>(1) << 30;  // weights do not fit in registers
  return 4 * kDenseTrials * 17 * sizeof(float) + static_cast<size_t>(kDenseTrials) * (kpad / 32 + 4) * sizeof(uint32_t);
}

__global__ void k_dense_clear_flags(uint32_t* flags, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) flags[i] = 0u;
}

// Cooperative launch when every workgroup fits on the device at once;
// returns hipErrorCooperativeLaunchTooLarge otherwise (the caller falls back
// to per-step launches).
hipError_t launch_dense_persist(const DenseArgs& a, uint32_t* flags, uint32_t* status, int32_t t0, int32_t steps,
                                hipStream_t s) {
  const size_t lds = dense_persist_lds_bytes(a.kpad);
  if (a.kpad / 128 > 4 * kMaxJPerWave) return hipErrorInvalidValue;  // weights would not fit in registers
  const void* fn = a.wt8 ? reinterpret_cast<const void*>(&k_dense_persist<true>)
                         : reinterpret_cast<const void*>(&k_dense_persist<false>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e != hipSuccess) return e;
  const dim3 grid(a.n.Npad / 16, (a.n.B + kDenseTrials - 1) / kDenseTrials);
  const int nflags = static_cast<int>(grid.x * grid.y * 64);
  hipLaunchKernelGGL(k_dense_clear_flags, dim3((nflags + 255) / 256), dim3(256), 0, s, flags, nflags);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  void* args[] = {const_cast<DenseArgs*>(&a), &flags, &status, &t0, &steps};
  return hipLaunchCooperativeKernel(fn, grid, dim3(kDenseThreads), args, static_cast<unsigned>(lds), s);
}

size_t dense_lds_bytes(int32_t kpad) {
  return 256 * sizeof(uint4) + 4 * kDenseTrials * 17 * sizeof(float) +
         static_cast<size_t>(kDenseTrials) * (kpad / 32 + 1) * sizeof(uint32_t);
}

hipError_t launch_dense_step(const DenseArgs& a, int32_t t, hipStream_t s) {
  const size_t lds = dense_lds_bytes(a.kpad);
  const dim3 grid(a.n.Npad / 16, (a.n.B + kDenseTrials - 1) / kDenseTrials);
  hipLaunchKernelGGL(k_dense_step, grid, dim3(kDenseThreads), lds, s, a, t);
  return hipGetLastError();
}

hipError_t prepare_dense_kernel(int32_t kpad) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dense_step), hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(dense_lds_bytes(kpad)));
}

}  // namespace snmi
