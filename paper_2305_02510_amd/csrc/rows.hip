// Event-driven dense delivery for large nets with few trials ("rows" path).
//
// With delay-1 dense weights the input of step t is I = s(t-1) x W (§2.1):
// for one trial, the sum of the rows of W that belong to the neurons that
// spiked at t - 1.  At the paper's largest size (100,000 neurons all-to-all,
// §4) W does not fit on chip, and reading all of it every step would move
// N^2 bytes; reading only the spiking rows moves (spikes) x N bytes.  W is
// held row-major in HBM as int8 numerators k, W = k * 2^-e, so each row is a
// contiguous stream and the sums are exact integers.
//
// One launch per step.  Workgroup (x, b) owns posts 256x .. 256x + 255 of
// trial b (lane l of every wave holds posts 256x + 4l .. + 3, one 32-bit load
// per row).  It
//   1. lists the spiking pre-neurons of step t - 1 from the raster row in LDS
//      (popcount, block scan, then every thread writes the indices of its
//      words), in rounds of at most kRowsCap neurons;
//   2. streams the listed rows of its 256 columns, the waves splitting the
//      list, kRowsUnroll rows in flight per wave, summing the int8 weights in
//      32-bit integer registers;
//   3. adds the waves' sums in LDS, scales by 2^-e (exact: |sum| < 2^24) and
//      applies the fused LIF update, writing V, the refractory counters and the
//      spike word of every 64 posts.
#include <hip/hip_runtime.h>

#include "sn_device.h"
#include "sn_internal.h"

namespace snmi {

constexpr int kRowsThreads = 512;
constexpr int kRowsWaves = kRowsThreads / 64;
constexpr int kRowsSlab = 256;   // posts per workgroup: 64 lanes x 4 int8 weights
constexpr int kRowsCap = 8192;   // spiking neurons listed per round
constexpr int kRowsUnroll = 16;  // rows in flight per wave
constexpr int kRowsWordsPerThread = 4;
static_assert(kRowsThreads * kRowsWordsPerThread * 64 >= kRowsMaxNeurons, "raster row must fit one pass");

__device__ __forceinline__ void add_bytes(int (&acc)[4], uint32_t v) {
  const int x = static_cast<int>(v);
  acc[0] += (x << 24) >> 24;
  acc[1] += (x << 16) >> 24;
  acc[2] += (x << 8) >> 24;
  acc[3] += x >> 24;
}

__global__ __launch_bounds__(kRowsThreads) void k_dense_rows(const RowsArgs a, int32_t t) {
  const DevNet& n = a.n;
  const int b = blockIdx.y;
  const int slab0 = blockIdx.x * kRowsSlab;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ int32_t list[kRowsCap];
  __shared__ int4 part[kRowsWaves][64];
  __shared__ int32_t wtot[kRowsWaves];

  int acc[4] = {0, 0, 0, 0};
  const bool lane_cols = slab0 + 4 * lane < n.Npad;  // Npad is a multiple of 64
  if (t > 0) {
    // 1. spiking neurons of step t - 1: thread tid owns raster words
    //    4 tid .. 4 tid + 3; bits of neurons >= N are cleared so that no row
    //    outside W is ever listed
    const uint64_t* prev = n.raster + row_word(n, t - 1, b, 0);
    const int g0 = tid * kRowsWordsPerThread;
    uint64_t word[kRowsWordsPerThread];
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < kRowsWordsPerThread; ++q) {
      const int g = g0 + q;
      uint64_t x = g < n.G ? prev[g] : 0ull;
      const int hi = n.N - 64 * g;  // valid bits of this word
      if (hi < 64) x = hi <= 0 ? 0ull : (x & ((1ull << hi) - 1ull));
      word[q] = x;
      cnt += __popcll(x);
    }
    int incl = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(incl, off);
      if (lane >= off) incl += y;
    }
    if (lane == 63) wtot[wave] = incl;
    __syncthreads();
    int before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kRowsWaves; ++w) {
      const int v = wtot[w];
      before += w < wave ? v : 0;
      total += v;
    }
    const int pos0 = before + incl - cnt;
    const uint32_t lane_off = 4u * lane + static_cast<uint32_t>(slab0);
    for (int r0 = 0; r0 < total; r0 += kRowsCap) {
      if (r0 > 0) __syncthreads();  // the previous round has finished reading the list
      if (pos0 < r0 + kRowsCap && pos0 + cnt > r0) {
        int pos = pos0;
#pragma unroll
        for (int q = 0; q < kRowsWordsPerThread; ++q) {
          uint64_t x = word[q];
          while (x) {
            const int bit = __builtin_ctzll(x);
            x &= x - 1ull;
            if (pos >= r0 && pos < r0 + kRowsCap) list[pos - r0] = 64 * (g0 + q) + bit;
            ++pos;
          }
        }
      }
      __syncthreads();
      // 2. rows of the listed neurons, columns of this workgroup.  A list
      //    entry is the same for the whole wave: its row address is scalar.
      const int m = min(total - r0, kRowsCap);
      if (lane_cols) {
        int e = wave * kRowsUnroll;
        for (; e + kRowsUnroll <= m; e += kRowsWaves * kRowsUnroll) {
          uint32_t v[kRowsUnroll];
#pragma unroll
          for (int u = 0; u < kRowsUnroll; ++u) {
            const uint32_t i = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(list[e + u]));
            v[u] = *reinterpret_cast<const uint32_t*>(a.w8 + static_cast<uint64_t>(i) * a.pitch + lane_off);
          }
#pragma unroll
          for (int u = 0; u < kRowsUnroll; ++u) add_bytes(acc, v[u]);
        }
        if (e < m) {  // last, partial block of this wave
          for (int u = 0; e + u < m; ++u) {
            const uint32_t i = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(list[e + u]));
            add_bytes(acc, *reinterpret_cast<const uint32_t*>(a.w8 + static_cast<uint64_t>(i) * a.pitch + lane_off));
          }
        }
      }
    }
  }
  // 3. sum over waves, update
  part[wave][lane] = make_int4(acc[0], acc[1], acc[2], acc[3]);
  __syncthreads();
  if (tid < kRowsSlab) {
    const int j = slab0 + tid;
    if (j < n.Npad) {  // uniform per wave
      const int* pw = reinterpret_cast<const int*>(&part[0][0]);
      int sum = 0;
#pragma unroll
      for (int w = 0; w < kRowsWaves; ++w) sum += pw[w * kRowsSlab + tid];
      const float syn = static_cast<float>(sum) * a.scale;
      const size_t sj = static_cast<size_t>(b) * n.Npad + j;
      float V = n.V[sj];
      int ref = n.ref[sj];
      const int g = j >> 6;
      const bool ext = (n.ext[row_word(n, t, b, g)] >> lane) & 1ull;
      const bool s = lif_update(V, ref, syn, ext, n.theta[j], n.leak[j], n.reset[j], n.amp[j], n.refr[j]);
      const uint64_t sw = __ballot(s);
      n.V[sj] = V;
      n.ref[sj] = static_cast<uint8_t>(ref);
      if (lane == 0) n.raster[row_word(n, t, b, g)] = sw;
    }
  }
}

hipError_t launch_dense_rows(const RowsArgs& a, int32_t t, hipStream_t s) {
  if (a.n.N > kRowsMaxNeurons || a.pitch < a.n.Npad) return hipErrorInvalidValue;
  const dim3 grid((a.n.Npad + kRowsSlab - 1) / kRowsSlab, a.n.B);
  hipLaunchKernelGGL(k_dense_rows, grid, dim3(kRowsThreads), 0, s, a, t);
  return hipGetLastError();
}

}  // namespace snmi
