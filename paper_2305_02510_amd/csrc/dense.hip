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

constexpr int kDenseTrials = 64;  // trials per workgroup
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
