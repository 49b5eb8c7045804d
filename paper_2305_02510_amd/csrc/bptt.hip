// Surrogate-gradient backpropagation through time for a recurrent LIF layer
// (the model of §2.1 with delay-1 recurrent weights, input through W_in and
// no refractory period), on FP32 matrix cores (v_mfma_f32_16x16x4_f32) and,
// for the spike term of the hard forward product, on bfloat16 ones.
//
//   U_t = leak(V_{t-1}) + [s_{t-1} | x_t] W_cat      W_cat = [W_rec ; W_in]
//   s_t = H(U_t - theta)  (relaxed: 1/2 + x / (1 + k|x|), x = U_t - theta)
//   V_t = (1 - s_t) U_t + s_t r
// The threshold's derivative is the fast-sigmoid surrogate 1/(1 + k|x|)^2,
// the exact derivative of the relaxed spike; the clamped leak passes the
// gradient where it does not clamp (|V - r| > lambda).  Backward, with
// dL/ds_t = dL/dcount (a spike count is a sum over steps):
//   g_t = (dL/dcount + g_{t+1} W_rec^T) sigma'_t
//         + [|V_t - r| > lambda] g_{t+1} ((1 - s_t) + (r - U_t) sigma'_t)
//   dW_cat = sum_t [s_{t-1} | x_t]^T g_t
//
// All three products use one tile scheme: a workgroup of 4 waves computes a
// 64 x 64 output tile, K in chunks of 64 staged through two LDS buffers, each
// wave 2 x 2 accumulators of 16 x 16.  The per-step products (128 trials:
// few output tiles) split K over several workgroups and a small epilogue
// kernel sums the parts in a fixed order and applies the step.  Operand
// layout of v_mfma_f32_16x16x4_f32: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; the result D[4 (l/16) + r][l % 16], r = 0..3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "../../include/superneuro_mi.h"
#include "sn_internal.h"

namespace snmi {

// Forward workspace of sn_bptt_forward_noalloc, for callers that cannot
// allocate: one copy on every device the library runs on, alive until the
// process ends, shared by every call on that device.  Host code never passes
// this name to a kernel (on the host it is only a stand-in for the symbol):
// it uses the device address that hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[SN_BPTT_NOALLOC_WORKSPACE_BYTES];

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

struct BpttDev {
  int32_t N, Nin, B;
  float theta, leak, reset, slope;
  int32_t relaxed;
};

__device__ __forceinline__ float leak_clamped(float v, float r, float lam) {
  if (v > r) return fmaxf(v - lam, r);
  if (v < r) return fminf(v + lam, r);
  return v;
}

__device__ __forceinline__ float surrogate_grad(float x, float k) {
  const float d = 1.f + k * fabsf(x);
  return 1.f / (d * d);
}

// 64 x 64 tile of a row-major product, K staged 64 at a time through two
// LDS buffers with the next chunk prefetched into registers.  Wave (wr, wc)
// owns the 32 x 32 quarter (32 wr .., 32 wc ..) as 2 x 2 accumulators of
// 16 x 16, so every pair of operand reads feeds two matrix-core operations.
// acc[rb][cb] element r is (row0 + 32 wr + 16 rb + 4 (lane/16) + r,
// col0 + 32 wc + 16 cb + lane % 16).
constexpr int kT64 = 64;
struct Acc64 {
  f32x4 v[2][2];
};

template <class AL, class BL>
__device__ __forceinline__ Acc64 tile_product64(int k0, int K, AL Aload, BL Bload, float (*As)[64][kT64 + 4],
                                                float (*Bs)[kT64][80]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  Acc64 acc;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc.v[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // element e of this thread's share: A (row idx / 64, k idx % 64), B (k idx / 64, col idx % 64)
  constexpr int kPer = 64 * kT64 / 256;
  float ra[kPer], rb[kPer];
  auto fetch = [&](int kc) {
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int idx = tid + 256 * e;
      ra[e] = Aload(idx >> 6, kc + (idx & 63));
      rb[e] = Bload(kc + (idx >> 6), idx & 63);
    }
  };
  fetch(k0);
  int buf = 0;
  for (int kc = k0; kc < K; kc += kT64) {
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int idx = tid + 256 * e;
      As[buf][idx >> 6][idx & 63] = ra[e];
      Bs[buf][idx >> 6][idx & 63] = rb[e];
    }
    __syncthreads();
    if (kc + kT64 < K) fetch(kc + kT64);
#pragma unroll
    for (int kk = 0; kk < kT64; kk += 4) {
      float av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        av[i] = As[buf][32 * wr + 16 * i + (lane & 15)][kk + (lane >> 4)];
        bv[i] = Bs[buf][kk + (lane >> 4)][32 * wc + 16 * i + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc.v[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc.v[i][j], 0, 0, 0);
    }
    buf ^= 1;
  }
  return acc;
}

// Per-step products, K split over gridDim.z workgroups (each a multiple of
// kT64): tile (cols 64 blockIdx.x .., trials 64 blockIdx.y ..) of part z
// of   forward:  [s_prev | x_t] W_cat   (s_prev null: no spikes yet)
//      backward: g_next W_rec^T          (WrT = W_rec^T)
// written to part[z][B][N]; the epilogue kernels sum the parts in a fixed
// order.
template <bool FWD>
__global__ __launch_bounds__(256) void k_bptt_part(const BpttDev p, const float* __restrict__ Bm,
                                                   const float* s_prev, const float* __restrict__ x_t, int kc,
                                                   float* __restrict__ part) {
  __shared__ float As[2][64][kT64 + 4];  // row strides 68 and 80 words: the
  __shared__ float Bs[2][kT64][80];      // matrix-core operand reads are 2-way in the 32 banks
  const int col0 = 64 * blockIdx.x, row0 = 64 * blockIdx.y;
  const int N = p.N, Nin = p.Nin, B = p.B, K = FWD ? N + Nin : N;
  const int k0 = blockIdx.z * kc, k1 = min(K, k0 + kc);
  auto Aload = [&](int r, int k) -> float {
    const int b = row0 + r;
    if (b >= B || k >= k1) return 0.f;
    if (!FWD) return s_prev[static_cast<size_t>(b) * N + k];  // g_next
    if (k < N) return s_prev ? s_prev[static_cast<size_t>(b) * N + k] : 0.f;
    return x_t[static_cast<size_t>(b) * Nin + (k - N)];
  };
  auto Bload = [&](int k, int c) -> float {
    const int j = col0 + c;
    return (k < k1 && j < N) ? Bm[static_cast<size_t>(k) * N + j] : 0.f;
  };
  Acc64 acc;
  if (FWD ? (s_prev || k1 > N) : true) {
    acc = tile_product64(k0, k1, Aload, Bload, As, Bs);
  } else {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc.v[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  float* out = part + static_cast<size_t>(blockIdx.z) * B * N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int b = row0 + 32 * wr + 16 * i + 4 * (lane >> 4) + r;
        const int col = col0 + 32 * wc + 16 * j + (lane & 15);
        if (b < B && col < N) out[static_cast<size_t>(b) * N + col] = acc.v[i][j][r];
      }
}

// ---------------------------------------------------------------------------
// Hard-spike forward on bfloat16 matrix cores.  The spikes s_{t-1} are 0 or
// 1, exact in bfloat16, and W_rec splits exactly into three bfloat16 pieces,
// W = hi + mid + lo (each the leading 8 significand bits of what the previous
// pieces leave), so s W_rec = sum over the pieces of s piece: every product is
// exact and only the FP32 accumulation rounds, as in the FP32 product.  The
// pieces are stored transposed and concatenated along K: wsT[j][p N + k] =
// piece p of W_rec[k][j], a contraction of length 3N per output.
// v_mfma_f32_16x16x32_bf16 operands: lane l holds A[l % 16][8 (l/16) + e] and
// B[8 (l/16) + e][l % 16], e = 0..7; D as the FP32 16 x 16 x 4 form.
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;

__device__ __forceinline__ void split3(float w, uint16_t& hi, uint16_t& mid, uint16_t& lo) {
  const uint32_t u = __float_as_uint(w);
  hi = static_cast<uint16_t>(u >> 16);
  const float r1 = w - __uint_as_float(u & 0xFFFF0000u);  // exact: the low 16 significand bits
  const uint32_t u1 = __float_as_uint(r1);
  mid = static_cast<uint16_t>(u1 >> 16);
  const float r2 = r1 - __uint_as_float(u1 & 0xFFFF0000u);  // exact, at most 8 significant bits
  lo = static_cast<uint16_t>(__float_as_uint(r2) >> 16);
}

// wsT [N][3 Np] from W_rec = the first N rows of W_cat [N + Nin][N], Np = N
// rounded up to 64 (entries k in [N, Np) of each piece are zero); 64 x 64
// tiles through LDS so that reads and writes are both along rows.
// Grid (ceil(N / 64), Np / 64).
__global__ __launch_bounds__(256) void k_split_weights(const float* __restrict__ W, uint16_t* __restrict__ wsT, int N,
                                                       int Np) {
  __shared__ float tile[64][65];
  const int k0 = 64 * blockIdx.y, j0 = 64 * blockIdx.x;
  for (int i = threadIdx.x; i < 64 * 64; i += 256) {
    const int r = i >> 6, c = i & 63;
    tile[r][c] = (k0 + r < N && j0 + c < N) ? W[static_cast<size_t>(k0 + r) * N + j0 + c] : 0.f;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 64 * 64; i += 256) {
    const int c = i >> 6, r = i & 63;  // output row j0 + c, column k0 + r of each piece
    if (j0 + c < N) {
      uint16_t h, m, l;
      split3(tile[r][c], h, m, l);
      uint16_t* row = wsT + static_cast<size_t>(j0 + c) * 3 * Np + k0 + r;
      row[0] = h;
      row[Np] = m;
      row[2 * Np] = l;
    }
  }
}

// bit-packed spikes [B][N/16] u16 -> bfloat16 0 / 1 [B][Np]
__global__ void k_bits_to_bf16(const uint16_t* __restrict__ bits, uint16_t* out, int B, int N, int Np) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= static_cast<size_t>(B) * N) return;
  const size_t b = i / N, n = i - b * N;
  out[b * Np + n] = ((bits[i / 16] >> (i % 16)) & 1u) ? 0x3F80u : 0u;
}

__global__ void k_zero_u16(uint16_t* p, size_t count) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0u;
}

// C[r][c] (= or +=) sum over k' < 3P of A[r][k' mod P] Bt[c][k'] on bfloat16
// matrix cores, A [R][P] (0 / 1 spikes) and Bt [C][3P] (three pieces of an
// FP32 operand, transposed), P a multiple of 64; 64 x 64 tiles, the
// contraction split over gridDim.z in chunks of kcs (a multiple of 64, so no
// chunk straddles two pieces); C row stride ldc, part z at C + z zstride.
// Used for the forward spike term s_{t-1} W_rec (A = spikes [B][Np], Bt =
// pieces of W_rec) and the weight gradient of W_rec (A = spikes transposed
// [N][Mp], Bt = pieces of the segment's g transposed).  A null: zero.
__global__ __launch_bounds__(256) void k_gemm_split(const uint16_t* A, int R, int P, const uint16_t* __restrict__ Bt,
                                                    int C, int kcs, float* __restrict__ Cm, int ldc, size_t zstride,
                                                    int accumulate) {
  const int col0 = 64 * blockIdx.x, row0 = 64 * blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  Acc64 acc;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc.v[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  if (A) {
    // LDS rows of 64 bf16 (+8 pad, 144 bytes: 16-byte aligned, operand reads
    // spread over the banks)
    __shared__ __attribute__((aligned(16))) uint16_t Ah[2][64][72];
    __shared__ __attribute__((aligned(16))) uint16_t Bh[2][64][72];
    const int K3 = 3 * P;
    const int k0 = blockIdx.z * kcs, k1 = min(K3, k0 + kcs);
    // staging share of a thread: row (of A and of Bt) tid / 4, k' 16 (tid % 4) .. + 15
    const int sr = threadIdx.x >> 2, sk = 16 * (threadIdx.x & 3);
    const int ra_row = row0 + sr, rb_row = col0 + sr;
    uint4 ra[2], rb[2];
    auto fetch = [&](int kc) {
      const int kp = kc + sk;
      const int k = kp % P;  // the 16 entries are k .. k + 15 of one piece
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        ra[h] = ra_row < R ? *reinterpret_cast<const uint4*>(A + static_cast<size_t>(ra_row) * P + k + 8 * h)
                           : make_uint4(0u, 0u, 0u, 0u);
        rb[h] = rb_row < C ? *reinterpret_cast<const uint4*>(Bt + static_cast<size_t>(rb_row) * K3 + kp + 8 * h)
                           : make_uint4(0u, 0u, 0u, 0u);
      }
    };
    fetch(k0);
    int buf = 0;
    for (int kc = k0; kc < k1; kc += kT64) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        *reinterpret_cast<uint4*>(&Ah[buf][sr][sk + 8 * h]) = ra[h];
        *reinterpret_cast<uint4*>(&Bh[buf][sr][sk + 8 * h]) = rb[h];
      }
      __syncthreads();
      if (kc + kT64 < k1) fetch(kc + kT64);
#pragma unroll
      for (int kk = 0; kk < kT64; kk += 32) {
        bf16x8 av[2], bv[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          av[i] = *reinterpret_cast<const bf16x8*>(&Ah[buf][32 * wr + 16 * i + (lane & 15)][kk + 8 * (lane >> 4)]);
          bv[i] = *reinterpret_cast<const bf16x8*>(&Bh[buf][32 * wc + 16 * i + (lane & 15)][kk + 8 * (lane >> 4)]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int jj = 0; jj < 2; ++jj)
            acc.v[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[jj], acc.v[i][jj], 0, 0, 0);
      }
      buf ^= 1;
    }
  }
  float* out = Cm + blockIdx.z * zstride;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = row0 + 32 * wr + 16 * i + 4 * (lane >> 4) + r;
        const int cc = col0 + 32 * wc + 16 * jj + (lane & 15);
        if (rr < R && cc < C) {
          float* o = out + static_cast<size_t>(rr) * ldc + cc;
          *o = accumulate ? *o + acc.v[i][jj][r] : acc.v[i][jj][r];
        }
      }
}

// Transposed bfloat16 copies of a segment for the weight gradient (hard
// mode), 64 x 64 tiles through LDS, grid (ceil(cols / 64), Mp / 64):
//   spikes: At[k][m] = A_seg[m][k] (0 / 1), k < N (the W_rec rows of A)
//   g:      Gt[j][p Mp + m] = piece p of g_seg[m][j]
// rows m in [M, Mp) are zero.
__global__ __launch_bounds__(256) void k_seg_transpose(const float* __restrict__ Aseg, int KA, const float* __restrict__ G,
                                                       int N, int M, int Mp, uint16_t* __restrict__ At,
                                                       uint16_t* __restrict__ Gt) {
  __shared__ float ta[64][65];
  __shared__ float tg[64][65];
  const int c0 = 64 * blockIdx.x, m0 = 64 * blockIdx.y;
  for (int i = threadIdx.x; i < 64 * 64; i += 256) {
    const int r = i >> 6, c = i & 63;
    const bool ok = m0 + r < M && c0 + c < N;
    ta[r][c] = ok ? Aseg[static_cast<size_t>(m0 + r) * KA + c0 + c] : 0.f;
    tg[r][c] = ok ? G[static_cast<size_t>(m0 + r) * N + c0 + c] : 0.f;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 64 * 64; i += 256) {
    const int c = i >> 6, r = i & 63;  // output row c0 + c, column m0 + r
    if (c0 + c < N) {
      At[static_cast<size_t>(c0 + c) * Mp + m0 + r] = static_cast<uint16_t>(__float_as_uint(ta[r][c]) >> 16);
      uint16_t h, md, l;
      split3(tg[r][c], h, md, l);
      uint16_t* row = Gt + static_cast<size_t>(c0 + c) * 3 * Mp + m0 + r;
      row[0] = h;
      row[Mp] = md;
      row[2 * Mp] = l;
    }
  }
}

// Input term of every step at once (hard mode): XW [T B][N] = X [T B][Nin]
// times W_in (rows N .. N + Nin - 1 of W_cat), FP32 matrix cores, one 64 x 64
// tile per workgroup.
__global__ __launch_bounds__(256) void k_bptt_xw(const BpttDev p, int M, const float* __restrict__ X,
                                                 const float* __restrict__ W, float* __restrict__ XW) {
  __shared__ float As[2][64][kT64 + 4];
  __shared__ float Bs[2][kT64][80];
  const int col0 = 64 * blockIdx.x, row0 = 64 * blockIdx.y;
  const int N = p.N, Nin = p.Nin;
  auto Aload = [&](int r, int k) -> float {
    const int m = row0 + r;
    return (m < M && k < Nin) ? X[static_cast<size_t>(m) * Nin + k] : 0.f;
  };
  auto Bload = [&](int k, int c) -> float {
    const int j = col0 + c;
    return (k < Nin && j < N) ? W[static_cast<size_t>(N + k) * N + j] : 0.f;
  };
  const Acc64 acc = tile_product64(0, Nin, Aload, Bload, As, Bs);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = row0 + 32 * wr + 16 * i + 4 * (lane >> 4) + r;
        const int col = col0 + 32 * wc + 16 * jj + (lane & 15);
        if (m < M && col < N) XW[static_cast<size_t>(m) * N + col] = acc.v[i][jj][r];
      }
}

// Forward epilogue of step t, one thread per (trial, neuron), element
// e = b N + n: U = leak(V_prev) + sum of the parts, the spike (hard or
// relaxed), V, the spike count; optionally U and bit-packed spikes (64
// consecutive elements per wave ballot, written as 16-bit pieces) and the A
// row [s_prev | x_t] of the step (A_keep [B][N + Nin]).
__global__ __launch_bounds__(256) void k_bptt_fwd_epi(const BpttDev p, const float* __restrict__ part, int nparts,
                                                      const float* s_prev, const float* __restrict__ x_t,
                                                      const float* V_prev, float* s_out, float* V_out, float* counts,
                                                      float* U_keep, float* A_keep, uint16_t* bits_out,
                                                      uint16_t* s_bf, int Np, const float* xw) {
  const size_t total = static_cast<size_t>(p.B) * p.N;
  const size_t e = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  bool spike = false;
  if (e < total) {
    float acc = 0.f;
    for (int z = 0; z < nparts; ++z) acc += part[static_cast<size_t>(z) * total + e];
    if (xw) acc += xw[e];  // hard mode: the input term, after the spike parts
    const float vp = V_prev ? V_prev[e] : p.reset;
    const float U = leak_clamped(vp, p.reset, p.leak) + acc;
    float s;
    if (p.relaxed) {
      const float xx = U - p.theta;
      s = 0.5f + xx / (1.f + p.slope * fabsf(xx));
    } else {
      s = U > p.theta ? 1.f : 0.f;
    }
    spike = s != 0.f;
    s_out[e] = s;
    if (s_bf) {  // the spike as bfloat16 0 / 1, rows of Np, for the next step's product
      const size_t b = e / p.N;
      s_bf[b * Np + (e - b * p.N)] = spike ? 0x3F80u : 0u;
    }
    V_out[e] = (1.f - s) * U + s * p.reset;
    counts[e] += s;
    if (U_keep) U_keep[e] = U;
  }
  if (bits_out) {
    const uint64_t m = __ballot(spike);
    const int lane = threadIdx.x & 63;
    if ((lane & 15) == 0 && e < total) bits_out[e / 16] = static_cast<uint16_t>(m >> lane);
  }
  if (A_keep) {  // A row of this step: K = N + Nin entries per trial
    const int K = p.N + p.Nin;
    const size_t totalA = static_cast<size_t>(p.B) * K;
    for (size_t i = e; i < totalA; i += static_cast<size_t>(gridDim.x) * blockDim.x) {
      const size_t b = i / K, k = i - b * K;
      A_keep[i] = k < static_cast<size_t>(p.N) ? (s_prev ? s_prev[b * p.N + k] : 0.f) : x_t[b * p.Nin + (k - p.N)];
    }
  }
}

// Backward epilogue of step t: g_out = (dcount + sum of the parts) sigma'(U_t - theta)
//                  + [|V_t - r| > lambda] g_next ((1 - s_t) + (r - U_t) sigma')
// (nparts = 0: g_next is zero, the last step).
__global__ __launch_bounds__(256) void k_bptt_bwd_epi(const BpttDev p, const float* __restrict__ part, int nparts,
                                                      const float* g_next, const float* __restrict__ dcount,
                                                      const float* __restrict__ U_t, const float* __restrict__ V_t,
                                                      const float* __restrict__ s_t, float* g_out) {
  const size_t total = static_cast<size_t>(p.B) * p.N;
  const size_t e = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= total) return;
  float acc = 0.f;
  for (int z = 0; z < nparts; ++z) acc += part[static_cast<size_t>(z) * total + e];
  const float U = U_t[e], V = V_t[e], s = s_t[e];
  const float sg = surrogate_grad(U - p.theta, p.slope);
  const float gn = g_next ? g_next[e] : 0.f;
  const float gv = fabsf(V - p.reset) > p.leak ? gn : 0.f;
  g_out[e] = (dcount[e] + acc) * sg + gv * ((1.f - s) + (p.reset - U) * sg);
}

// dW[K][N] += A^T G over M rows: A [M][K], G [M][N] (row-major); rows
// k >= kbase of dW only (grid y covers K - kbase).  With mc > 0 the rows m
// are split over gridDim.z in ranges of mc and part z is stored (not added)
// at Pz + z (K - kbase) N, rows k - kbase, for k_add_parts.
__global__ __launch_bounds__(256) void k_bptt_wgrad(int M, int K, int N, const float* __restrict__ A,
                                                    const float* __restrict__ G, float* dW, int kbase, int mc,
                                                    float* Pz) {
  __shared__ float As[2][64][kT64 + 4];  // row strides 68 and 80 words: the
  __shared__ float Bs[2][kT64][80];      // matrix-core operand reads are 2-way in the 32 banks
  const int col0 = 64 * blockIdx.x, row0 = kbase + 64 * blockIdx.y;  // columns of dW (j), rows of dW (k)
  const int m0 = mc > 0 ? static_cast<int>(blockIdx.z) * mc : 0;
  const int m1 = mc > 0 ? min(M, m0 + mc) : M;
  auto Aload = [&](int r, int m) -> float {  // (A^T)[row0 + r][m]
    const int k = row0 + r;
    return (k < K && m < m1) ? A[static_cast<size_t>(m) * K + k] : 0.f;
  };
  auto Bload = [&](int m, int c) -> float {
    const int j = col0 + c;
    return (m < m1 && j < N) ? G[static_cast<size_t>(m) * N + j] : 0.f;
  };
  const Acc64 acc = tile_product64(m0, m1, Aload, Bload, As, Bs);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = row0 + 32 * wr + 16 * i + 4 * (lane >> 4) + r;
        const int col = col0 + 32 * wc + 16 * jj + (lane & 15);
        if (k < K && col < N) {
          if (mc > 0)
            Pz[(static_cast<size_t>(blockIdx.z) * (K - kbase) + (k - kbase)) * N + col] = acc.v[i][jj][r];
          else
            dW[static_cast<size_t>(k) * N + col] += acc.v[i][jj][r];
        }
      }
}

// dst[i] += sum over z < nz of parts[z count + i], in order z = 0, 1, ...
__global__ void k_add_parts(float* dst, const float* __restrict__ parts, int nz, size_t count) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float a = 0.f;
  for (int z = 0; z < nz; ++z) a += parts[static_cast<size_t>(z) * count + i];
  dst[i] += a;
}

__global__ void k_transpose(const float* __restrict__ src, float* dst, int n) {
  __shared__ float tile[32][33];
  const int x = 32 * blockIdx.x + threadIdx.x, y0 = 32 * blockIdx.y;
  for (int i = threadIdx.y; i < 32; i += 8)
    if (x < n && y0 + i < n) tile[i][threadIdx.x] = src[static_cast<size_t>(y0 + i) * n + x];
  __syncthreads();
  const int x2 = y0 + threadIdx.x, y2 = 32 * blockIdx.x;
  for (int i = threadIdx.y; i < 32; i += 8)
    if (x2 < n && y2 + i < n) dst[static_cast<size_t>(y2 + i) * n + x2] = tile[threadIdx.x][i];
}

// bit-packed spikes [B][N/16] u16 -> floats [B][N]
__global__ void k_bits_to_float(const uint16_t* __restrict__ bits, float* out, size_t count) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) out[i] = ((bits[i / 16] >> (i % 16)) & 1u) ? 1.f : 0.f;
}

__global__ void k_fill(float* p, float v, size_t count) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}


// ---------------------------------------------------------------------------
// Host orchestration.  Workspace (device, bytes, each part 256-aligned):
//   spikes   hard: bit-packed [T][B][N/16] u16; relaxed: [T][B][N] float
//   vckpt    [nseg][B][N]   V before the first step of every segment
//   sbuf, vbuf  [2][B][N]   forward ping-pong
//   useg, vseg, sseg, gseg  [K][B][N]   one segment, recomputed in backward
//   aseg     [K][B][N + Nin]  the A rows [s_{t-1} | x_t] of the segment
//   wrt      [N][N]         W_rec^T
//   carry, sprev, junk  [B][N]
//   part     [parts][B][N]  partial products of a step
//   wsplit   [N][3 Np]      hard mode: bfloat16 pieces of W_rec, transposed
//   sbf      [2][B][Np]     hard mode: spikes as bfloat16, forward ping-pong
//   xw       [T][B][N]      hard mode: the input term x_t W_in of every step
//   segt     [N][Mp] + [N][3 Mp]  hard mode: a segment's spikes and g, transposed bfloat16 (Mp = K B padded to 64)
// ---------------------------------------------------------------------------
namespace {

struct WsLayout {
  size_t spikes, vckpt, sbuf, vbuf, useg, vseg, sseg, gseg, aseg, wrt, carry, sprev, junk, part, wsplit, sbf, xw, segt,
      total;
  size_t part_floats;
};

// K split of a per-step product over about two workgroups per compute unit
// (tiles of 64 x 64 outputs): chunk length kc (a multiple of kT64), parts.
struct KSplit {
  int kc, parts;
};
KSplit ksplit(int K, int N, int B, int target = 512) {
  const int tiles = ((N + 63) / 64) * ((B + 63) / 64);
  const int want = std::max(1, std::min(16, (target + tiles - 1) / tiles));
  const int kc = std::max(kT64, (K + want * kT64 - 1) / (want * kT64) * kT64);
  return {kc, (K + kc - 1) / kc};
}

int pad64(int n) { return (n + 63) / 64 * 64; }

constexpr int kHardSplitTarget = 512;  // workgroups of a hard-mode forward product
constexpr int kBwdSplitTarget = 512;   // workgroups of a backward product g W_rec^T

// hard mode: spike parts of the forward product (contraction 3 Np) plus
// the FP32 input part
KSplit ksplit_hard(int N, int B) { return ksplit(3 * pad64(N), N, B, kHardSplitTarget); }

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

WsLayout ws_layout(const sn_bptt_desc& d) {
  const size_t N = d.n_neurons, Nin = d.n_inputs, B = d.n_trials, T = d.n_steps, K = d.checkpoint_every;
  const size_t nseg = (T + K - 1) / K;
  const size_t bn = B * N * sizeof(float);
  WsLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o += align256(bytes); return at; };
  L.spikes = take(d.relaxed ? T * bn : T * B * N / 8);
  L.vckpt = take(nseg * bn);
  L.sbuf = take(2 * bn);
  L.vbuf = take(2 * bn);
  L.useg = take(K * bn);
  L.vseg = take(K * bn);
  L.sseg = take(K * bn);
  L.gseg = take(K * bn);
  L.aseg = take(K * B * (N + Nin) * sizeof(float));
  L.wrt = take(N * N * sizeof(float));
  L.carry = take(bn);
  L.sprev = take(bn);
  L.junk = take(bn);
  const int pf = d.relaxed ? ksplit(static_cast<int>(N + Nin), static_cast<int>(N), static_cast<int>(B)).parts
                           : ksplit_hard(static_cast<int>(N), static_cast<int>(B)).parts;
  const int pb = ksplit(static_cast<int>(N), static_cast<int>(N), static_cast<int>(B), kBwdSplitTarget).parts;
  L.part_floats = static_cast<size_t>(std::max(pf, pb)) * B * N;
  L.part = take(L.part_floats * sizeof(float));
  const size_t Np = pad64(static_cast<int>(N));
  L.wsplit = take(d.relaxed ? 0 : N * 3 * Np * sizeof(uint16_t));
  L.sbf = take(d.relaxed ? 0 : 2 * B * Np * sizeof(uint16_t));
  L.xw = take(d.relaxed || Nin == 0 ? 0 : T * bn);
  L.segt = take(d.relaxed ? 0 : N * 4 * static_cast<size_t>(pad64(static_cast<int>(K * B))) * sizeof(uint16_t));
  L.total = o;
  return L;
}

BpttDev dev_of(const sn_bptt_desc& d) {
  BpttDev p{};
  p.N = d.n_neurons;
  p.Nin = d.n_inputs;
  p.B = d.n_trials;
  p.theta = d.threshold;
  p.leak = d.leak;
  p.reset = d.reset;
  p.slope = d.slope;
  p.relaxed = d.relaxed;
  return p;
}

template <class T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

hipError_t fill(float* p, float v, size_t count, hipStream_t s) {
  if (!count) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}

}  // namespace

size_t bptt_workspace_bytes(const sn_bptt_desc& d) { return ws_layout(d).total; }

#define SN_TRY(call)                      \
  do {                                    \
    const hipError_t e_ = (call);         \
    if (e_ != hipSuccess) return e_;      \
  } while (0)

hipError_t bptt_forward(const sn_bptt_desc& d, const float* W, const float* x, float* counts, void* ws, hipStream_t s) {
  const WsLayout L = ws_layout(d);
  const BpttDev p = dev_of(d);
  const int N = d.n_neurons, Nin = d.n_inputs, B = d.n_trials, T = d.n_steps, K = d.checkpoint_every;
  const size_t bn = static_cast<size_t>(B) * N;
  const dim3 grid64((N + 63) / 64, (B + 63) / 64);
  const dim3 epi(static_cast<unsigned>((bn + 255) / 256));
  const KSplit kf = ksplit(N + Nin, N, B);
  float* part = at<float>(ws, L.part);
  const int Np = pad64(N);
  const KSplit kh = ksplit_hard(N, B);
  uint16_t* wsplit = at<uint16_t>(ws, L.wsplit);
  uint16_t* sbf = at<uint16_t>(ws, L.sbf);
  float* xw_all = Nin > 0 && !d.relaxed ? at<float>(ws, L.xw) : nullptr;
  const size_t bnp = static_cast<size_t>(B) * Np;
  SN_TRY(fill(counts, 0.f, bn, s));
  if (!d.relaxed) {
    hipLaunchKernelGGL(k_split_weights, dim3((N + 63) / 64, Np / 64), dim3(256), 0, s, W, wsplit, N, Np);
    SN_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_zero_u16, dim3(static_cast<unsigned>((2 * bnp + 255) / 256)), dim3(256), 0, s, sbf, 2 * bnp);
    SN_TRY(hipGetLastError());
    if (Nin > 0) {
      const int M = T * B;
      hipLaunchKernelGGL(k_bptt_xw, dim3((N + 63) / 64, (M + 63) / 64), dim3(256), 0, s, p, M, x, W, xw_all);
      SN_TRY(hipGetLastError());
    }
  }
  for (int t = 0; t < T; ++t) {
    float* s_out = at<float>(ws, L.sbuf) + (t & 1) * bn;
    float* v_out = at<float>(ws, L.vbuf) + (t & 1) * bn;
    const float* s_prev = t > 0 ? at<float>(ws, L.sbuf) + ((t - 1) & 1) * bn : nullptr;
    const float* v_prev = t > 0 ? at<float>(ws, L.vbuf) + ((t - 1) & 1) * bn : nullptr;
    uint16_t* bits = d.relaxed ? nullptr : at<uint16_t>(ws, L.spikes) + static_cast<size_t>(t) * bn / 16;
    const float* x_t = x + static_cast<size_t>(t) * B * Nin;
    int nparts = kf.parts;
    uint16_t* sb_out = nullptr;
    if (d.relaxed) {
      hipLaunchKernelGGL(k_bptt_part<true>, dim3(grid64.x, grid64.y, kf.parts), dim3(256), 0, s, p, W, s_prev, x_t,
                         kf.kc, part);
    } else {
      const uint16_t* sb_prev = t > 0 ? sbf + static_cast<size_t>((t - 1) & 1) * bnp : nullptr;
      sb_out = sbf + static_cast<size_t>(t & 1) * bnp;
      nparts = kh.parts;
      hipLaunchKernelGGL(k_gemm_split, dim3(grid64.x, grid64.y, nparts), dim3(256), 0, s, sb_prev, B, Np,
                         static_cast<const uint16_t*>(wsplit), N, kh.kc, part, N, bn, 0);
    }
    SN_TRY(hipGetLastError());
    const float* xw_t = xw_all ? xw_all + static_cast<size_t>(t) * bn : nullptr;
    hipLaunchKernelGGL(k_bptt_fwd_epi, epi, dim3(256), 0, s, p, part, nparts, s_prev, x_t, v_prev, s_out, v_out,
                       counts, static_cast<float*>(nullptr), static_cast<float*>(nullptr), bits, sb_out, Np, xw_t);
    SN_TRY(hipGetLastError());
    if (d.relaxed)
      SN_TRY(hipMemcpyAsync(at<float>(ws, L.spikes) + static_cast<size_t>(t) * bn, s_out, bn * sizeof(float),
                            hipMemcpyDeviceToDevice, s));
    if ((t + 1) % K == 0 && t + 1 < T)
      SN_TRY(hipMemcpyAsync(at<float>(ws, L.vckpt) + static_cast<size_t>((t + 1) / K) * bn, v_out, bn * sizeof(float),
                            hipMemcpyDeviceToDevice, s));
  }
  return hipSuccess;
}

hipError_t bptt_forward_noalloc(const sn_bptt_desc& d, const float* W, const float* x, float* counts, hipStream_t s) {
  // the scratch array's address on the current device, looked up once per
  // device with that device current (each device holds its own copy)
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = -1;
  SN_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
      void* p = nullptr;
      SN_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
      addr[dev] = p;
    }
    ws = addr[dev];
  }
  // the forward writes every workspace word before reading it (counts are
  // filled with zeros, the bfloat16 spike rows cleared by a kernel, every
  // other buffer written by the step that reads it), so what an earlier call
  // left in the scratch array does not matter
  return bptt_forward(d, W, x, counts, ws, s);
}

hipError_t bptt_backward(const sn_bptt_desc& d, const float* W, const float* x, const float* dcounts, const void* ws_c,
                         float* dW, hipStream_t s) {
  void* ws = const_cast<void*>(ws_c);
  const WsLayout L = ws_layout(d);
  const BpttDev p = dev_of(d);
  const int N = d.n_neurons, Nin = d.n_inputs, B = d.n_trials, T = d.n_steps, K = d.checkpoint_every;
  const int KA = N + Nin;
  const size_t bn = static_cast<size_t>(B) * N;
  const dim3 grid64((N + 63) / 64, (B + 63) / 64);
  const dim3 epi(static_cast<unsigned>((bn + 255) / 256));
  const KSplit kf = ksplit(KA, N, B), kb = ksplit(N, N, B, kBwdSplitTarget);
  float* part = at<float>(ws, L.part);
  const size_t part_floats = L.part_floats;
  const int Np = pad64(N);
  const KSplit kh = ksplit_hard(N, B);
  const uint16_t* wsplit = at<uint16_t>(ws, L.wsplit);  // written by the forward pass from the same W
  uint16_t* sbf = at<uint16_t>(ws, L.sbf);
  const float* xw_all = Nin > 0 && !d.relaxed ? at<float>(ws, L.xw) : nullptr;  // from the forward pass
  const size_t bnp = static_cast<size_t>(B) * Np;
  float* wrt = at<float>(ws, L.wrt);
  hipLaunchKernelGGL(k_transpose, dim3((N + 31) / 32, (N + 31) / 32), dim3(32, 8), 0, s, W, wrt, N);
  SN_TRY(hipGetLastError());
  SN_TRY(fill(dW, 0.f, static_cast<size_t>(KA) * N, s));
  const int nseg = (T + K - 1) / K;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int t0 = seg * K, t1 = std::min(T, t0 + K);
    // recompute the segment's forward from its checkpoint
    const float* s_prev = nullptr;
    const float* v_prev = t0 > 0 ? at<float>(ws, L.vckpt) + static_cast<size_t>(seg) * bn : nullptr;
    if (t0 > 0) {
      float* sp = at<float>(ws, L.sprev);
      if (d.relaxed) {
        SN_TRY(hipMemcpyAsync(sp, at<float>(ws, L.spikes) + static_cast<size_t>(t0 - 1) * bn, bn * sizeof(float),
                              hipMemcpyDeviceToDevice, s));
      } else {
        hipLaunchKernelGGL(k_bits_to_float, dim3(static_cast<unsigned>((bn + 255) / 256)), dim3(256), 0, s,
                           at<uint16_t>(ws, L.spikes) + static_cast<size_t>(t0 - 1) * bn / 16, sp, bn);
        SN_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_bits_to_bf16, dim3(static_cast<unsigned>((bn + 255) / 256)), dim3(256), 0, s,
                           at<uint16_t>(ws, L.spikes) + static_cast<size_t>(t0 - 1) * bn / 16,
                           sbf + static_cast<size_t>((t0 - 1) & 1) * bnp, B, N, Np);
        SN_TRY(hipGetLastError());
      }
      s_prev = sp;
    }
    for (int t = t0; t < t1; ++t) {
      const size_t i = static_cast<size_t>(t - t0);
      float* s_out = at<float>(ws, L.sseg) + i * bn;
      float* v_out = at<float>(ws, L.vseg) + i * bn;
      const float* x_t = x + static_cast<size_t>(t) * B * Nin;
      int nparts = kf.parts;
      uint16_t* sb_out = nullptr;
      if (d.relaxed) {
        hipLaunchKernelGGL(k_bptt_part<true>, dim3(grid64.x, grid64.y, kf.parts), dim3(256), 0, s, p, W, s_prev, x_t,
                           kf.kc, part);
      } else {
        const uint16_t* sb_prev = s_prev ? sbf + static_cast<size_t>((t - 1) & 1) * bnp : nullptr;
        sb_out = sbf + static_cast<size_t>(t & 1) * bnp;
        nparts = kh.parts;
        hipLaunchKernelGGL(k_gemm_split, dim3(grid64.x, grid64.y, nparts), dim3(256), 0, s, sb_prev, B, Np, wsplit, N,
                           kh.kc, part, N, bn, 0);
      }
      SN_TRY(hipGetLastError());
      const float* xw_t = xw_all ? xw_all + static_cast<size_t>(t) * bn : nullptr;
      hipLaunchKernelGGL(k_bptt_fwd_epi, epi, dim3(256), 0, s, p, part, nparts, s_prev, x_t, v_prev, s_out, v_out,
                         at<float>(ws, L.junk), at<float>(ws, L.useg) + i * bn, at<float>(ws, L.aseg) + i * B * KA,
                         static_cast<uint16_t*>(nullptr), sb_out, Np, xw_t);
      SN_TRY(hipGetLastError());
      s_prev = s_out;
      v_prev = v_out;
    }
    // backward through the segment
    for (int t = t1 - 1; t >= t0; --t) {
      const size_t i = static_cast<size_t>(t - t0);
      const float* g_next = nullptr;
      if (t < T - 1) g_next = (t == t1 - 1) ? at<float>(ws, L.carry) : at<float>(ws, L.gseg) + (i + 1) * bn;
      if (g_next) {
        hipLaunchKernelGGL(k_bptt_part<false>, dim3(grid64.x, grid64.y, kb.parts), dim3(256), 0, s, p, wrt, g_next,
                           static_cast<const float*>(nullptr), kb.kc, part);
        SN_TRY(hipGetLastError());
      }
      hipLaunchKernelGGL(k_bptt_bwd_epi, epi, dim3(256), 0, s, p, part, g_next ? kb.parts : 0, g_next, dcounts,
                         at<float>(ws, L.useg) + i * bn, at<float>(ws, L.vseg) + i * bn, at<float>(ws, L.sseg) + i * bn,
                         at<float>(ws, L.gseg) + i * bn);
      SN_TRY(hipGetLastError());
    }
    SN_TRY(hipMemcpyAsync(at<float>(ws, L.carry), at<float>(ws, L.gseg), bn * sizeof(float), hipMemcpyDeviceToDevice, s));
    // dW_cat += A_seg^T G_seg
    const int M = (t1 - t0) * B;
    if (d.relaxed) {
      hipLaunchKernelGGL(k_bptt_wgrad, dim3((N + 63) / 64, (KA + 63) / 64), dim3(256), 0, s, M, KA, N,
                         at<float>(ws, L.aseg), at<float>(ws, L.gseg), dW, 0, 0, static_cast<float*>(nullptr));
      SN_TRY(hipGetLastError());
    } else {
      // W_rec rows: spikes (0 / 1) times the three bfloat16 pieces of g;
      // W_in rows (x may be any real value): FP32
      const int Mp = pad64(M);
      uint16_t* At = at<uint16_t>(ws, L.segt);
      uint16_t* Gt = At + static_cast<size_t>(N) * Mp;
      hipLaunchKernelGGL(k_seg_transpose, dim3((N + 63) / 64, Mp / 64), dim3(256), 0, s, at<float>(ws, L.aseg), KA,
                         at<float>(ws, L.gseg), N, M, Mp, At, Gt);
      SN_TRY(hipGetLastError());
      hipLaunchKernelGGL(k_gemm_split, dim3((N + 63) / 64, (N + 63) / 64, 1), dim3(256), 0, s,
                         static_cast<const uint16_t*>(At), N, Mp, static_cast<const uint16_t*>(Gt), N, 3 * Mp, dW, N,
                         static_cast<size_t>(0), 1);
      SN_TRY(hipGetLastError());
      if (Nin > 0) {
        // few output tiles: the rows m split over nz workgroups per tile,
        // partial products in the part buffer, added in a fixed order
        const size_t xcount = static_cast<size_t>(Nin) * N;
        const int nz = static_cast<int>(std::min<size_t>(4, part_floats / xcount));  // parts that fit the buffer
        if (nz >= 2) {
          const int mc = (M + nz * kT64 - 1) / (nz * kT64) * kT64;
          const int zz = (M + mc - 1) / mc;  // <= nz
          hipLaunchKernelGGL(k_bptt_wgrad, dim3((N + 63) / 64, (Nin + 63) / 64, zz), dim3(256), 0, s, M, KA, N,
                             at<float>(ws, L.aseg), at<float>(ws, L.gseg), dW, N, mc, part);
          SN_TRY(hipGetLastError());
          hipLaunchKernelGGL(k_add_parts, dim3(static_cast<unsigned>((xcount + 255) / 256)), dim3(256), 0, s,
                             dW + static_cast<size_t>(N) * N, static_cast<const float*>(part), zz, xcount);
        } else {
          hipLaunchKernelGGL(k_bptt_wgrad, dim3((N + 63) / 64, (Nin + 63) / 64), dim3(256), 0, s, M, KA, N,
                             at<float>(ws, L.aseg), at<float>(ws, L.gseg), dW, N, 0, static_cast<float*>(nullptr));
        }
        SN_TRY(hipGetLastError());
      }
    }
  }
  return hipSuccess;
}

}  // namespace snmi
