// Surrogate-gradient backpropagation through time for a recurrent LIF layer
// (the model of §2.1 with delay-1 recurrent weights, input through W_in and
// no refractory period), on FP32 matrix cores (v_mfma_f32_16x16x4_f32).
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
// 32 x 32 output tile, K in chunks of 32 staged through LDS, each wave one
// 16 x 16 accumulator.  Operand layout of v_mfma_f32_16x16x4_f32: lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16]; the result D[4 (l/16) + r]
// [l % 16], r = 0..3.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/superneuro_mi.h"
#include "sn_internal.h"

namespace snmi {

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

// 32 x 32 tile of a row-major product, K staged 128 at a time through two
// LDS buffers (padded rows: see the kernels' declarations); the next chunk's operands are loaded into registers while the
// matrix cores work on the current one, so there is one barrier per chunk.
//   Aload(row, k) -> A[row][k]; Bload(k, col) -> B[k][col]
// Returns the wave's 16 x 16 accumulator; (row0 + 16 wr + 4 (lane/16) + r,
// col0 + 16 wc + lane % 16) is element r.
constexpr int kTileK = 128;

template <class AL, class BL>
__device__ __forceinline__ f32x4 tile_product(int K, AL Aload, BL Bload, float (*As)[32][kTileK + 4],
                                              float (*Bs)[kTileK][48]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  // element e of this thread's share: A (row idx / kTileK, k idx % kTileK),
  // B (k idx / 32, col idx % 32), idx = tid + 256 e
  constexpr int kPer = 32 * kTileK / 256;
  float ra[kPer], rb[kPer];
  auto fetch = [&](int kc) {
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int idx = tid + 256 * e;
      ra[e] = Aload(idx / kTileK, kc + (idx % kTileK));
      rb[e] = Bload(kc + (idx >> 5), idx & 31);
    }
  };
  fetch(0);
  int buf = 0;
  for (int kc = 0; kc < K; kc += kTileK) {
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int idx = tid + 256 * e;
      As[buf][idx / kTileK][idx % kTileK] = ra[e];
      Bs[buf][idx >> 5][idx & 31] = rb[e];
    }
    __syncthreads();
    if (kc + kTileK < K) fetch(kc + kTileK);
#pragma unroll
    for (int kk = 0; kk < kTileK; kk += 4) {
      const float av = As[buf][16 * wr + (lane & 15)][kk + (lane >> 4)];
      const float bv = Bs[buf][kk + (lane >> 4)][16 * wc + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
    }
    buf ^= 1;
  }
  return acc;
}

// Forward step t: tile (cols 32 blockIdx.x .., trials 32 blockIdx.y ..).
// s_prev [B][N] (null: no spikes yet), V_prev [B][N] (null: rest state),
// x_t [B][Nin].  Writes s_out, V_out [B][N]; adds s into counts; optionally
// keeps U [B][N], the A row [B][N + Nin], and bit-packed spikes [B][N/32]
// (16-bit halves per wave, N a multiple of 32).
__global__ __launch_bounds__(256) void k_bptt_forward(const BpttDev p, const float* __restrict__ W, const float* s_prev,
                                                      const float* __restrict__ x_t, const float* V_prev, float* s_out,
                                                      float* V_out, float* counts, float* U_keep, float* A_keep,
                                                      uint16_t* bits_out) {
  __shared__ float As[2][32][kTileK + 4];  // row stride 132 and 48 words: the
  __shared__ float Bs[2][kTileK][48];      // matrix-core operand reads are 2-way in the 32 banks
  const int col0 = 32 * blockIdx.x, row0 = 32 * blockIdx.y;
  const int N = p.N, Nin = p.Nin, B = p.B, K = N + Nin;
  auto Aload = [&](int r, int k) -> float {
    const int b = row0 + r;
    if (b >= B || k >= K) return 0.f;
    if (k < N) return s_prev ? s_prev[static_cast<size_t>(b) * N + k] : 0.f;
    return x_t[static_cast<size_t>(b) * Nin + (k - N)];
  };
  auto Bload = [&](int k, int c) -> float {
    const int j = col0 + c;
    return (k < K && j < N) ? W[static_cast<size_t>(k) * N + j] : 0.f;
  };
  const f32x4 acc = tile_product(K, Aload, Bload, As, Bs);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int col = col0 + 16 * wc + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int b = row0 + 16 * wr + 4 * (lane >> 4) + r;
    bool spike = false;
    if (b < B && col < N) {
      const size_t e = static_cast<size_t>(b) * N + col;
      const float vp = V_prev ? V_prev[e] : p.reset;
      const float U = leak_clamped(vp, p.reset, p.leak) + acc[r];
      float s;
      if (p.relaxed) {
        const float xx = U - p.theta;
        s = 0.5f + xx / (1.f + p.slope * fabsf(xx));
      } else {
        s = U > p.theta ? 1.f : 0.f;
      }
      spike = s != 0.f;
      s_out[e] = s;
      V_out[e] = (1.f - s) * U + s * p.reset;
      counts[e] += s;
      if (U_keep) U_keep[e] = U;
    }
    if (bits_out) {
      const uint64_t m = __ballot(spike);
      // lanes (lane & 15) == 0 hold rows 4 (lane/16) + r: 16 spike bits each
      if ((lane & 15) == 0 && b < B && col < N)
        bits_out[(static_cast<size_t>(b) * N + col) / 16] = static_cast<uint16_t>(m >> (16 * (lane >> 4)));
    }
  }
  if (A_keep) {  // the A rows of this step, for the weight gradient
    for (int i = threadIdx.x; i < 32 * 32; i += 256) {
      const int r = i >> 5, c = i & 31;
      const int b = row0 + r;
      if (b >= B) continue;
      for (int k = col0 + c; k < K; k += 32 * gridDim.x) A_keep[static_cast<size_t>(b) * K + k] = Aload(r, k);
    }
  }
}

// Backward step t: g_out = (dcount + g_next W_rec^T) sigma'(U_t - theta)
//                  + [|V_t - r| > lambda] g_next ((1 - s_t) + (r - U_t) sigma')
// WrT = W_rec^T [N][N]; g_next null at the last step (zero).
__global__ __launch_bounds__(256) void k_bptt_backward(const BpttDev p, const float* __restrict__ WrT,
                                                       const float* g_next, const float* __restrict__ dcount,
                                                       const float* __restrict__ U_t, const float* __restrict__ V_t,
                                                       const float* __restrict__ s_t, float* g_out) {
  __shared__ float As[2][32][kTileK + 4];  // row stride 132 and 48 words: the
  __shared__ float Bs[2][kTileK][48];      // matrix-core operand reads are 2-way in the 32 banks
  const int col0 = 32 * blockIdx.x, row0 = 32 * blockIdx.y;
  const int N = p.N, B = p.B;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  if (g_next) {
    auto Aload = [&](int r, int k) -> float {
      const int b = row0 + r;
      return (b < B && k < N) ? g_next[static_cast<size_t>(b) * N + k] : 0.f;
    };
    auto Bload = [&](int k, int c) -> float {
      const int j = col0 + c;
      return (k < N && j < N) ? WrT[static_cast<size_t>(k) * N + j] : 0.f;
    };
    acc = tile_product(N, Aload, Bload, As, Bs);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int col = col0 + 16 * wc + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int b = row0 + 16 * wr + 4 * (lane >> 4) + r;
    if (b >= B || col >= N) continue;
    const size_t e = static_cast<size_t>(b) * N + col;
    const float U = U_t[e], V = V_t[e], s = s_t[e];
    const float sg = surrogate_grad(U - p.theta, p.slope);
    const float gn = g_next ? g_next[e] : 0.f;
    const float gv = fabsf(V - p.reset) > p.leak ? gn : 0.f;
    g_out[e] = (dcount[e] + acc[r]) * sg + gv * ((1.f - s) + (p.reset - U) * sg);
  }
}

// dW[K][N] += A^T G over M rows: A [M][K], G [M][N] (row-major).
__global__ __launch_bounds__(256) void k_bptt_wgrad(int M, int K, int N, const float* __restrict__ A,
                                                    const float* __restrict__ G, float* dW) {
  __shared__ float As[2][32][kTileK + 4];  // row stride 132 and 48 words: the
  __shared__ float Bs[2][kTileK][48];      // matrix-core operand reads are 2-way in the 32 banks
  const int col0 = 32 * blockIdx.x, row0 = 32 * blockIdx.y;  // columns of dW (j), rows of dW (k)
  auto Aload = [&](int r, int m) -> float {  // (A^T)[row0 + r][m]
    const int k = row0 + r;
    return (k < K && m < M) ? A[static_cast<size_t>(m) * K + k] : 0.f;
  };
  auto Bload = [&](int m, int c) -> float {
    const int j = col0 + c;
    return (m < M && j < N) ? G[static_cast<size_t>(m) * N + j] : 0.f;
  };
  const f32x4 acc = tile_product(M, Aload, Bload, As, Bs);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int col = col0 + 16 * wc + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int k = row0 + 16 * wr + 4 * (lane >> 4) + r;
    if (k < K && col < N) dW[static_cast<size_t>(k) * N + col] += acc[r];
  }
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
// ---------------------------------------------------------------------------
namespace {

struct WsLayout {
  size_t spikes, vckpt, sbuf, vbuf, useg, vseg, sseg, gseg, aseg, wrt, carry, sprev, junk, total;
};

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
  const dim3 grid((N + 31) / 32, (B + 31) / 32);
  SN_TRY(fill(counts, 0.f, bn, s));
  for (int t = 0; t < T; ++t) {
    float* s_out = at<float>(ws, L.sbuf) + (t & 1) * bn;
    float* v_out = at<float>(ws, L.vbuf) + (t & 1) * bn;
    const float* s_prev = t > 0 ? at<float>(ws, L.sbuf) + ((t - 1) & 1) * bn : nullptr;
    const float* v_prev = t > 0 ? at<float>(ws, L.vbuf) + ((t - 1) & 1) * bn : nullptr;
    uint16_t* bits = d.relaxed ? nullptr : at<uint16_t>(ws, L.spikes) + static_cast<size_t>(t) * bn / 16;
    hipLaunchKernelGGL(k_bptt_forward, grid, dim3(256), 0, s, p, W, s_prev, x + static_cast<size_t>(t) * B * Nin,
                       v_prev, s_out, v_out, counts, static_cast<float*>(nullptr), static_cast<float*>(nullptr), bits);
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

hipError_t bptt_backward(const sn_bptt_desc& d, const float* W, const float* x, const float* dcounts, const void* ws_c,
                         float* dW, hipStream_t s) {
  void* ws = const_cast<void*>(ws_c);
  const WsLayout L = ws_layout(d);
  const BpttDev p = dev_of(d);
  const int N = d.n_neurons, Nin = d.n_inputs, B = d.n_trials, T = d.n_steps, K = d.checkpoint_every;
  const int KA = N + Nin;
  const size_t bn = static_cast<size_t>(B) * N;
  const dim3 grid((N + 31) / 32, (B + 31) / 32);
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
      }
      s_prev = sp;
    }
    for (int t = t0; t < t1; ++t) {
      const size_t i = static_cast<size_t>(t - t0);
      float* s_out = at<float>(ws, L.sseg) + i * bn;
      float* v_out = at<float>(ws, L.vseg) + i * bn;
      hipLaunchKernelGGL(k_bptt_forward, grid, dim3(256), 0, s, p, W, s_prev, x + static_cast<size_t>(t) * B * Nin,
                         v_prev, s_out, v_out, at<float>(ws, L.junk), at<float>(ws, L.useg) + i * bn,
                         at<float>(ws, L.aseg) + i * B * KA, static_cast<uint16_t*>(nullptr));
      SN_TRY(hipGetLastError());
      s_prev = s_out;
      v_prev = v_out;
    }
    // backward through the segment
    for (int t = t1 - 1; t >= t0; --t) {
      const size_t i = static_cast<size_t>(t - t0);
      const float* g_next = nullptr;
      if (t < T - 1) g_next = (t == t1 - 1) ? at<float>(ws, L.carry) : at<float>(ws, L.gseg) + (i + 1) * bn;
      hipLaunchKernelGGL(k_bptt_backward, grid, dim3(256), 0, s, p, wrt, g_next, dcounts, at<float>(ws, L.useg) + i * bn,
                         at<float>(ws, L.vseg) + i * bn, at<float>(ws, L.sseg) + i * bn, at<float>(ws, L.gseg) + i * bn);
      SN_TRY(hipGetLastError());
    }
    SN_TRY(hipMemcpyAsync(at<float>(ws, L.carry), at<float>(ws, L.gseg), bn * sizeof(float), hipMemcpyDeviceToDevice, s));
    // dW_cat += A_seg^T G_seg
    const int M = (t1 - t0) * B;
    hipLaunchKernelGGL(k_bptt_wgrad, dim3((N + 31) / 32, (KA + 31) / 32), dim3(256), 0, s, M, KA, N,
                       at<float>(ws, L.aseg), at<float>(ws, L.gseg), dW);
    SN_TRY(hipGetLastError());
  }
  return hipSuccess;
}

}  // namespace snmi
