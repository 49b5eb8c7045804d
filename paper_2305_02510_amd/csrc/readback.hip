// Raster readback into device memory (sn_read_raster_device): the simulation
// keeps its spikes as rows [t][b][G] of 64-bit words, one word per 64-neuron
// group; callers get the API layout [B][steps][ceil(N/32)] of 32-bit words.
#include <hip/hip_runtime.h>

#include "sn_device.h"
#include "sn_internal.h"

namespace snmi {

// One output word per thread: the writes are coalesced, and the two halves
// of a row word are read by neighbouring threads (one cache line).
__global__ void k_unpack_raster(const DevNet n, int t0, int steps, uint32_t* __restrict__ out) {
  const int W32 = (n.N + 31) / 32;
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t total = static_cast<size_t>(n.B) * steps * W32;
  if (i >= total) return;
  const int w = static_cast<int>(i % W32);
  const size_t bt = i / W32;
  const int tt = static_cast<int>(bt % steps);
  const int b = static_cast<int>(bt / steps);
  const uint64_t v = n.raster[row_word(n, t0 + tt, b, w >> 1)];
  out[i] = static_cast<uint32_t>(v >> (32 * (w & 1)));
}

hipError_t launch_unpack_raster(const DevNet& n, int32_t t0, int32_t steps, uint32_t* out, hipStream_t s) {
  const size_t total = static_cast<size_t>(n.B) * steps * ((n.N + 31) / 32);
  if (total == 0) return hipSuccess;
  const unsigned blocks = static_cast<unsigned>((total + 255) / 256);
  hipLaunchKernelGGL(k_unpack_raster, dim3(blocks), dim3(256), 0, s, n, t0, steps, out);
  return hipGetLastError();
}

}  // namespace snmi
