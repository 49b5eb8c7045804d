// Device helpers shared by the HIP kernels: the fused LIF neuron update.
#pragma once

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

}  // namespace snmi
