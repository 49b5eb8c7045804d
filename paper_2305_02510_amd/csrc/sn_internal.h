// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace snmi {

// Neurons are processed in groups of one wavefront: 64 consecutive post-neurons
// whose spikes form one 64-bit word (one ballot).
constexpr int kGroup = 64;

// One incoming synapse of a post-neuron group, 8 bytes:
//   w      binary32 weight
//   meta   bits  0..19  pre-neuron index
//          bits 20..25  delay - 1
//          bits 26..31  post-neuron index within its group
struct Rec {
  float w;
  uint32_t meta;
};

__host__ __device__ constexpr uint32_t pack_meta(uint32_t pre, uint32_t delay, uint32_t post_local) {
  return pre | ((delay - 1u) << 20) | (post_local << 26);
}

// Work unit of the persistent kernel ("chunk"): up to kChunk = 4 x 64
// consecutive records of one group, one batch of a wavefront.
// x = first record, y = group | count << 20.
constexpr int kChunk = 256;

// Host-side result of the layout builder.
struct HostLayout {
  std::vector<Rec> recs;        // grouped by post-group, round-robin over posts inside a group
  std::vector<int32_t> gptr;    // [G + 1] record offset of every group
  std::vector<uint2> chunks;    // chunk table (kChunk records max per chunk)
  std::vector<int32_t> gchunk;  // [G + 1] first chunk of every group
  int32_t max_group_records = 0;
};

// Partition of the groups into P contiguous slices for the persistent kernel.
struct SlicePlan {
  std::vector<int32_t> wg_group;  // [P + 1]
  std::vector<int32_t> wg_chunk;  // [P + 1]
  int32_t P = 0;
  int32_t ng_max = 0;
  int64_t max_recs = 0;
  bool recs_lds = false;
  bool ring_lds = false;
};

// Splits groups into `slices` contiguous slices balancing record counts, no
// slice holding more than `max_groups` groups.  slices is clamped to [1, G].
SlicePlan partition_groups(const HostLayout& L, int32_t G, int32_t slices, int32_t max_groups);

HostLayout build_layout(int32_t n, int64_t nnz, const int32_t* pre, const int32_t* post, const float* w,
                        const uint8_t* delay);

// Plain pointers and sizes handed to every kernel.
struct DevNet {
  int32_t N;      // neurons
  int32_t Npad;   // G * 64
  int32_t G;      // groups = words per spike row
  int32_t B;      // trials
  int32_t D;      // max delay
  int32_t nchunks;
  int64_t nnz;
  // per-neuron parameters, padded to Npad (padding: threshold = +inf, rest 0)
  const float* theta;
  const float* leak;
  const float* reset;
  const float* amp;
  const uint8_t* refr;
  // state [B][Npad]
  float* V;
  uint8_t* ref;
  // spike raster and external spikes, [Tcap][B][G] 64-bit words (time-major)
  uint64_t* raster;
  const uint64_t* ext;
  // synapses
  const Rec* recs;
  const int32_t* gptr;
  const uint2* chunks;
};

// Arguments of the persistent kernel: the network plus a partition of its
// post-neuron groups into P slices (one workgroup per slice and trial).
struct SimArgs {
  DevNet n;
  const int32_t* wg_group;  // [P + 1] first group of every slice
  const int32_t* wg_chunk;  // [P + 1] first chunk of every slice
  uint32_t* flags;          // [B][P] last step + 1 published by every slice
  uint32_t* status;         // set to nonzero when a barrier wait times out
  int32_t P;
  int32_t ng_max;           // most groups in one slice
  int64_t max_recs;         // most records in one slice
};

// Kernel launchers (kernels.hip).  All return hipSuccess or the launch error.
size_t sim_lds_bytes(const DevNet& n, int ng_max, int64_t max_recs, bool recs_lds, bool ring_lds);
size_t lds_limit();
int sim_threads(int ng_max);
int sim_npt(int ng_max);
hipError_t launch_sim(const SimArgs& a, bool recs_lds, bool ring_lds, int32_t t0, int32_t steps, hipStream_t s);
hipError_t launch_clear_u32(uint32_t* p, int count, hipStream_t s);
hipError_t launch_step(const DevNet& n, int32_t t, hipStream_t s);
hipError_t launch_reset_state(const DevNet& n, hipStream_t s);
hipError_t launch_repack_input(const DevNet& n, int32_t t0, int32_t steps, const uint32_t* bits,
                               hipStream_t s);

}  // namespace snmi
