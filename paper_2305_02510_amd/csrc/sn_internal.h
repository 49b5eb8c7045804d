// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
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

// Work unit of a wavefront ("chunk"): kChunk = 4 x 64 consecutive records of
// one part of one group.
constexpr int kChunk = 256;

// Host-side result of the layout builder (layout.cpp): the records of every
// group, delay >= 2 part then delay-1 part, each part in lane-owned rows of
// 64 (lane l: a synapse of post l or a zero-weight filler) followed by the
// overflow of high in-degree posts; every section a multiple of 64 records.
// Fillers carry the weight -0.0f (input weights of zero are stored as +0.0f),
// which adds nothing and marks them for the plasticity kernel.
struct HostLayout {
  std::vector<Rec> recs;
  std::vector<int32_t> src;     // input index of every record, -1 for fillers
  std::vector<int32_t> gptr;    // [G + 1] record offset of every group
  std::vector<int32_t> gsplit;  // [G] first delay-1 record of every group
  // short sections (block > 2): ssec[g * (block - 1) + d - 1] is the first
  // record of group g's section of delay d, d = 1 .. block - 1 (the sections
  // follow phase 0 in the order d = block - 1 .. 1; ssec of d = 1 = gsplit)
  int32_t block = 2;
  std::vector<int32_t> ssec;  // [G][block - 1]
  int32_t max_group_records = 0;
  // set when the records with fillers would pass INT32_MAX (offsets are
  // 32-bit on the device); the other fields are then incomplete
  bool too_large = false;
  // delay phases of the wide per-step kernel: with phase_rows > 0, part A of
  // group g holds the sections of phases P-1 .. 1 and then phase 0 (delays
  // >= 2), each in lane-owned rows; wsec[g * P + p] is the first record of
  // phase p's section (phase p: delays p * phase_rows + 1 .. (p+1) * phase_rows;
  // phase 0 runs on to the end of part B).  P = 1 without phases.
  int32_t phases = 1;
  int32_t phase_rows = 0;
  std::vector<int32_t> wsec;  // [G][P]
};


// Partition of the groups into P contiguous slices for the persistent kernel.
struct SlicePlan {
  std::vector<int32_t> wg_group;  // [P + 1]
  int32_t P = 0;
  int32_t ng_max = 0;
  int64_t max_recs = 0;
  bool recs_lds = false;
  bool ring_lds = false;
};

// Splits groups into `slices` contiguous slices balancing record counts, no
// slice holding more than `max_groups` groups.  slices is clamped to [1, G].
SlicePlan partition_groups(const HostLayout& L, int32_t G, int32_t slices, int32_t max_groups);

// phase_rows > 0 splits part A into delay phases of that many delays each
// (see HostLayout), for nets of at least two phases; 0 = no phases.
// lane_only: no overflow sections, every record in its post's lane (as many
// rows as a section's largest in-degree).  block >= 2: part A holds the
// delays >= block, and the delays 1 .. block - 1 get a section each after it
// (block 2: part B, the delay-1 records); needs phase_rows >= block - 1.
HostLayout build_layout(int32_t n, int64_t nnz, const int32_t* pre, const int32_t* post, const float* w,
                        const uint8_t* delay, int32_t max_delay = 64, int32_t phase_rows = 0, bool lane_only = false,
                        int32_t block = 2);

// Lane record, 4 bytes, of a lane_only layout (the post is the lane) for the
// wide per-step kernel when every delay is staged in LDS, nets whose weights
// are all k * 2^-e with |k| <= 127:
//   bits 0..4    the source's bit in its 32-bit history word (pre mod 32)
//   bits 5..22   LDS byte offset of that word among the phase's staged rows,
//                (((delay - 1) mod phase_rows + block - 1) * 2G + pre / 32) * 4:
//                LDS row r holds the history of step t - (first delay of the
//                phase) - r + block - 2, so the word i rows below is the same
//                source's word for step t + i (blocks of steps)
//   bits 24..31  k (int8)
// A filler has k = 0.  The kernel reads batches of kLaneBatchRows rows and
// skips the rows of a batch past its section's end (sections are whole
// rows), so the device array carries one batch of zero records of slack
// after the last section.
constexpr int32_t kLaneBatchRows = 8;
constexpr uint32_t kLaneMaxOffset = 1u << 18;
__host__ __device__ inline uint32_t lane_record(int32_t k, uint32_t byte_offset, uint32_t bit) {
  return (static_cast<uint32_t>(k) << 24) | (byte_offset << 5) | bit;
}
// Lane records of a lane_only layout for G groups and the layout's phases
// and block (phase_rows = 0: no phases, every delay staged at once), or empty
// when a record is not in its post's lane, a weight does not allow it or an
// offset does not fit; *scale = 2^-e.
std::vector<uint32_t> lane_records(const HostLayout& L, int32_t G, float* scale);

// Plain pointers and sizes handed to every kernel.
struct DevNet {
  int32_t N;      // neurons
  int32_t Npad;   // G * 64
  int32_t G;      // groups = words per spike row
  int32_t B;      // trials
  int32_t D;      // max delay
  int64_t nnz;    // synapses (records, with fillers: gptr[G])
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
  const int32_t* gptr;    // [G + 1]
  const int32_t* gsplit;  // [G] first delay-1 record of every group
  // delay phases of part A (HostLayout::wsec), for the wide per-step kernel
  const int32_t* wsec;    // [G][phases]
  int32_t phases;         // 1: no phases
  int32_t phase_rows;
  // 4-byte copies of the records (same order), or null: see compact_record
  const uint32_t* crecs;
  float cscale;           // 2^-e: weight = (int8 numerator) * cscale
  // wide nets: lane records of a lane_only layout with the same delay phases
  // (own offsets), or null: see lane_record
  const uint32_t* lrecs;
  const int32_t* lgptr;   // [G + 1]
  const int32_t* lwsec;   // [G][phases]
  const int32_t* lsec;    // [G][lblock - 1] first lane record of the section of delay d (index d - 1)
  float* held;            // [lblock - 1][B][Npad] input of steps t + 1 .. gathered by a block's first kernel
  int32_t lblock;         // steps per block of the lane layout (2 or 4)
  float lscale;
};

// Compact record, 4 bytes, for the batch kernel, whose workgroups hold the
// spike history as a ring of D + 1 rows of 2G words in LDS; for nets with
// (D + 1) * 2G <= 2^13 and every weight k * 2^-e with |k| <= 127:
//   bits  0..4   the source's bit in its 32-bit word (pre mod 32)
//   bits  5..17  offset of the source word from the current row:
//                (D + 1 - delay) * 2G + pre / 32 (the row of step t - delay
//                is the current row minus delay, modulo D + 1)
//   bits 18..23  (post-neuron within its group - lane) mod 64, where the lane
//                is the record's position mod 64: 0 for the lane-owned rows,
//                so only overflow records carry a nonzero value
//   bits 24..31  k (int8)
constexpr uint32_t kCompactMaxRing = 1u << 13;
// Records per lane in one chunk of the batch kernel with compact records.
// Sections are whole rows of 64, so the kernel masks a chunk's rows past its
// section's end as a whole and loads them unclamped: the device array
// carries one chunk (kCompactChunkRows rows) of zero records as slack after
// its last record.
constexpr int32_t kCompactChunkRows = 12;
__host__ __device__ inline uint32_t compact_record(int32_t k, uint32_t offset, uint32_t bit, uint32_t post_delta) {
  return (static_cast<uint32_t>(k) << 24) | (post_delta << 18) | (offset << 5) | bit;
}

// Arguments of the persistent kernel: the network plus a partition of its
// post-neuron groups into P slices (one workgroup per slice and trial).
struct SimArgs {
  DevNet n;
  const int32_t* wg_group;  // [P + 1] first group of every slice
  uint64_t* mailbox;        // [D + 1][B][2G] tagged spike words: (step + 1) << 32 | 32 spike bits
  uint32_t* status;         // set to nonzero when a wait times out
  int32_t P;
  int32_t ng_max;           // most groups in one slice
  int64_t max_recs;         // most records in one slice
};

// Plasticity (sn_set_stdp): the rule of the header, applied to the pull
// records after the update of step t by k_stdp.
struct StdpArgs {
  DevNet n;
  Rec* recs;        // the records of n, written in place
  int32_t window;   // W, 1..16
  float ltp[16];    // ltp[lag], lag = t - arrival < W
  float ltd[16];    // ltd[lag - 1], lag = t - post spike in 1..W
  float w_min, w_max;
  uint64_t* hist;   // [2][Npad] spike-history words (bit k: spike k steps before)
  int32_t chunk;    // records per workgroup (a group's records split over `chunks` workgroups)
  int32_t chunks;
};
constexpr int kStdpThreads = 256;
constexpr int kStdpUnroll = 4;  // records per thread loaded together
// records of a group per plasticity workgroup, and workgroups per group
inline void stdp_chunks(int32_t max_group_records, int32_t& chunk, int32_t& chunks) {
  chunk = kStdpThreads * kStdpUnroll;
  chunks = std::max(1, (max_group_records + chunk - 1) / chunk);
}

// Dense delay-1 weights for the matrix-core path, bfloat16, tiled for
// v_mfma_f32_16x16x32_bf16.  K (pre-neurons) is padded to kpad, a multiple
// of 128, and walked in blocks j of 128 = 4 steps s x 4 lane groups q x 8:
// at step (j, s) lane group q contracts pre-neurons 8 * (16 j + 4 q + s) + e,
// e = 0..7, so one 32-bit word of a trial's spike bits feeds four steps.
// Element (col tile c, j, s, q, col, e) = W[8 (16 j + 4 q + s) + e][16 c + col].
//
// When every weight is an integer multiple k * 2^-e of one power of two with
// |k| <= 127, the weights are also kept as int8 numerators for
// v_mfma_i32_16x16x64_i8: the same K blocks j of 128 in 2 steps s x 4 lane
// groups q x 16, lane group q at step (j, s) contracting pre-neurons
// 32 (4 j + q) + 16 s + i, i = 0..15 (one 16-bit half of a spike word).
// Element (col tile c, j, s, q, col, i) = k(W[32 (4j+q) + 16 s + i][16 c + col]).
// Integer products and sums are exact; the sum times 2^-e is the exact input.
struct DenseArgs {
  DevNet n;
  const uint16_t* wt;  // [Npad / 16][kpad / 128][4][4][16][8] bf16 bits
  int32_t kpad;
  const int8_t* wt8;   // [Npad / 16][kpad / 128][2][4][16][16] int8 numerators, or null
  float scale8;        // 2^-e
};

size_t dense_tiled_elems(int32_t npad, int32_t kpad);
void tile_dense_weights(const float* W, int32_t n, int32_t npad, int32_t kpad, uint16_t* out);
// Smallest e in [0, 24] with every W * 2^e an integer of magnitude <= 127, or -1.
int32_t int8_exponent(const float* W, int64_t count);
void tile_dense_weights_i8(const float* W, int32_t n, int32_t npad, int32_t kpad, int32_t e, int8_t* out);

// Dense delay-1 weights of a large net, row-major int8 numerators:
// W[i][j] = w8[i * pitch + j] * scale, scale = 2^-e, pitch = Npad (rows N).
// Sums of at most kRowsMaxNeurons numerators of magnitude <= 128 stay below
// 2^24 and convert to binary32 exactly.
constexpr int32_t kRowsMaxNeurons = 131072;
struct RowsArgs {
  DevNet n;
  const int8_t* w8;
  int64_t pitch;
  float scale;
};

// Event-driven ("push") delivery: out-going synapses of every neuron (CSR by
// pre-neuron) and a ring of D + 1 accumulator rows; a spike of neuron i at t
// adds w into row (t + d) mod (D+1) at the post-neuron.
// Push record meta: bits 0..19 post-neuron, bits 20..25 delay - 1.
struct PushArgs {
  DevNet n;
  const Rec* orecs;         // [nnz] out-going records grouped by pre-neuron
  const int32_t* optr;      // [Npad + 1] first out-record of every neuron
  const int32_t* wg_group;  // [P + 1] first group of every slice
  float* accum;             // [D + 1][B][Npad] pending synaptic input
  uint32_t* flags;          // [B][P][64] step + 1 finished by every slice (one flag per 256 bytes)
  uint32_t* status;         // set to nonzero when a wait times out
  int32_t P;
  int32_t ng_max;
};

struct HostPush {
  std::vector<Rec> orecs;
  std::vector<int32_t> optr;  // [Npad + 1]
};
HostPush build_push_layout(int32_t n, int32_t npad, int64_t nnz, const int32_t* pre, const int32_t* post,
                           const float* w, const uint8_t* delay);

// Batched execution of independent networks in one persistent launch.
// Networks too large for one workgroup run as a team of workgroups (their
// slices, exchanging spikes through the network's mailbox); the others are
// pulled one (network, trial) at a time from a work queue by whichever
// workgroup is free.  Records are read from global memory (L2-resident for
// small networks); the spike ring of every network lives in LDS.
struct BatchNet {
  SimArgs team;    // slice plan of a team network (P > 1)
  SimArgs single;  // one-slice plan (P = 1)
};

struct BatchArgs {
  const BatchNet* nets;
  const int4* team;    // [n_team] (network, slice, trial, t0) of workgroups 0 .. n_team - 1
  const int4* queue;   // [n_queue] (network, trial, t0, -) in the order they are taken
  int32_t n_team;
  int32_t n_queue;
  int32_t* queue_head; // next queue entry to take (zero before the launch)
};

constexpr int kBatchThreads = 512;
constexpr int kBatchMaxGroups = 24;  // groups per slice: 8 waves x 3 groups per wave

}  // namespace snmi
#include "../../include/superneuro_mi.h"
namespace snmi {
size_t bptt_workspace_bytes(const sn_bptt_desc& d);
hipError_t bptt_forward(const sn_bptt_desc& d, const float* W, const float* x, float* counts, void* ws, hipStream_t s);
// bptt_forward with the library's per-device scratch array as workspace; the
// caller has checked bptt_workspace_bytes(d) <= SN_BPTT_NOALLOC_WORKSPACE_BYTES
hipError_t bptt_forward_noalloc(const sn_bptt_desc& d, const float* W, const float* x, float* counts, hipStream_t s);
hipError_t bptt_backward(const sn_bptt_desc& d, const float* W, const float* x, const float* dcounts, const void* ws,
                         float* dW, hipStream_t s);

// Kernel launchers (kernels.hip).  All return hipSuccess or the launch error.
size_t sim_lds_bytes(const DevNet& n, int ng_max, int64_t max_recs, int nwave, bool recs_lds, bool ring_lds,
                     bool compact = false);
size_t lds_limit();
int sim_threads(int ng_max, int64_t max_recs);
int sim_npt(int ng_max, int64_t max_recs);
hipError_t launch_sim(const SimArgs& a, bool recs_lds, bool ring_lds, int32_t t0, int32_t steps, hipStream_t s);
hipError_t launch_prefill_mailbox(const SimArgs& a, int32_t t0, hipStream_t s);
size_t batch_lds_bytes(const DevNet& n, int ng_max);
int batch_blocks_per_cu(size_t lds, bool compact);
hipError_t launch_zero_i32(int32_t* p, hipStream_t s);
hipError_t launch_batch(const BatchArgs& a, int grid, size_t lds, int32_t steps, bool compact, hipStream_t s);
// 4-byte copies of the layout's records (compact_record) for a net of n
// neurons and maximum delay max_delay, or empty when the net or a weight
// does not allow them; *scale receives 2^-e.
std::vector<uint32_t> compact_records(const HostLayout& L, int32_t n, int32_t max_delay, float* scale);
hipError_t launch_step(const DevNet& n, int32_t t, hipStream_t s);
// Per-step kernel of nets whose D history rows do not fit in 64 KB of LDS
// (wide.hip).  `grid` workgroups per trial own gpw groups each and stage Dl
// history rows at a time in LDS (plus the row of one step later for step
// pairs); with P > 1 phases the layout orders part A
// by delay phase so that every lookup is an LDS read (at most kWideMaxPhases
// phases; otherwise P = 1 and delays above Dl read the raster in memory).
constexpr int kWideMaxPhases = 4;
struct WidePlan {
  int grid = 0, gpw = 0, Dl = 0, P = 1;
  int block = 1;  // steps per block (lane records): 4, 2, or 1 (no extra rows)
  int shift = 0;  // block - 1: LDS rows kept for the rows of later steps
};
bool wide_net(const DevNet& n);
WidePlan wide_plan(const DevNet& n, int cus);
hipError_t prepare_wide_kernel(const DevNet& n, int cus);
hipError_t launch_step_wide(const DevNet& n, int32_t t, int cus, hipStream_t s);
// A block of K = step_block(n) > 1 steps t .. t + K - 1 (wide nets with
// lane records and n.held): one pass over every record, a record of delay d
// adding into steps t .. t + min(d, K) - 1 (its source word for step t + i
// is i staged rows below its word for step t), then for i = 1 .. K - 1 a
// short kernel that adds the records of delays 1 .. i to step t + i and
// updates it.  1: no blocks.
int step_block(const DevNet& n);
hipError_t launch_step_block(const DevNet& n, int32_t t, hipStream_t s);
int wide_block(const DevNet& n, int cus);
hipError_t launch_block_wide(const DevNet& n, int32_t t, int cus, hipStream_t s);
hipError_t launch_stdp(const StdpArgs& a, int32_t t, hipStream_t s);
hipError_t launch_hist_build(const StdpArgs& a, int32_t t0, hipStream_t s);
// per-step kernel with plasticity: applies the rule of step t - 1 when apply != 0
hipError_t launch_step_stdp(const StdpArgs& a, int32_t t, int apply, hipStream_t s);
hipError_t prepare_stdp_kernel();
hipError_t prepare_step_kernel(const DevNet& n);
hipError_t launch_dense_step(const DenseArgs& a, int32_t t, hipStream_t s);
hipError_t launch_dense_rows(const RowsArgs& a, int32_t t, hipStream_t s);
hipError_t launch_push(const PushArgs& a, int32_t t0, int32_t steps, hipStream_t s);
hipError_t prepare_dense_kernel(int32_t kpad);
size_t dense_persist_lds_bytes(int32_t kpad);
hipError_t launch_dense_persist(const DenseArgs& a, uint32_t* flags, uint32_t* status, int32_t t0, int32_t steps,
                                hipStream_t s);
size_t dense_lds_bytes(int32_t kpad);
hipError_t launch_reset_state(const DevNet& n, hipStream_t s);
hipError_t launch_repack_input(const DevNet& n, int32_t t0, int32_t steps, const uint32_t* bits,
                               hipStream_t s);
hipError_t launch_unpack_raster(const DevNet& n, int32_t t0, int32_t steps, uint32_t* out, hipStream_t s);

}  // namespace snmi
