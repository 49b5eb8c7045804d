/*
 * superneuro_mi.h -- C ABI of an MI355X (gfx950) library that simulates
 * homogeneous networks of leaky integrate-and-fire neurons with synaptic
 * delays in the matrix form of SuperNeuro (Date et al., ICONS'23, §2.1).
 *
 * Model (§2.1).  Every neuron j carries four parameters -- threshold theta_j,
 * leak lambda_j, reset state r_j, refractory period R_j -- plus the amplitude
 * a_j of an external spike.  Parameters and state are vectors over neurons.
 * A synapse i -> j carries a weight w (entry (i, j) of the weight matrix:
 * row = pre-neuron, column = post-neuron) and an integer delay d >= 1; the
 * paper realises d > 1 with d-1 unit-delay relay neurons, this library with a
 * spike history, which yields the same spike times.  Step t, for every
 * neuron, using only spikes of steps < t and the external spikes of step t:
 *   1. leak: U = V(t-1) moved towards r_j by lambda_j without crossing r_j;
 *   2. synaptic input: U += sum of w over synapses whose pre-neuron spiked at
 *      t - d;
 *   3. external input: U += a_j if neuron j has an external spike at t;
 *   4. candidate spike: U > theta_j (strictly greater);
 *   5. refractory: while the refractory counter is non-zero the spike is
 *      suppressed and the counter decremented;
 *   6. reset: an emitted spike sets V = r_j and the counter to R_j;
 *      otherwise V = U.
 * Initial state (and after sn_reset_state): V = r, counters 0, no spikes.
 *
 * Numbers.  State and arithmetic are IEEE binary32.  When every weight,
 * threshold, leak, reset and amplitude is a multiple of 2^-6 and every
 * partial sum stays below 2^17 in magnitude, all sums are exact, so results
 * do not depend on summation order and match any exact reference bit for bit.
 *
 * Threading.  A network object may be used from one host thread at a time.
 * All device work of a network is issued on the stream given at creation.
 *
 * Errors.  Every call returns SN_OK (0) or a negative sn_status; no C++
 * exception crosses this interface.  sn_last_error() returns a thread-local
 * message describing the most recent failure of the calling thread.
 * Validation failures (SN_EINVAL, SN_ERANGE, SN_EINEXACT) leave the network
 * unchanged.  A failed HIP call returns SN_EDEVICE and poisons the network:
 * every later call on it except sn_destroy_network returns SN_ESTATE.
 */
#ifndef SUPERNEURO_MI_H
#define SUPERNEURO_MI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sn_status;
enum {
  SN_OK = 0,
  SN_EINVAL = -1,    /* malformed argument (null pointer, bad size, non-finite value) */
  SN_ENOMEM = -2,    /* device or host allocation failed */
  SN_EDEVICE = -3,   /* a HIP call failed; the network is poisoned */
  SN_ESTATE = -4,    /* call out of order, or network poisoned earlier */
  SN_ERANGE = -5,    /* index, delay, size or step outside the supported range */
  SN_EINEXACT = -6   /* a dense weight is not exactly representable in bfloat16 */
};

/* Limits of this build. */
#define SN_MAX_NEURONS (1 << 20)  /* pre-neuron index packs into 20 bits */
#define SN_MAX_DELAY 64           /* delay - 1 packs into 6 bits */

/* Delivery / execution strategies (sn_set_path).  AUTO picks one from the
 * network's size, density and trial count; the others force one, for
 * benchmarking and testing.  Every strategy computes identical results. */
enum {
  SN_PATH_AUTO = 0,
  SN_PATH_SMALL = 1,    /* one workgroup per trial runs all requested steps in one launch */
  SN_PATH_STEP = 2,     /* one launch per step: pull delivery over post-neuron groups */
  SN_PATH_PERSIST = 3,  /* one cooperative launch for all steps, grid barrier per step */
  SN_PATH_DENSE = 4,    /* dense weights on matrix cores (needs sn_load_dense_weights): one cooperative
                           launch with the weights resident on chip when they fit, else as SN_PATH_DENSE_STEP */
  SN_PATH_PUSH = 5,     /* event-driven: only synapses of spiking neurons are touched (low firing rates) */
  SN_PATH_DENSE_STEP = 6, /* dense weights on matrix cores, one launch per step */
  SN_PATH_DENSE_ROWS = 10 /* dense int8 rows (needs sn_load_dense_rows_i8): one launch per step reading
                             only the rows of the neurons that spiked at the step before */
};

/* Device-memory allocator.  alloc returns device memory of at least `bytes`
 * bytes (256-byte aligned) or NULL; free releases it.  Both are called only
 * from the thread that calls into the library.  A NULL allocator means
 * hipMalloc / hipFree. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} sn_allocator;

/* Neuron population (§2.1: threshold, leak, reset state and refractory
 * period per neuron, plus the external-spike amplitude).  Each per-neuron
 * array is optional: NULL selects the matching *_scalar for every neuron.
 * Arrays are host memory of n_neurons elements, read during the call only.
 * Requirements: thresholds, resets and amplitudes finite; leaks >= 0
 * (+infinity allowed: the state returns to r every step, as the paper's
 * relay neurons); refractory periods 0..255. */
typedef struct {
  int32_t n_neurons;          /* N, 1 .. SN_MAX_NEURONS */
  int32_t n_trials;           /* B >= 1 independent copies of the state and inputs, sharing weights and parameters */
  int32_t max_delay;          /* D, 1 .. SN_MAX_DELAY: largest synaptic delay that will be loaded */
  const float* threshold;
  const float* leak;
  const float* reset;
  const uint8_t* refractory;
  const float* amplitude;
  float threshold_scalar;
  float leak_scalar;
  float reset_scalar;
  float amplitude_scalar;
  uint8_t refractory_scalar;
} sn_net_desc;

typedef struct sn_net sn_net;

/* Creates a network on the current HIP device.  `hip_stream` is a
 * hipStream_t (NULL: the null stream); all device work of the network is
 * ordered on it.  `alloc` may be NULL (see sn_allocator).  On success *out
 * owns every device buffer it allocates; the state is the initial state.
 * Errors: SN_EINVAL (null desc/out, non-finite parameter, negative leak),
 * SN_ERANGE (N, B or D outside the limits), SN_ENOMEM, SN_EDEVICE. */
sn_status sn_create_network(const sn_net_desc* desc, const sn_allocator* alloc,
                            void* hip_stream, sn_net** out);

/* Loads the synapses as a host COO list of nnz entries (§2.1: weight and
 * delay per synapse, W[pre][post]).  pre/post in [0, N), w finite,
 * delay in [1, D].  Duplicate (pre, post) pairs act as separate synapses
 * (their weights add); self-synapses are allowed.  nnz may be 0.  Replaces
 * any earlier synapses; the simulation state is kept.  Arrays are read during
 * the call only.  On the device the synapses are grouped by 64 post-neurons
 * and padded with filler records (about 1.2 records per synapse for random
 * nets, more for skewed in-degrees); the padded count must stay below 2^31.
 * Errors: SN_EINVAL (null arrays with nnz > 0, non-finite w), SN_ERANGE
 * (index or delay out of range, nnz >= 2^31, or the padded count >= 2^31),
 * SN_ENOMEM (the network is unchanged), SN_EDEVICE. */
sn_status sn_load_weights_delays(sn_net* net, int64_t nnz, const int32_t* pre, const int32_t* post,
                                 const float* w, const uint8_t* delay);

/* Loads a dense N x N weight matrix (host, row-major, row = pre-neuron,
 * column = post-neuron, §2.1) whose synapses all have delay `delay`; zero
 * entries are absent synapses.  This build supports delay == 1.  Weights are
 * held as bfloat16 for the matrix cores, so every entry must be exactly
 * representable in bfloat16 (SN_EINEXACT otherwise).  Enables SN_PATH_DENSE
 * and also loads the nonzeros as a sparse list for the other paths.
 * Errors: SN_EINVAL, SN_ERANGE (delay), SN_EINEXACT, SN_ENOMEM, SN_EDEVICE. */
sn_status sn_load_dense_weights(sn_net* net, const float* W, int32_t delay);

/* Dense delay-1 weights of a large net (the paper's largest run is 100,000
 * neurons all-to-all, §4), given block by block as int8 numerators:
 * W[i][j] = k[i][j] * 2^-e (row = pre-neuron, column = post-neuron, §2.1).
 * `k` is host memory holding rows row0 .. row0+n_rows-1, [n_rows][N]
 * row-major, read during the call only (the copy is complete on return).
 * The first call after creation or after another sn_load_* allocates N x Npad
 * bytes of device memory (Npad = N rounded up to a multiple of 64), zeroed,
 * and drops earlier synapses or dense weights; rows never given stay zero.
 * Every call on the same weights must pass the same e.  A later
 * sn_load_weights_delays or sn_load_dense_weights frees the rows.  Either
 * change of weights returns a path set for the other kind to SN_PATH_AUTO.
 * The net then runs on SN_PATH_DENSE_ROWS (chosen by SN_PATH_AUTO; other
 * paths return SN_ESTATE): each step reads only the rows of the neurons that
 * spiked at the step before, (spikes) x N bytes per trial.  Integer sums of
 * at most 131,072 numerators are exact, and so is their scaling by 2^-e; the
 * results are then exact when thresholds, leaks, resets and amplitudes are
 * multiples of 2^-max(e, 6) and every partial sum of the update stays below
 * 2^(24 - max(e, 6)).  Plasticity and sn_read_weights do not apply.
 * Errors: SN_EINVAL (k NULL with n_rows > 0, e differing from the first
 * call's), SN_ERANGE (N > 131,072, rows outside [0, N), e outside [0, 24]),
 * SN_ENOMEM, SN_EDEVICE. */
sn_status sn_load_dense_rows_i8(sn_net* net, int32_t row0, int32_t n_rows, const int8_t* k, int32_t e);

/* External spikes (§2.1, third step) for steps t0 .. t0+n_steps-1.  `bits`
 * is host memory laid out [B][n_steps][ceil(N/32)] uint32 words; bit (j % 32)
 * of word j / 32 is neuron j.  Bits of neurons >= N are ignored.  Steps never
 * given have no external spikes.  Steps already simulated may be rewritten;
 * that affects only a later sn_reset_state + sn_run.  Errors: SN_EINVAL,
 * SN_ERANGE (t0 < 0 or n_steps < 0), SN_ENOMEM, SN_EDEVICE. */
sn_status sn_set_input_spikes(sn_net* net, int32_t t0, int32_t n_steps, const uint32_t* bits);

/* Same, with `bits` in device memory (same layout), copied on the stream. */
sn_status sn_set_input_spikes_device(sn_net* net, int32_t t0, int32_t n_steps, const uint32_t* bits);

/* Advances the simulation by n_steps steps (t -> t + n_steps), asynchronously
 * on the network's stream.  Resumable: run(a) followed by run(b) equals
 * run(a + b).  Requires synapses (sn_load_* may have loaded zero synapses).
 * Errors: SN_ESTATE (no synapses loaded, or poisoned), SN_ERANGE, SN_ENOMEM,
 * SN_EDEVICE. */
sn_status sn_run(sn_net* net, int32_t n_steps);

/* Blocks until all device work of the network has finished. */
sn_status sn_synchronize(sn_net* net);

/* Copies the spikes of steps t0 .. t0+n_steps-1 to host memory `out`, laid
 * out like sn_set_input_spikes ([B][n_steps][ceil(N/32)] words).  Waits for
 * the work in flight.  Errors: SN_EINVAL, SN_ERANGE (steps not simulated). */
sn_status sn_read_raster(sn_net* net, int32_t t0, int32_t n_steps, uint32_t* out);

/* Copies the state after the last simulated step: V [B][N] floats and the
 * remaining refractory steps [B][N] (either pointer may be NULL).  Waits for
 * the work in flight. */
sn_status sn_read_state(sn_net* net, float* V, uint8_t* refractory_left);

/* Device-memory variants of sn_read_raster and sn_read_state, for callers
 * that keep the results on the GPU (as input of their own kernels, or to
 * overlap the readback with host work).  Same layouts; `out`, `V` and
 * `refractory_left` are device memory of the network's device, owned by the
 * caller and not overlapping the network's own buffers.  Asynchronous on the
 * network's stream: they enqueue a repack kernel (raster) or strided copies
 * (state) and return without waiting, so the outputs are complete once the
 * stream has reached them (sn_synchronize, or the caller's own event wait on
 * that stream).  A spike-exchange time-out of an earlier run is reported by
 * the next synchronising call (sn_synchronize, sn_read_raster,
 * sn_read_state), not by these.  Errors: SN_EINVAL (NULL out with
 * n_steps > 0), SN_ERANGE (steps not simulated), SN_ESTATE (another device
 * current), SN_EDEVICE. */
sn_status sn_read_raster_device(sn_net* net, int32_t t0, int32_t n_steps, uint32_t* out);
sn_status sn_read_state_device(sn_net* net, float* V, uint8_t* refractory_left);

/* Returns to the initial state (t = 0, V = r, counters 0, history cleared);
 * synapses and external spikes are kept.  Asynchronous on the stream. */
sn_status sn_reset_state(sn_net* net);

/* Selects the execution strategy (SN_PATH_*); checked at the next sn_run. */
sn_status sn_set_path(sn_net* net, int32_t path);

/* Number of slices (workgroups per trial) of SN_PATH_PERSIST: 0 picks one
 * slice per 64-neuron group, up to one per compute unit; 1..256 requests a
 * count, raised to the
 * minimum a slice can hold (128 groups of 64 neurons per slice) and lowered
 * to the number of groups.  A tuning knob: results do not change.
 * Errors: SN_ERANGE. */
sn_status sn_set_slices(sn_net* net, int32_t slices);

/* Spike-timing-dependent plasticity (§2.1 names STDP as the learning of the
 * matrix mode without a rule; this is a chosen, table-driven nearest-neighbour
 * pair rule).  A spike of pre-neuron i at step tau arrives at j at tau + d.
 * After the update of step t, for every synapse i -> j of delay d:
 *   - if j spiked at t, the latest arrival t_a <= t with lag = t - t_a < window
 *     adds ltp[lag];
 *   - if a spike of i arrives at t, the latest spike of j at t - lag,
 *     1 <= lag <= window, subtracts ltd[lag - 1];
 *   - the weight is then clipped to [w_min, w_max].
 * The new weights act from step t + 1.  With table entries and bounds that
 * are multiples of 2^-6 the weights stay on that grid and runs stay exact. */
typedef struct {
  int32_t window;  /* 1..16 steps */
  float ltp[16];   /* entries 0 .. window - 1 are used */
  float ltd[16];
  float w_min, w_max;
} sn_stdp_desc;

/* Turns plasticity on with the rule above (desc copied), or off (desc NULL).
 * Needs a synapse list (not dense weights) and one trial.  While on, sn_run
 * uses the per-step path (SN_PATH_AUTO or SN_PATH_STEP, else SN_ESTATE) and
 * applies the rule after every step; the weights change in place
 * (sn_reset_state does not restore them; sn_load_weights_delays does), and
 * the event-driven path refuses to run (SN_ESTATE) until the weights are
 * loaded again.  Turning it on also drops the 4-byte copies of the records
 * that some kernels read, so that after it is turned off every other path
 * runs with the learned weights (until sn_load_weights_delays rebuilds them).
 * Errors: SN_ESTATE, SN_ERANGE (window, trials), SN_EINVAL (non-finite
 * entries, w_min > w_max), SN_EDEVICE. */
sn_status sn_set_stdp(sn_net* net, const sn_stdp_desc* desc);

/* Copies the current synapse weights to w [nnz], in the order of the last
 * sn_load_weights_delays (dense weights: their non-zero entries, row-major).
 * Synchronizes the network's stream. */
sn_status sn_read_weights(sn_net* net, float* w);

/* Autotuner: times every strategy that can run this network (the
 * single-workgroup and multi-slice persistent kernels, the latter at several
 * slice counts, the per-step and event-driven paths; for dense weights the
 * persistent and per-step matrix-core paths) over `steps` steps from the
 * initial state, each after one untimed run of the same length, with HIP
 * events on the network's stream.  The fastest becomes the network's path and
 * slice count, as if set with sn_set_path / sn_set_slices; results do not
 * depend on the choice.  Uses the external spikes already set for those
 * steps.  The state is reset (t = 0) before every trial and at the end.
 * *path_out / *slices_out (either may be NULL) receive the choice
 * (slices 0 = the default plan).  1 <= steps <= 4096, else SN_ERANGE; a
 * device error poisons the network as sn_run would; SN_ESTATE while
 * plasticity is on. */
sn_status sn_autotune(sn_net* net, int32_t steps, int32_t* path_out, int32_t* slices_out);

/* Reports the number of simulated steps so far (*t) and the strategy the
 * last sn_run used (*path, SN_PATH_AUTO before the first run): one of the
 * SN_PATH_* values, or 7 (a batch, sn_batch_run), 8 (SN_PATH_DENSE as one
 * persistent launch on bfloat16 matrix cores) or 9 (the same on int8 matrix
 * cores, used when every dense weight is k * 2^-e with |k| <= 127). */
sn_status sn_get_progress(sn_net* net, int32_t* t, int32_t* path);

/* ---- Batched execution of many independent networks --------------------
 * A batch runs its networks together in one persistent launch: networks too
 * large for one workgroup are split across a team of workgroups, the others
 * are taken one at a time from a device work queue by free workgroups.  Each
 * network keeps its own state, history and inputs and stays readable with
 * sn_read_raster / sn_read_state; results equal separate sn_run calls.
 * All networks must be on the same device, have synapses loaded, and have no
 * unfinished work on other streams; the batch uses the first network's
 * stream.  Networks may have different sizes, delays, trial counts and step
 * counters.  The batch holds no reference count: destroy it before its
 * networks.  Limits: N <= 2048 * (number of compute units), spike ring
 * (D + 1) * ceil(N/32) * 4 bytes <= 96 KB per network. */
typedef struct sn_batch sn_batch;

/* Plans a batch over nets[0 .. count-1].  Errors: SN_EINVAL (null or
 * duplicate networks), SN_ESTATE (a network without a synapse list, with
 * plasticity on -- a batch does not apply the rule -- or poisoned),
 * SN_ERANGE (a network outside the limits, or count outside [1, 65536]),
 * SN_ENOMEM, SN_EDEVICE. */
sn_status sn_batch_create(sn_net* const* nets, int32_t count, sn_batch** out);

/* Advances every network of the batch by n_steps steps, asynchronously on
 * the batch's stream.  Errors: SN_ESTATE (as sn_batch_create: plasticity was
 * turned on or dense rows loaded since), SN_ERANGE, SN_ENOMEM, SN_EDEVICE
 * (poisons the batch and its networks). */
sn_status sn_batch_run(sn_batch* batch, int32_t n_steps);

/* Schedule autotuner of a batch (the batching direction: a schedule per
 * size class of networks): times candidate schedules of the batch -- how
 * large a share of one step's records a slice of a network may take before
 * the network is split across a team of workgroups (as a multiple of the
 * average load per workgroup), and what share of the workgroups teams may
 * occupy, the rest running the smaller networks from the queue -- over
 * `steps` steps from the initial state, each after one untimed run of the
 * same length, with HIP events on the batch's stream, and keeps the fastest.
 * Results do not depend on the schedule.  Every network of the batch is
 * reset (t = 0) before every candidate and at the end; external spikes are
 * kept.  *target_mult_out / *team_share_out (either may be NULL) receive the
 * chosen knobs (sn_batch_create uses 1.0 and 0.75).  1 <= steps <= 4096, else
 * SN_ERANGE; SN_ESTATE as sn_batch_run; a device error poisons the batch. */
sn_status sn_batch_autotune(sn_batch* batch, int32_t steps, float* target_mult_out, float* team_share_out);

/* Frees the batch (not its networks).  NULL is ignored. */
void sn_batch_destroy(sn_batch* batch);

/* ---- Surrogate-gradient training of a recurrent LIF layer --------------
 * The layer is the model above with delay-1 recurrent weights W_rec
 * [N][N], an external input x_t [B][Nin] entering through W_in [Nin][N],
 * one threshold / leak / reset for all neurons and no refractory period:
 *   U_t = leak(V_{t-1}) + s_{t-1} W_rec + x_t W_in,  s_t = (U_t > theta),
 *   V_t = (1 - s_t) U_t + s_t r,   count = sum over t of s_t.
 * Weights are passed stacked as W_cat [N + Nin][N] (rows 0..N-1: W_rec).
 * The backward pass replaces the threshold's derivative by the fast-sigmoid
 * surrogate 1 / (1 + k |U - theta|)^2 (k = slope), which is the exact
 * derivative of the relaxed spike 1/2 + x / (1 + k|x|), x = U - theta; with
 * relaxed != 0 the forward itself uses the relaxed spike, so the gradient is
 * then the exact gradient of that forward.
 * The clamped leak passes gradient only where it does not clamp.  Spikes are
 * kept bit-packed (relaxed: as floats) and V every checkpoint_every steps;
 * the backward pass recomputes each segment from its checkpoint.
 * All arrays are device memory in binary32, row-major; work is issued on
 * hip_stream (NULL: the null stream). */
typedef struct {
  int32_t n_neurons;         /* N, a multiple of 32 */
  int32_t n_inputs;          /* Nin >= 0 */
  int32_t n_trials;          /* B >= 1 */
  int32_t n_steps;           /* T >= 1 */
  int32_t checkpoint_every;  /* K >= 1 */
  float threshold, leak, reset, slope;
  int32_t relaxed;
} sn_bptt_desc;

/* Bytes of device workspace sn_bptt_forward / sn_bptt_backward need (0 if
 * the descriptor is invalid). */
size_t sn_bptt_workspace_bytes(const sn_bptt_desc* d);

/* Forward pass: x [T][B][Nin] (spikes as 0/1 or any real input) -> spike
 * counts [B][N]; fills the workspace for the backward pass.
 * Errors: SN_EINVAL (null pointer, bad descriptor), SN_EDEVICE. */
sn_status sn_bptt_forward(const sn_bptt_desc* d, const float* W_cat, const float* x, float* counts,
                          void* workspace, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * forward pass of sn_bptt_forward, same arguments and results, with its
 * workspace in a device buffer the library holds instead of a caller's.  The
 * call allocates nothing.  The buffer is SN_BPTT_NOALLOC_WORKSPACE_BYTES on
 * every device the library runs on, kept until the process ends; a
 * descriptor whose sn_bptt_workspace_bytes exceeds it gets SN_ERANGE.  Every
 * call on a device uses that device's one buffer, so calls that overlap on
 * one device (different streams or host threads) race and give undefined
 * counts; order them on one stream.  Only counts are produced: the buffer
 * is not kept for a backward pass.  Work is issued on hip_stream, which
 * must belong to the current device.
 * Errors: SN_EINVAL (null pointer, bad descriptor), SN_ERANGE, SN_EDEVICE. */
#define SN_BPTT_NOALLOC_WORKSPACE_BYTES ((size_t)64 << 20)
sn_status sn_bptt_forward_noalloc(const sn_bptt_desc* d, const float* W_cat, const float* x, float* counts,
                                  void* hip_stream);

/* Backward pass after sn_bptt_forward with the same inputs and workspace:
 * given dL/dcounts [B][N], writes dL/dW_cat [N + Nin][N].
 * Errors: SN_EINVAL, SN_EDEVICE. */
sn_status sn_bptt_backward(const sn_bptt_desc* d, const float* W_cat, const float* x, const float* dcounts,
                           const void* workspace, float* dW_cat, void* hip_stream);

/* Frees the network and its device memory after its work has finished.
 * NULL is ignored. */
void sn_destroy_network(sn_net* net);

/* Message of the calling thread's most recent failure ("" if none). */
const char* sn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SUPERNEURO_MI_H */
