// C ABI (include/superneuro_mi.h): validation, device memory, layout upload,
// path selection and launches.  Host-only code; kernels live in kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/superneuro_mi.h"
#include "sn_internal.h"

using namespace snmi;

namespace {

thread_local std::string g_err;

sn_status fail(sn_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

}  // namespace

struct sn_net {
  DevNet d{};
  hipStream_t stream = nullptr;
  sn_allocator alloc{};
  bool custom_alloc = false;
  int device = 0;
  std::vector<float> h_reset;
  // owned device buffers
  std::vector<void*> owned;
  int64_t tcap = 0;  // rows allocated in raster and ext
  int32_t t = 0;     // steps simulated
  bool synapses_loaded = false;
  bool poisoned = false;
  int32_t path = SN_PATH_AUTO;
  int32_t last_path = SN_PATH_AUTO;
  // synapse buffers (replaced by a new load)
  void* recs = nullptr;
  void* gptr = nullptr;
  void* gsplit = nullptr;
  void* wsec = nullptr;  // delay-phase sections of the wide per-step kernel
  void* crecs = nullptr; // 4-byte record copies (compact_records), when the net allows them
  void* lrecs = nullptr; // lane records of a lane-only layout (wide nets) and their offsets
  void* lgptr = nullptr;
  void* lwsec = nullptr;
  // persistent-kernel plans: one slice (SMALL) and several slices (PERSIST)
  struct DevPlan {
    SlicePlan host;
    void* wg = nullptr;  // [P + 1] int32: first group of every slice
    bool ok = false;
  };
  DevPlan small, persist;
  // event-driven delivery: out-going records, accumulator ring, flags
  void* orecs = nullptr;
  void* optr = nullptr;
  void* push_wg = nullptr;
  float* accum = nullptr;
  uint32_t* push_flags = nullptr;
  int32_t push_P = 0, push_ng_max = 0;
  // dense matrix-core weights (sn_load_dense_weights)
  void* wt = nullptr;
  void* wt8 = nullptr;   // int8 numerators when the weights allow (see DenseArgs)
  float scale8 = 0.f;
  int32_t kpad = 0;
  bool dense_loaded = false;
  // dense int8 rows (sn_load_dense_rows_i8): [N][Npad] numerators, scale 2^-rows_e
  void* rows8 = nullptr;
  int32_t rows_e = -1;
  bool rows_loaded = false;
  // cached graph of per-step launches
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  int32_t graph_path = -1, graph_t0 = -1, graph_steps = -1, graph_stdp = -1;
  const void* graph_key[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int32_t slices_req = 0;
  // plasticity (sn_set_stdp): on, its arguments, a generation for the graph
  // cache, and whether the event-driven records still hold the loaded weights
  bool stdp_on = false;
  StdpArgs stdp{};
  int32_t stdp_gen = 0;
  uint64_t* stdp_hist = nullptr;  // [2][Npad] spike-history words of the plasticity kernel
  bool push_stale = false;
  int64_t nnz_loaded = 0;
  uint64_t* mailbox = nullptr;  // [D + 1][B][2G] tagged spike words
  uint32_t* slice_flags = nullptr;  // [B][256][64]
  uint32_t* status = nullptr;
  HostLayout layout;          // kept to re-plan when the slice count changes
};

namespace {

void* dev_alloc(sn_net* n, size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (n->custom_alloc) {
    p = n->alloc.alloc(bytes, n->alloc.ctx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  return p;
}

void dev_free(sn_net* n, void* p) {
  if (!p) return;
  if (n->custom_alloc) {
    n->alloc.free(p, n->alloc.ctx);
  } else {
    (void)hipFree(p);
  }
}

sn_status device_error(sn_net* n, hipError_t e, const char* what) {
  n->poisoned = true;
  return fail(SN_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define SN_HIP(net, call)                                  \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return device_error(net, e_, #call); \
  } while (0)

// The cached graph holds kernel arguments by value (sizes, plans, rule
// parameters); a new set of weights invalidates it.  Called after the stream
// has been synchronized.
void drop_graph(sn_net* n) {
  if (n->graph) (void)hipGraphExecDestroy(n->graph);
  n->graph = nullptr;
  n->graph_path = -1;
}

sn_status check_usable(sn_net* n) {
  if (!n) return fail(SN_EINVAL, "network is NULL");
  if (n->poisoned) return fail(SN_ESTATE, "network is poisoned by an earlier device error");
  return SN_OK;
}

// Grows raster and ext to hold at least `rows` steps (doubling), preserving
// the simulated rows of the raster and all rows of ext.
sn_status ensure_rows(sn_net* n, int64_t rows) {
  if (rows <= n->tcap) return SN_OK;
  int64_t cap = std::max<int64_t>(rows, std::max<int64_t>(64, n->tcap * 2));
  const size_t row_bytes = static_cast<size_t>(n->d.B) * n->d.G * sizeof(uint64_t);
  void* nr = dev_alloc(n, cap * row_bytes);
  void* ne = dev_alloc(n, cap * row_bytes);
  if (!nr || !ne) {
    dev_free(n, nr);
    dev_free(n, ne);
    return fail(SN_ENOMEM, "cannot allocate %lld spike rows", static_cast<long long>(cap));
  }
  SN_HIP(n, hipMemsetAsync(nr, 0, cap * row_bytes, n->stream));
  SN_HIP(n, hipMemsetAsync(ne, 0, cap * row_bytes, n->stream));
  if (n->tcap > 0) {
    SN_HIP(n, hipMemcpyAsync(nr, n->d.raster, n->tcap * row_bytes, hipMemcpyDeviceToDevice, n->stream));
    SN_HIP(n, hipMemcpyAsync(ne, n->d.ext, n->tcap * row_bytes, hipMemcpyDeviceToDevice, n->stream));
  }
  // old buffers may still be read by queued kernels: free after the stream drains
  if (n->tcap > 0) {
    SN_HIP(n, hipStreamSynchronize(n->stream));
    dev_free(n, n->d.raster);
    dev_free(n, const_cast<uint64_t*>(n->d.ext));
  }
  n->d.raster = static_cast<uint64_t*>(nr);
  n->d.ext = static_cast<const uint64_t*>(ne);
  n->tcap = cap;
  return SN_OK;
}

// Chooses where the persistent kernel keeps records and the spike ring;
// false if the slice plan cannot run at all.
bool fit_plan(const DevNet& d, SlicePlan& p) {
  if (p.P < 1 || sim_npt(p.ng_max, p.max_recs) > 8) return false;
  const int nwave = sim_threads(p.ng_max, p.max_recs) / kGroup;
  // the spike ring goes to LDS whenever it fits beside the accumulators: a
  // global ring costs a device-scope load per synapse
  const bool ring_fits = sim_lds_bytes(d, p.ng_max, 0, nwave, false, true) <= 96 * 1024;
  // (records in LDS, ring in LDS), preferred first
  const bool opts[4][2] = {{true, true}, {false, true}, {true, false}, {false, false}};
  for (const auto& o : opts) {
    if (ring_fits && !o[1]) continue;
    if (sim_lds_bytes(d, p.ng_max, p.max_recs, nwave, o[0], o[1]) <= lds_limit()) {
      p.recs_lds = o[0];
      p.ring_lds = o[1];
      return true;
    }
  }
  return false;
}

constexpr int32_t kMaxCoopGroups = 256;  // one workgroup per CU of an MI355X

// Slice plan for the multi-workgroup persistent kernel: as many slices as
// groups, up to one per compute unit (a slice's delivery time grows with its
// records while the spike exchange costs about the same for any count).
SlicePlan plan_persist(const DevNet& d, const HostLayout& L, int32_t slices_req) {
  const int32_t pmax = std::max(1, kMaxCoopGroups / d.B);
  const int32_t top = std::min(d.G, pmax);
  // a slice holds at most 128 groups (8 per wave of a 1024-thread workgroup)
  const int32_t want = slices_req > 0 ? std::max(slices_req, (d.G + 127) / 128) : top;
  SlicePlan p = partition_groups(L, d.G, std::min(want, top), 128);
  if (!fit_plan(d, p)) p.P = 0;
  return p;
}

// Device slice table of a plan (NULL for a plan that cannot run).  `bad` is
// set when the allocation fails.
void* alloc_plan(sn_net* n, const SlicePlan& p, bool& bad) {
  if (p.P <= 0) return nullptr;
  void* wg = dev_alloc(n, p.wg_group.size() * sizeof(int32_t));
  if (!wg) bad = true;
  return wg;
}

// Installs plan p with its table `wg` (from alloc_plan), freeing the old one.
// The caller has synchronized the stream when queued work may read the old one.
sn_status install_plan(sn_net* n, sn_net::DevPlan& dp, const SlicePlan& p, void* wg) {
  dev_free(n, dp.wg);
  dp.wg = wg;
  dp.host = p;
  dp.ok = p.P > 0;
  if (!dp.ok) return SN_OK;
  SN_HIP(n, hipMemcpyAsync(dp.wg, p.wg_group.data(), p.wg_group.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           n->stream));
  SN_HIP(n, hipStreamSynchronize(n->stream));  // the host table may die after return
  return SN_OK;
}

// Replaces one plan; on ENOMEM the old plan stays.
sn_status upload_plan(sn_net* n, sn_net::DevPlan& dp, const SlicePlan& p) {
  bool bad = false;
  void* wg = alloc_plan(n, p, bad);
  if (bad) return fail(SN_ENOMEM, "cannot allocate slice tables");
  SN_HIP(n, hipStreamSynchronize(n->stream));  // queued launches may read the old table
  return install_plan(n, dp, p, wg);
}

SimArgs sim_args(sn_net* n, const sn_net::DevPlan& dp) {
  SimArgs a{};
  a.n = n->d;
  a.wg_group = static_cast<const int32_t*>(dp.wg);
  a.mailbox = n->mailbox;
  a.status = n->status;
  a.P = dp.host.P;
  a.ng_max = dp.host.ng_max;
  a.max_recs = dp.host.max_recs;
  return a;
}

// Reads the barrier-timeout flag of the persistent kernel (after a sync).
sn_status check_status(sn_net* n) {
  uint32_t st = 0;
  SN_HIP(n, hipMemcpy(&st, n->status, sizeof(st), hipMemcpyDeviceToHost));
  if (st != 0) {
    n->poisoned = true;
    return fail(SN_EDEVICE, "a spike-exchange wait of the persistent kernel timed out");
  }
  return SN_OK;
}

// Launches steps t0 .. t0+steps-1 of a per-step path, through a cached HIP
// graph when the run is long enough to amortise the capture.
sn_status run_per_step(sn_net* n, int32_t path, int32_t t0, int32_t steps) {
  // wide nets with lane records run blocks of steps (see launch_step_block)
  const int32_t blk = path == SN_PATH_STEP && !n->stdp_on ? step_block(n->d) : 1;
  auto launch_all = [&](hipStream_t s) -> hipError_t {
    for (int32_t k = 0; k < steps; ++k) {
      hipError_t e;
      if (path == SN_PATH_DENSE) {
        DenseArgs a{n->d, static_cast<const uint16_t*>(n->wt), n->kpad, nullptr, 0.f};
        e = launch_dense_step(a, t0 + k, s);
      } else if (path == SN_PATH_DENSE_ROWS) {
        RowsArgs a{n->d, static_cast<const int8_t*>(n->rows8), n->d.Npad, std::ldexp(1.f, -n->rows_e)};
        e = launch_dense_rows(a, t0 + k, s);
      } else if (n->stdp_on) {
        // the rule of step t - 1 is applied inside step t's kernel; the rule
        // of the run's last step by the plasticity kernel
        StdpArgs a = n->stdp;
        a.n = n->d;
        e = launch_step_stdp(a, t0 + k, k > 0 ? 1 : 0, s);
        if (e == hipSuccess && k == steps - 1) e = launch_stdp(a, t0 + k, s);
      } else if (blk > 1 && k + blk <= steps) {
        e = launch_step_block(n->d, t0 + k, s);  // steps t0 + k .. t0 + k + blk - 1
        k += blk - 1;
      } else {
        e = launch_step(n->d, t0 + k, s);
      }
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  if (steps < 32) {
    SN_HIP(n, launch_all(n->stream));
    return SN_OK;
  }
  const void* key[5] = {n->d.raster, n->d.ext, n->d.recs, n->wt, n->rows8};
  const int32_t stdp_key = n->stdp_on ? n->stdp_gen : 0;
  const bool hit = n->graph && n->graph_path == path && n->graph_t0 == t0 && n->graph_steps == steps &&
                   n->graph_stdp == stdp_key && std::equal(key, key + 5, n->graph_key);
  if (!hit) {
    if (n->graph) {
      SN_HIP(n, hipGraphExecDestroy(n->graph));
      n->graph = nullptr;
    }
    if (!n->capture_stream) SN_HIP(n, hipStreamCreateWithFlags(&n->capture_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    SN_HIP(n, hipStreamBeginCapture(n->capture_stream, hipStreamCaptureModeThreadLocal));
    const hipError_t le = launch_all(n->capture_stream);
    const hipError_t ce = hipStreamEndCapture(n->capture_stream, &g);
    if (le != hipSuccess) return device_error(n, le, "kernel launch during graph capture");
    if (ce != hipSuccess) return device_error(n, ce, "hipStreamEndCapture");
    const hipError_t ie = hipGraphInstantiate(&n->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return device_error(n, ie, "hipGraphInstantiate");
    n->graph_path = path;
    n->graph_t0 = t0;
    n->graph_steps = steps;
    n->graph_stdp = stdp_key;
    std::copy(key, key + 5, n->graph_key);
  }
  SN_HIP(n, hipGraphLaunch(n->graph, n->stream));
  return SN_OK;
}

// Event-driven path: slices of whole groups, one workgroup per CU at most.
sn_status run_push(sn_net* n, int32_t t0, int32_t steps) {
  if (!n->push_wg) {
    const int32_t P = std::max(1, std::min(n->d.G, kMaxCoopGroups / n->d.B));
    std::vector<int32_t> wg(P + 1);
    for (int32_t w = 0; w <= P; ++w) wg[w] = static_cast<int32_t>(static_cast<int64_t>(n->d.G) * w / P);
    int32_t ng_max = 0;
    for (int32_t w = 0; w < P; ++w) ng_max = std::max(ng_max, wg[w + 1] - wg[w]);
    const size_t acc_bytes = static_cast<size_t>(n->d.D + 1) * n->d.B * n->d.Npad * sizeof(float);
    const size_t flag_bytes = static_cast<size_t>(n->d.B) * P * 64 * sizeof(uint32_t);
    void* wgp = dev_alloc(n, wg.size() * sizeof(int32_t));
    void* acc = dev_alloc(n, acc_bytes + flag_bytes);
    if (!wgp || !acc) {
      dev_free(n, wgp);
      dev_free(n, acc);
      return fail(SN_ENOMEM, "cannot allocate the accumulator ring");
    }
    SN_HIP(n, hipMemcpyAsync(wgp, wg.data(), wg.size() * sizeof(int32_t), hipMemcpyHostToDevice, n->stream));
    SN_HIP(n, hipStreamSynchronize(n->stream));
    n->push_wg = wgp;
    n->accum = static_cast<float*>(acc);
    n->push_flags = reinterpret_cast<uint32_t*>(static_cast<char*>(acc) + acc_bytes);
    n->push_P = P;
    n->push_ng_max = ng_max;
  }
  PushArgs a{};
  a.n = n->d;
  a.orecs = static_cast<const Rec*>(n->orecs);
  a.optr = static_cast<const int32_t*>(n->optr);
  a.wg_group = static_cast<const int32_t*>(n->push_wg);
  a.accum = n->accum;
  a.flags = n->push_flags;
  a.status = n->status;
  a.P = n->push_P;
  a.ng_max = n->push_ng_max;
  SN_HIP(n, launch_push(a, t0, steps, n->stream));
  return SN_OK;
}

constexpr int32_t kPathBatch = 7;          // sn_get_progress after a batch run
constexpr int32_t kPathDensePersist = 8;   // SN_PATH_DENSE ran as one cooperative launch
constexpr int32_t kPathDensePersistI8 = 9; // ... on the int8 matrix cores

bool on_device_ok(sn_net* n) {
  int cur = -1;
  return hipGetDevice(&cur) == hipSuccess && cur == n->device;
}

}  // namespace

struct sn_batch {
  std::vector<sn_net*> nets;
  hipStream_t stream = nullptr;
  std::vector<SlicePlan> plans;  // per network: team plan (P > 1) or one slice
  void* plan_buf = nullptr;      // device copy of every plan's slice tables
  std::vector<size_t> plan_off;  // int32 offset of each network's tables in plan_buf
  std::vector<int4> team, queue; // task templates (t0 filled at run time)
  std::vector<BatchNet> descs;
  void* nets_buf = nullptr;
  void* team_buf = nullptr;
  void* queue_buf = nullptr;
  void* head_buf = nullptr;
  int grid = 0;
  size_t lds = 0;
  // schedule knobs (sn_batch_autotune): the per-slice cost target as a
  // multiple of the average load per workgroup, and the share of the
  // workgroups that teams of slices may take (the rest run the queue)
  float target_mult = 1.f;
  float team_share = 0.75f;
  bool poisoned = false;
};

namespace {

void batch_free(sn_batch* bt) {
  if (bt->nets.empty()) return;
  sn_net* a = bt->nets[0];
  dev_free(a, bt->plan_buf);
  dev_free(a, bt->nets_buf);
  dev_free(a, bt->team_buf);
  dev_free(a, bt->queue_buf);
  dev_free(a, bt->head_buf);
  bt->plan_buf = bt->nets_buf = bt->team_buf = bt->queue_buf = bt->head_buf = nullptr;
}

// Plans the batch's schedule with the given knobs: how many slices every
// network gets (a team when more than one), the team tasks (largest first,
// slices of a team contiguous) and the queue, and their device tables.  The
// old tables are freed only once the new ones are in place.
sn_status plan_batch(sn_batch* bt, float target_mult, float team_share) {
  const std::vector<sn_net*>& v = bt->nets;
  const int32_t count = static_cast<int32_t>(v.size());
  // cost of one step of one trial: records streamed plus neuron updates
  std::vector<double> cost(count);
  double total = 0;
  for (int32_t k = 0; k < count; ++k) {
    cost[k] = static_cast<double>(v[k]->d.nnz) + 4.0 * v[k]->d.Npad;
    total += cost[k] * v[k]->d.B;
  }
  // team sizes: no slice above ~target; teams take at most team_share of the workgroups
  double target = std::max(1.0, total / bt->grid * target_mult);
  const int64_t team_cap = static_cast<int64_t>(team_share * bt->grid);
  std::vector<int32_t> P(count);
  for (int iter = 0; iter < 200; ++iter) {
    int64_t team_wgs = 0;
    for (int32_t k = 0; k < count; ++k) {
      const int32_t G = v[k]->d.G;
      int32_t p = std::max<int32_t>((G + kBatchMaxGroups - 1) / kBatchMaxGroups,
                                    static_cast<int32_t>(std::min(1e9, std::ceil(cost[k] / target))));
      p = std::min(p, G);
      p = std::min(p, std::max(1, kMaxCoopGroups / v[k]->d.B));  // slice flags hold 256 slices per trial
      P[k] = p;
      if (p > 1) team_wgs += static_cast<int64_t>(p) * v[k]->d.B;
    }
    if (team_wgs <= team_cap) break;
    target *= 1.25;
  }
  std::vector<SlicePlan> plans(count);
  std::vector<size_t> plan_off(count);
  std::vector<int32_t> tables;
  for (int32_t k = 0; k < count; ++k) {
    SlicePlan p = partition_groups(v[k]->layout, v[k]->d.G, P[k], kBatchMaxGroups);
    if (p.ng_max > kBatchMaxGroups) return fail(SN_ERANGE, "network %d: too many neurons for a batch", k);
    plan_off[k] = tables.size();
    tables.insert(tables.end(), p.wg_group.begin(), p.wg_group.end());
    plans[k] = std::move(p);
  }
  std::vector<int32_t> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return cost[x] > cost[y]; });
  std::vector<int4> team, queue;
  for (int32_t k : order) {
    if (plans[k].P > 1) {
      for (int32_t b = 0; b < v[k]->d.B; ++b)
        for (int32_t w = 0; w < plans[k].P; ++w) team.push_back(make_int4(k, w, b, 0));
    } else {
      for (int32_t b = 0; b < v[k]->d.B; ++b) queue.push_back(make_int4(k, b, 0, 0));
    }
  }
  if (static_cast<int64_t>(team.size()) > bt->grid) return fail(SN_ERANGE, "batch teams need more workgroups than the device holds");
  sn_net* a = v[0];
  void* plan_buf = dev_alloc(a, tables.size() * sizeof(int32_t));
  void* nets_buf = dev_alloc(a, count * sizeof(BatchNet));
  void* team_buf = dev_alloc(a, std::max<size_t>(1, team.size()) * sizeof(int4));
  void* queue_buf = dev_alloc(a, std::max<size_t>(1, queue.size()) * sizeof(int4));
  void* head_buf = dev_alloc(a, 256);
  if (!plan_buf || !nets_buf || !team_buf || !queue_buf || !head_buf) {
    for (void* p : {plan_buf, nets_buf, team_buf, queue_buf, head_buf}) dev_free(a, p);
    return fail(SN_ENOMEM, "cannot allocate batch tables");
  }
  if (hipStreamSynchronize(bt->stream) != hipSuccess ||  // queued batch launches may read the old tables
      hipMemcpyAsync(plan_buf, tables.data(), tables.size() * sizeof(int32_t), hipMemcpyHostToDevice, bt->stream) !=
          hipSuccess ||
      hipStreamSynchronize(bt->stream) != hipSuccess) {
    for (void* p : {plan_buf, nets_buf, team_buf, queue_buf, head_buf}) dev_free(a, p);
    return fail(SN_EDEVICE, "cannot upload batch tables");
  }
  batch_free(bt);
  bt->plan_buf = plan_buf;
  bt->nets_buf = nets_buf;
  bt->team_buf = team_buf;
  bt->queue_buf = queue_buf;
  bt->head_buf = head_buf;
  bt->plans = std::move(plans);
  bt->plan_off = std::move(plan_off);
  bt->team = std::move(team);
  bt->queue = std::move(queue);
  bt->target_mult = target_mult;
  bt->team_share = team_share;
  return SN_OK;
}

}  // namespace

extern "C" {

const char* sn_last_error(void) { return g_err.c_str(); }

sn_status sn_batch_create(sn_net* const* nets, int32_t count, sn_batch** out) {
  if (!nets || !out) return fail(SN_EINVAL, "nets and out must not be NULL");
  *out = nullptr;
  if (count < 1 || count > 65536) return fail(SN_ERANGE, "count %d outside [1, 65536]", count);
  std::vector<sn_net*> v(nets, nets + count);
  {
    std::vector<sn_net*> sorted(v);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) return fail(SN_EINVAL, "a network appears twice");
  }
  for (int32_t k = 0; k < count; ++k) {
    sn_net* n = v[k];
    if (!n) return fail(SN_EINVAL, "network %d is NULL", k);
    if (n->poisoned) return fail(SN_ESTATE, "network %d is poisoned", k);
    if (!n->synapses_loaded) return fail(SN_ESTATE, "network %d has no synapses", k);
    if (n->stdp_on) return fail(SN_ESTATE, "network %d has plasticity on, which a batch does not apply", k);
    if (n->device != v[0]->device) return fail(SN_EINVAL, "networks are on different devices");
    if (batch_lds_bytes(n->d, 1) > 96 * 1024) return fail(SN_ERANGE, "network %d: spike ring too large for a batch", k);
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, v[0]->device) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SN_EDEVICE, "cannot query the device");
  }
  sn_batch* bt = new (std::nothrow) sn_batch();
  if (!bt) return fail(SN_ENOMEM, "out of host memory");
  bt->nets = v;
  bt->stream = v[0]->stream;
  // workgroups resident at once, for the largest LDS any network needs
  // (its spike ring, accumulators, partial sums and group offsets)
  size_t lds = 0;
  for (sn_net* n : v) lds = std::max(lds, batch_lds_bytes(n->d, std::min<int32_t>(n->d.G, kBatchMaxGroups)));
  // the grid must fit either kernel variant (a net reloaded later may lose
  // its compact records)
  const int per_cu = std::min(batch_blocks_per_cu(lds, false), batch_blocks_per_cu(lds, true));
  if (per_cu < 1) {
    delete bt;
    return fail(SN_ERANGE, "batch kernel does not fit on a compute unit");
  }
  bt->grid = per_cu * cus;
  bt->lds = lds;
  const sn_status st = plan_batch(bt, 1.f, 0.75f);
  if (st != SN_OK) {
    batch_free(bt);
    delete bt;
    return st;
  }
  *out = bt;
  return SN_OK;
}

sn_status sn_batch_run(sn_batch* bt, int32_t n_steps) {
  if (!bt) return fail(SN_EINVAL, "batch is NULL");
  if (bt->poisoned) return fail(SN_ESTATE, "batch is poisoned by an earlier device error");
  if (n_steps < 0) return fail(SN_ERANGE, "n_steps must be >= 0");
  if (n_steps == 0) return SN_OK;
  const int32_t count = static_cast<int32_t>(bt->nets.size());
  for (sn_net* n : bt->nets) {
    sn_status st = check_usable(n);
    if (st != SN_OK) return st;
    if (n->stdp_on) return fail(SN_ESTATE, "a network of the batch has plasticity on, which a batch does not apply");
    if (!n->synapses_loaded) return fail(SN_ESTATE, "a network of the batch has no synapse list (dense rows?)");
    if (static_cast<int64_t>(n->t) + n_steps > INT32_MAX) return fail(SN_ERANGE, "step counter overflows");
  }
  auto poison = [&](hipError_t e, const char* what) {
    bt->poisoned = true;
    for (sn_net* n : bt->nets) n->poisoned = true;
    return fail(SN_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  };
  for (sn_net* n : bt->nets) {
    sn_status st = ensure_rows(n, static_cast<int64_t>(n->t) + n_steps);
    if (st != SN_OK) return st;
    if (n->stream != bt->stream) {
      const hipError_t e = hipStreamSynchronize(n->stream);
      if (e != hipSuccess) return poison(e, "hipStreamSynchronize");
    }
  }
  const int32_t* tables = static_cast<const int32_t*>(bt->plan_buf);
  bt->descs.resize(count);
  for (int32_t k = 0; k < count; ++k) {
    sn_net* n = bt->nets[k];
    const SlicePlan& p = bt->plans[k];
    SimArgs a{};
    a.n = n->d;
    a.wg_group = tables + bt->plan_off[k];
    a.mailbox = n->mailbox;
    a.status = n->status;
    a.P = p.P;
    a.ng_max = p.ng_max;
    a.max_recs = p.max_recs;
    bt->descs[k].team = a;
    bt->descs[k].single = a;
    if (p.P > 1) {
      const hipError_t e = launch_prefill_mailbox(a, n->t, bt->stream);
      if (e != hipSuccess) return poison(e, "mailbox prefill");
    }
  }
  for (int4& x : bt->team) x.w = bt->nets[x.x]->t;
  for (int4& x : bt->queue) x.z = bt->nets[x.x]->t;
  hipError_t e = hipMemcpyAsync(bt->nets_buf, bt->descs.data(), count * sizeof(BatchNet), hipMemcpyHostToDevice, bt->stream);
  if (e == hipSuccess && !bt->team.empty())
    e = hipMemcpyAsync(bt->team_buf, bt->team.data(), bt->team.size() * sizeof(int4), hipMemcpyHostToDevice, bt->stream);
  if (e == hipSuccess && !bt->queue.empty())
    e = hipMemcpyAsync(bt->queue_buf, bt->queue.data(), bt->queue.size() * sizeof(int4), hipMemcpyHostToDevice, bt->stream);
  if (e != hipSuccess) return poison(e, "batch table upload");
  e = launch_zero_i32(static_cast<int32_t*>(bt->head_buf), bt->stream);
  if (e != hipSuccess) return poison(e, "queue reset");
  BatchArgs ba{};
  ba.nets = static_cast<const BatchNet*>(bt->nets_buf);
  ba.team = static_cast<const int4*>(bt->team_buf);
  ba.queue = static_cast<const int4*>(bt->queue_buf);
  ba.n_team = static_cast<int32_t>(bt->team.size());
  ba.n_queue = static_cast<int32_t>(bt->queue.size());
  ba.queue_head = static_cast<int32_t*>(bt->head_buf);
  bool compact = true;
  for (sn_net* n : bt->nets) compact = compact && n->d.crecs != nullptr;
  e = launch_batch(ba, bt->grid, bt->lds, n_steps, compact, bt->stream);
  if (e != hipSuccess) return poison(e, "batch launch");
  for (sn_net* n : bt->nets) {
    n->t += n_steps;
    n->last_path = kPathBatch;
  }
  return SN_OK;
}

static bool bptt_desc_ok(const sn_bptt_desc* d) {
  return d && d->n_neurons >= 32 && d->n_neurons % 32 == 0 && d->n_inputs >= 0 && d->n_trials >= 1 && d->n_steps >= 1 &&
         d->checkpoint_every >= 1 && std::isfinite(d->threshold) && d->leak >= 0.f && std::isfinite(d->leak) &&
         std::isfinite(d->reset) && std::isfinite(d->slope) && d->slope > 0.f;
}

size_t sn_bptt_workspace_bytes(const sn_bptt_desc* d) { return bptt_desc_ok(d) ? bptt_workspace_bytes(*d) : 0; }

sn_status sn_bptt_forward(const sn_bptt_desc* d, const float* W_cat, const float* x, float* counts, void* workspace,
                          void* hip_stream) {
  if (!bptt_desc_ok(d)) return fail(SN_EINVAL, "invalid BPTT descriptor (N must be a positive multiple of 32)");
  if (!W_cat || !x || !counts || !workspace) return fail(SN_EINVAL, "null pointer");
  const hipError_t e = bptt_forward(*d, W_cat, x, counts, workspace, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(SN_EDEVICE, "BPTT forward: %s", hipGetErrorString(e));
  return SN_OK;
}

sn_status sn_bptt_forward_noalloc(const sn_bptt_desc* d, const float* W_cat, const float* x, float* counts,
                                  void* hip_stream) {
  if (!bptt_desc_ok(d)) return fail(SN_EINVAL, "invalid BPTT descriptor (N must be a positive multiple of 32)");
  if (!W_cat || !x || !counts) return fail(SN_EINVAL, "null pointer");
  const size_t need = bptt_workspace_bytes(*d);
  if (need > static_cast<size_t>(SN_BPTT_NOALLOC_WORKSPACE_BYTES))
    return fail(SN_ERANGE, "the forward needs %zu bytes of workspace, above the %zu of the library's buffer", need,
                static_cast<size_t>(SN_BPTT_NOALLOC_WORKSPACE_BYTES));
  const hipError_t e = bptt_forward_noalloc(*d, W_cat, x, counts, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(SN_EDEVICE, "BPTT forward (library workspace): %s", hipGetErrorString(e));
  return SN_OK;
}

sn_status sn_bptt_backward(const sn_bptt_desc* d, const float* W_cat, const float* x, const float* dcounts,
                           const void* workspace, float* dW_cat, void* hip_stream) {
  if (!bptt_desc_ok(d)) return fail(SN_EINVAL, "invalid BPTT descriptor (N must be a positive multiple of 32)");
  if (!W_cat || !x || !dcounts || !workspace || !dW_cat) return fail(SN_EINVAL, "null pointer");
  const hipError_t e = bptt_backward(*d, W_cat, x, dcounts, workspace, dW_cat, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(SN_EDEVICE, "BPTT backward: %s", hipGetErrorString(e));
  return SN_OK;
}

sn_status sn_batch_autotune(sn_batch* bt, int32_t steps, float* target_mult_out, float* team_share_out) {
  if (!bt) return fail(SN_EINVAL, "batch is NULL");
  if (bt->poisoned) return fail(SN_ESTATE, "batch is poisoned by an earlier device error");
  if (steps < 1 || steps > 4096) return fail(SN_ERANGE, "steps %d outside [1, 4096]", steps);
  for (sn_net* n : bt->nets) {
    const sn_status st = check_usable(n);
    if (st != SN_OK) return st;
  }
  struct Cand {
    float target_mult, team_share;
  };
  const Cand cands[] = {{1.f, 0.75f}, {0.5f, 0.75f}, {2.f, 0.75f}, {1.f, 0.5f}, {0.5f, 0.5f},
                        {1.f, 0.875f}, {0.5f, 0.875f}, {0.25f, 0.875f}};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    if (e0) (void)hipEventDestroy(e0);
    return fail(SN_EDEVICE, "cannot create events");
  }
  auto reset_all = [&]() -> sn_status {
    for (sn_net* n : bt->nets) {
      const sn_status st = sn_reset_state(n);
      if (st != SN_OK) return st;
      if (n->stream != bt->stream && hipStreamSynchronize(n->stream) != hipSuccess) return fail(SN_EDEVICE, "sync");
    }
    return SN_OK;
  };
  Cand best{0.f, 0.f};
  float best_ms = 0.f;
  sn_status st = SN_OK;
  for (const Cand& c : cands) {
    st = plan_batch(bt, c.target_mult, c.team_share);
    if (st == SN_ERANGE) {  // this schedule cannot run the batch
      st = SN_OK;
      continue;
    }
    if (st != SN_OK) break;
    float ms = 0.f;
    for (int rep = 0; rep < 2 && st == SN_OK; ++rep) {  // untimed run, then the timed one
      st = reset_all();
      if (st == SN_OK && hipEventRecord(e0, bt->stream) != hipSuccess) st = fail(SN_EDEVICE, "hipEventRecord");
      if (st == SN_OK) st = sn_batch_run(bt, steps);
      if (st == SN_OK && hipEventRecord(e1, bt->stream) != hipSuccess) st = fail(SN_EDEVICE, "hipEventRecord");
      if (st == SN_OK && hipEventSynchronize(e1) != hipSuccess) st = fail(SN_EDEVICE, "hipEventSynchronize");
      if (st == SN_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = fail(SN_EDEVICE, "hipEventElapsedTime");
    }
    if (st != SN_OK) break;
    for (sn_net* n : bt->nets) {
      st = check_status(n);  // a spike-exchange wait that timed out poisons the network
      if (st != SN_OK) break;
    }
    if (st != SN_OK) break;
    if (best.target_mult == 0.f || ms < best_ms) {
      best = c;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != SN_OK) {
    bt->poisoned = bt->poisoned || std::any_of(bt->nets.begin(), bt->nets.end(), [](sn_net* n) { return n->poisoned; });
    return st;
  }
  if (best.target_mult == 0.f) return fail(SN_ERANGE, "no schedule could run the batch");
  st = plan_batch(bt, best.target_mult, best.team_share);
  if (st == SN_OK) st = reset_all();
  if (st != SN_OK) return st;
  if (target_mult_out) *target_mult_out = best.target_mult;
  if (team_share_out) *team_share_out = best.team_share;
  return SN_OK;
}

void sn_batch_destroy(sn_batch* bt) {
  if (!bt) return;
  (void)hipStreamSynchronize(bt->stream);
  batch_free(bt);
  delete bt;
}

sn_status sn_create_network(const sn_net_desc* desc, const sn_allocator* alloc, void* hip_stream, sn_net** out) {
  if (!desc || !out) return fail(SN_EINVAL, "desc and out must not be NULL");
  *out = nullptr;
  const int32_t N = desc->n_neurons, B = desc->n_trials, D = desc->max_delay;
  if (N < 1 || N > SN_MAX_NEURONS) return fail(SN_ERANGE, "n_neurons %d outside [1, %d]", N, SN_MAX_NEURONS);
  if (B < 1 || B > 65535) return fail(SN_ERANGE, "n_trials %d outside [1, 65535]", B);
  if (D < 1 || D > SN_MAX_DELAY) return fail(SN_ERANGE, "max_delay %d outside [1, %d]", D, SN_MAX_DELAY);
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(SN_EINVAL, "allocator needs alloc and free");

  const int32_t G = (N + kGroup - 1) / kGroup, Npad = G * kGroup;
  std::vector<float> th(Npad, INFINITY), lk(Npad, 0.f), rs(Npad, 0.f), am(Npad, 0.f);
  std::vector<uint8_t> rf(Npad, 0);
  for (int32_t j = 0; j < N; ++j) {
    th[j] = desc->threshold ? desc->threshold[j] : desc->threshold_scalar;
    lk[j] = desc->leak ? desc->leak[j] : desc->leak_scalar;
    rs[j] = desc->reset ? desc->reset[j] : desc->reset_scalar;
    am[j] = desc->amplitude ? desc->amplitude[j] : desc->amplitude_scalar;
    rf[j] = desc->refractory ? desc->refractory[j] : desc->refractory_scalar;
    if (!std::isfinite(th[j])) return fail(SN_EINVAL, "threshold of neuron %d is not finite", j);
    if (!std::isfinite(rs[j])) return fail(SN_EINVAL, "reset of neuron %d is not finite", j);
    if (!std::isfinite(am[j])) return fail(SN_EINVAL, "amplitude of neuron %d is not finite", j);
    if (!(lk[j] >= 0.f)) return fail(SN_EINVAL, "leak of neuron %d must be >= 0 (got %g)", j, lk[j]);
  }

  sn_net* n = new (std::nothrow) sn_net();
  if (!n) return fail(SN_ENOMEM, "out of host memory");
  if (hipGetDevice(&n->device) != hipSuccess) {
    delete n;
    (void)hipGetLastError();
    return fail(SN_EDEVICE, "no HIP device available");
  }
  n->stream = static_cast<hipStream_t>(hip_stream);
  if (alloc) {
    n->alloc = *alloc;
    n->custom_alloc = true;
  }
  n->d.N = N;
  n->d.Npad = Npad;
  n->d.G = G;
  n->d.B = B;
  n->d.D = D;
  n->d.phases = 1;
  n->h_reset = rs;

  auto upload = [&](const void* src, size_t bytes) -> void* {
    void* p = dev_alloc(n, bytes);
    if (!p) return nullptr;
    n->owned.push_back(p);
    if (hipMemcpyAsync(p, src, bytes, hipMemcpyHostToDevice, n->stream) != hipSuccess) return nullptr;
    return p;
  };
  n->d.theta = static_cast<const float*>(upload(th.data(), Npad * sizeof(float)));
  n->d.leak = static_cast<const float*>(upload(lk.data(), Npad * sizeof(float)));
  n->d.reset = static_cast<const float*>(upload(rs.data(), Npad * sizeof(float)));
  n->d.amp = static_cast<const float*>(upload(am.data(), Npad * sizeof(float)));
  n->d.refr = static_cast<const uint8_t*>(upload(rf.data(), Npad));
  void* V = dev_alloc(n, static_cast<size_t>(B) * Npad * sizeof(float));
  if (V) n->owned.push_back(V);
  void* R = dev_alloc(n, static_cast<size_t>(B) * Npad);
  if (R) n->owned.push_back(R);
  n->d.V = static_cast<float*>(V);
  n->d.ref = static_cast<uint8_t*>(R);
  const size_t mail_bytes = static_cast<size_t>(D + 1) * B * 2 * G * sizeof(uint64_t);
  const size_t flag_bytes = static_cast<size_t>(std::min(B, kMaxCoopGroups)) * kMaxCoopGroups * 64 * sizeof(uint32_t);
  void* F = dev_alloc(n, mail_bytes + flag_bytes + 256);
  if (F) n->owned.push_back(F);
  n->mailbox = static_cast<uint64_t*>(F);
  n->slice_flags = F ? reinterpret_cast<uint32_t*>(static_cast<char*>(F) + mail_bytes) : nullptr;
  n->status = F ? reinterpret_cast<uint32_t*>(static_cast<char*>(F) + mail_bytes + flag_bytes) : nullptr;
  if (F && hipMemsetAsync(F, 0, mail_bytes + flag_bytes + 256, n->stream) != hipSuccess) F = nullptr;
  if (!n->d.theta || !n->d.leak || !n->d.reset || !n->d.amp || !n->d.refr || !V || !R || !F) {
    sn_destroy_network(n);
    return fail(SN_ENOMEM, "cannot allocate or upload neuron arrays");
  }
  if (launch_reset_state(n->d, n->stream) != hipSuccess) {
    sn_destroy_network(n);
    return fail(SN_EDEVICE, "state initialisation failed");
  }
  sn_status st = ensure_rows(n, 64);
  if (st != SN_OK) {
    sn_destroy_network(n);
    return st;
  }
  if (hipStreamSynchronize(n->stream) != hipSuccess) {
    sn_destroy_network(n);
    return fail(SN_EDEVICE, "stream synchronisation failed");
  }
  *out = n;
  return SN_OK;
}

sn_status sn_load_weights_delays(sn_net* n, int64_t nnz, const int32_t* pre, const int32_t* post, const float* w,
                                 const uint8_t* delay) {
  sn_status st = check_usable(n);
  if (st != SN_OK) return st;
  if (nnz < 0) return fail(SN_EINVAL, "nnz must be >= 0");
  if (nnz > 0 && (!pre || !post || !w || !delay)) return fail(SN_EINVAL, "synapse arrays must not be NULL");
  if (nnz >= (int64_t(1) << 31)) return fail(SN_ERANGE, "at most 2^31 - 1 synapses");
  for (int64_t k = 0; k < nnz; ++k) {
    if (pre[k] < 0 || pre[k] >= n->d.N) return fail(SN_ERANGE, "synapse %lld: pre %d outside [0, %d)", (long long)k, pre[k], n->d.N);
    if (post[k] < 0 || post[k] >= n->d.N) return fail(SN_ERANGE, "synapse %lld: post %d outside [0, %d)", (long long)k, post[k], n->d.N);
    if (delay[k] < 1 || delay[k] > n->d.D) return fail(SN_ERANGE, "synapse %lld: delay %d outside [1, %d]", (long long)k, delay[k], n->d.D);
    if (!std::isfinite(w[k])) return fail(SN_EINVAL, "synapse %lld: weight is not finite", (long long)k);
  }
  if (!on_device_ok(n)) return fail(SN_ESTATE, "the network belongs to device %d", n->device);
  // nets too wide for the per-group kernel's LDS history get their delay >= 2
  // records ordered by delay phase for the wide kernel (wide.hip)
  int32_t phase_rows = 0;
  bool staged_all = false;  // every delay's history row staged in LDS by the wide kernel
  int32_t lane_block = 1;   // steps per block of the wide kernel's lane layout
  if (wide_net(n->d)) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, n->device) != hipSuccess) {
      (void)hipGetLastError();
      return fail(SN_EDEVICE, "cannot query the device");
    }
    const WidePlan wp = wide_plan(n->d, cus);
    if (wp.P > 1) phase_rows = wp.Dl;
    // lane records address the staged rows of a block of steps
    staged_all = (wp.P > 1 || (wp.Dl >= n->d.D && wp.Dl > 0)) && wp.block >= 2;
    lane_block = wp.block;
  }
  HostLayout L = build_layout(n->d.N, nnz, pre, post, w, delay, n->d.D, phase_rows);
  if (L.too_large)
    return fail(SN_ERANGE, "%lld synapses need more than 2^31 - 1 records with the layout's fillers",
                static_cast<long long>(nnz));
  HostPush H = build_push_layout(n->d.N, n->d.Npad, nnz, pre, post, w, delay);
  float cscale = 0.f;
  std::vector<uint32_t> C = compact_records(L, n->d.N, n->d.D, &cscale);
  if (!C.empty()) C.resize(C.size() + static_cast<size_t>(kCompactChunkRows) * kGroup, 0u);  // slack of one chunk
  // wide nets with every delay staged: a lane-only copy of the layout as
  // 4-byte lane records, kept when it is at most 80% of the 8-byte records'
  // bytes
  std::vector<uint32_t> LR;
  std::vector<int32_t> lgp, lws, lss;
  float lscale = 0.f;
  if (staged_all && nnz > 0) {
    HostLayout LL = build_layout(n->d.N, nnz, pre, post, w, delay, n->d.D, phase_rows, true, lane_block);
    if (!LL.too_large && LL.phases == L.phases && 4.0 * LL.recs.size() <= 0.8 * 8.0 * L.recs.size()) {
      LR = lane_records(LL, n->d.G, &lscale);
      if (!LR.empty()) {
        // slack of one batch of fillers (k = 0, a word of the row of delay 1)
        const uint32_t row1 = static_cast<uint32_t>(lane_block - 1) * 2u * static_cast<uint32_t>(n->d.G) *
                              sizeof(uint32_t);
        LR.resize(LR.size() + static_cast<size_t>(kLaneBatchRows) * kGroup, lane_record(0, row1, 0u));
        lgp = std::move(LL.gptr);
        lws = std::move(LL.wsec);
        lss = std::move(LL.ssec);
      }
    }
  }
  SlicePlan one = partition_groups(L, n->d.G, 1, n->d.G);
  if (!fit_plan(n->d, one)) one.P = 0;
  SlicePlan many = plan_persist(n->d, L, n->slices_req);
  // every new buffer is allocated before an old one is freed, so ENOMEM
  // leaves the network as it was
  void* recs = dev_alloc(n, L.recs.size() * sizeof(Rec));
  void* gptr = dev_alloc(n, L.gptr.size() * sizeof(int32_t));
  void* gsplit = dev_alloc(n, L.gsplit.size() * sizeof(int32_t));
  void* orecs = dev_alloc(n, H.orecs.size() * sizeof(Rec));
  void* optr = dev_alloc(n, H.optr.size() * sizeof(int32_t));
  void* wsec = L.phases > 1 ? dev_alloc(n, L.wsec.size() * sizeof(int32_t)) : nullptr;
  void* crecs = C.empty() ? nullptr : dev_alloc(n, C.size() * sizeof(uint32_t));
  void* lrecs = LR.empty() ? nullptr : dev_alloc(n, LR.size() * sizeof(uint32_t));
  // lane offsets: [G + 1] group starts, [G][block - 1] starts of the short
  // delays' sections, then (256-byte aligned) the [block - 1][B][Npad] input
  // sums that the first kernel of a block of steps leaves for the later ones
  const size_t held_at = ((lgp.size() + lss.size()) * sizeof(int32_t) + 255) / 256 * 256;
  const size_t lmeta_bytes =
      held_at + static_cast<size_t>(lane_block - 1) * n->d.B * n->d.Npad * sizeof(float);
  void* lgptr = LR.empty() ? nullptr : dev_alloc(n, lmeta_bytes);
  void* lwsec = LR.empty() || L.phases <= 1 ? nullptr : dev_alloc(n, lws.size() * sizeof(int32_t));
  bool bad = !recs || !gptr || !gsplit || !orecs || !optr || (L.phases > 1 && !wsec) || (!C.empty() && !crecs) ||
             (!LR.empty() && (!lrecs || !lgptr || (L.phases > 1 && !lwsec)));
  void* wg_one = alloc_plan(n, one, bad);
  void* wg_many = alloc_plan(n, many, bad);
  if (bad) {
    for (void* p : {recs, gptr, gsplit, orecs, optr, wsec, crecs, lrecs, lgptr, lwsec, wg_one, wg_many}) dev_free(n, p);
    return fail(SN_ENOMEM, "cannot allocate synapse records");
  }
  // the previous buffers may be in use by queued work
  SN_HIP(n, hipStreamSynchronize(n->stream));
  drop_graph(n);
  for (void** p : {&n->recs, &n->gptr, &n->gsplit, &n->orecs, &n->optr, &n->wsec, &n->crecs, &n->lrecs, &n->lgptr,
                   &n->lwsec}) {
    dev_free(n, *p);
    *p = nullptr;
  }
  n->lrecs = lrecs;
  n->lgptr = lgptr;
  n->lwsec = lwsec;
  n->d.lrecs = static_cast<const uint32_t*>(lrecs);
  n->d.lgptr = static_cast<const int32_t*>(lgptr);
  n->d.lwsec = static_cast<const int32_t*>(lwsec);
  n->d.lsec = lgptr ? static_cast<const int32_t*>(lgptr) + lgp.size() : nullptr;
  n->d.held = lgptr ? reinterpret_cast<float*>(static_cast<char*>(lgptr) + held_at) : nullptr;
  n->d.lblock = lgptr ? lane_block : 0;
  n->d.lscale = lscale;
  n->recs = recs;
  n->gptr = gptr;
  n->gsplit = gsplit;
  n->orecs = orecs;
  n->optr = optr;
  n->wsec = wsec;
  n->crecs = crecs;
  n->d.crecs = static_cast<const uint32_t*>(crecs);
  n->d.cscale = cscale;
  n->d.recs = static_cast<const Rec*>(recs);
  n->d.gptr = static_cast<const int32_t*>(gptr);
  n->d.gsplit = static_cast<const int32_t*>(gsplit);
  n->d.wsec = static_cast<const int32_t*>(wsec);
  n->d.phases = L.phases;
  n->d.phase_rows = L.phase_rows;
  n->d.nnz = nnz;
  // from here on a failure is a device error, which poisons the network
  if (!L.recs.empty())
    SN_HIP(n, hipMemcpyAsync(recs, L.recs.data(), L.recs.size() * sizeof(Rec), hipMemcpyHostToDevice, n->stream));
  SN_HIP(n, hipMemcpyAsync(gptr, L.gptr.data(), L.gptr.size() * sizeof(int32_t), hipMemcpyHostToDevice, n->stream));
  SN_HIP(n, hipMemcpyAsync(gsplit, L.gsplit.data(), L.gsplit.size() * sizeof(int32_t), hipMemcpyHostToDevice, n->stream));
  if (!H.orecs.empty())
    SN_HIP(n, hipMemcpyAsync(orecs, H.orecs.data(), H.orecs.size() * sizeof(Rec), hipMemcpyHostToDevice, n->stream));
  SN_HIP(n, hipMemcpyAsync(optr, H.optr.data(), H.optr.size() * sizeof(int32_t), hipMemcpyHostToDevice, n->stream));
  if (wsec)
    SN_HIP(n, hipMemcpyAsync(wsec, L.wsec.data(), L.wsec.size() * sizeof(int32_t), hipMemcpyHostToDevice, n->stream));
  if (crecs)
    SN_HIP(n, hipMemcpyAsync(crecs, C.data(), C.size() * sizeof(uint32_t), hipMemcpyHostToDevice, n->stream));
  if (lrecs) {
    SN_HIP(n, hipMemcpyAsync(lrecs, LR.data(), LR.size() * sizeof(uint32_t), hipMemcpyHostToDevice, n->stream));
    SN_HIP(n, hipMemcpyAsync(lgptr, lgp.data(), lgp.size() * sizeof(int32_t), hipMemcpyHostToDevice, n->stream));
    SN_HIP(n, hipMemcpyAsync(static_cast<int32_t*>(lgptr) + lgp.size(), lss.data(), lss.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, n->stream));
    if (lwsec)
      SN_HIP(n, hipMemcpyAsync(lwsec, lws.data(), lws.size() * sizeof(int32_t), hipMemcpyHostToDevice, n->stream));
  }
  SN_HIP(n, hipStreamSynchronize(n->stream));  // host vectors die at return
  st = install_plan(n, n->small, one, wg_one);
  if (st != SN_OK) return st;
  st = install_plan(n, n->persist, many, wg_many);
  if (st != SN_OK) return st;
  n->synapses_loaded = true;
  dev_free(n, n->rows8);
  n->rows8 = nullptr;
  n->rows_loaded = false;
  n->rows_e = -1;
  if (n->path == SN_PATH_DENSE_ROWS) n->path = SN_PATH_AUTO;  // chosen for the rows, which are gone
  dev_free(n, n->wt);
  n->wt = nullptr;
  dev_free(n, n->wt8);
  n->wt8 = nullptr;
  n->dense_loaded = false;
  n->layout = std::move(L);
  n->push_stale = false;
  n->nnz_loaded = nnz;
  n->stdp.recs = static_cast<Rec*>(n->recs);
  stdp_chunks(n->layout.max_group_records, n->stdp.chunk, n->stdp.chunks);
  return SN_OK;
}

sn_status sn_set_slices(sn_net* n, int32_t slices) {
  sn_status st = check_usable(n);
  if (st != SN_OK) return st;
  if (slices < 0 || slices > kMaxCoopGroups) return fail(SN_ERANGE, "slices %d outside [0, %d]", slices, kMaxCoopGroups);
  n->slices_req = slices;
  if (n->synapses_loaded) return upload_plan(n, n->persist, plan_persist(n->d, n->layout, slices));
  return SN_OK;
}

sn_status sn_load_dense_weights(sn_net* n, const float* W, int32_t delay) {
  sn_status st = check_usable(n);
  if (st != SN_OK) return st;
  if (!W) return fail(SN_EINVAL, "W must not be NULL");
  if (delay != 1) return fail(SN_ERANGE, "dense weights support delay 1 only (got %d)", delay);
  if (delay > n->d.D) return fail(SN_ERANGE, "delay %d exceeds max_delay %d", delay, n->d.D);
  const int32_t N = n->d.N;
  const int32_t kpad = (n->d.Npad + 127) / 128 * 128;
  if (dense_lds_bytes(kpad) > lds_limit()) return fail(SN_ERANGE, "dense path supports up to 16,384 neurons");
  std::vector<int32_t> pre, post;
  std::vector<float> w;
  for (int32_t i = 0; i < N; ++i) {
    for (int32_t j = 0; j < N; ++j) {
      const float x = W[static_cast<size_t>(i) * N + j];
      if (!std::isfinite(x)) return fail(SN_EINVAL, "W[%d][%d] is not finite", i, j);
      uint32_t u;
      std::memcpy(&u, &x, 4);
      if ((u & 0xFFFFu) != 0u) return fail(SN_EINEXACT, "W[%d][%d] = %g is not exact in bfloat16", i, j, x);
      if (x != 0.f) {
        pre.push_back(i);
        post.push_back(j);
        w.push_back(x);
      }
    }
  }
  std::vector<uint8_t> d(w.size(), 1);
  st = sn_load_weights_delays(n, static_cast<int64_t>(w.size()), pre.data(), post.data(), w.data(), d.data());
  if (st != SN_OK) return st;
  std::vector<uint16_t> tiled(dense_tiled_elems(n->d.Npad, kpad));
  tile_dense_weights(W, N, n->d.Npad, kpad, tiled.data());
  void* wt = dev_alloc(n, tiled.size() * sizeof(uint16_t));
  if (!wt) return fail(SN_ENOMEM, "cannot allocate dense weights");
  n->wt = wt;
  n->kpad = kpad;
  SN_HIP(n, hipMemcpyAsync(wt, tiled.data(), tiled.size() * sizeof(uint16_t), hipMemcpyHostToDevice, n->stream));
  dev_free(n, n->wt8);
  n->wt8 = nullptr;
  const int32_t e8 = int8_exponent(W, static_cast<int64_t>(N) * N);
  if (e8 >= 0) {
    std::vector<int8_t> t8(dense_tiled_elems(n->d.Npad, kpad));
    tile_dense_weights_i8(W, N, n->d.Npad, kpad, e8, t8.data());
    void* w8 = dev_alloc(n, t8.size());
    if (!w8) return fail(SN_ENOMEM, "cannot allocate dense weights");
    SN_HIP(n, hipMemcpyAsync(w8, t8.data(), t8.size(), hipMemcpyHostToDevice, n->stream));
    SN_HIP(n, hipStreamSynchronize(n->stream));  // t8 dies at the end of this block
    n->wt8 = w8;
    n->scale8 = std::ldexp(1.f, -e8);
  }
  SN_HIP(n, hipStreamSynchronize(n->stream));
  SN_HIP(n, prepare_dense_kernel(kpad));
  n->dense_loaded = true;
  n->stdp_on = false;
  return SN_OK;
}

sn_status sn_load_dense_rows_i8(sn_net* n, int32_t row0, int32_t n_rows, const int8_t* k, int32_t e) {
  sn_status st = check_usable(n);
  if (st != SN_OK) return st;
  const int32_t N = n->d.N;
  if (N > kRowsMaxNeurons) return fail(SN_ERANGE, "dense rows support up to %d neurons (got %d)", kRowsMaxNeurons, N);
  if (e < 0 || e > 24) return fail(SN_ERANGE, "exponent %d outside [0, 24]", e);
  if (row0 < 0 || n_rows < 0 || static_cast<int64_t>(row0) + n_rows > N)
    return fail(SN_ERANGE, "rows %d .. %lld outside [0, %d)", row0, static_cast<long long>(row0) + n_rows - 1, N);
  if (n_rows > 0 && !k) return fail(SN_EINVAL, "k must not be NULL");
  if (n->rows_loaded && e != n->rows_e)
    return fail(SN_EINVAL, "exponent %d differs from the %d of the rows already loaded", e, n->rows_e);
  if (!on_device_ok(n)) return fail(SN_ESTATE, "the network belongs to device %d", n->device);
  const size_t pitch = static_cast<size_t>(n->d.Npad);
  if (!n->rows_loaded) {
    // queued work may still read the buffers dropped here
    SN_HIP(n, hipStreamSynchronize(n->stream));
    drop_graph(n);
    void* r = dev_alloc(n, static_cast<size_t>(N) * pitch);
    if (!r) return fail(SN_ENOMEM, "cannot allocate %zu bytes of dense rows", static_cast<size_t>(N) * pitch);
    for (void** p : {&n->rows8, &n->wt, &n->wt8, &n->recs, &n->gptr, &n->gsplit, &n->orecs, &n->optr, &n->wsec,
                     &n->crecs, &n->lrecs, &n->lgptr, &n->lwsec}) {
      dev_free(n, *p);
      *p = nullptr;
    }
    n->d.crecs = nullptr;
    n->d.lrecs = nullptr;
    n->d.lgptr = nullptr;
    n->d.lwsec = nullptr;
    n->d.lsec = nullptr;
    n->d.held = nullptr;
    n->d.lblock = 0;
    n->d.recs = nullptr;
    n->d.gptr = nullptr;
    n->d.gsplit = nullptr;
    n->d.wsec = nullptr;
    n->d.phases = 1;
    n->d.phase_rows = 0;
    n->d.nnz = 0;
    n->small.ok = n->persist.ok = false;
    n->synapses_loaded = n->dense_loaded = false;
    n->stdp_on = false;
    n->layout = HostLayout{};
    n->nnz_loaded = 0;
    n->rows8 = r;
    n->rows_e = e;
    n->rows_loaded = true;
    n->path = SN_PATH_AUTO;  // a path chosen for the dropped weights does not apply
    SN_HIP(n, hipMemsetAsync(r, 0, static_cast<size_t>(N) * pitch, n->stream));
  }
  if (n_rows > 0) {
    SN_HIP(n, hipMemcpy2DAsync(static_cast<int8_t*>(n->rows8) + static_cast<size_t>(row0) * pitch, pitch, k,
                               static_cast<size_t>(N), static_cast<size_t>(N), static_cast<size_t>(n_rows),
                               hipMemcpyHostToDevice, n->stream));
  }
  SN_HIP(n, hipStreamSynchronize(n->stream));  // the caller may reuse k on return
  return SN_OK;
}

sn_status sn_set_input_spikes(sn_net* n, int32_t t0, int32_t n_steps, const uint32_t* bits) {
  sn_status st = check_usable(n);
  if (st != SN_OK) return st;
  if (t0 < 0 || n_steps < 0) return fail(SN_ERANGE, "t0 and n_steps must be >= 0");
  if (n_steps > 0 && !bits) return fail(SN_EINVAL, "bits must not be NULL");
  if (n_steps == 0) return SN_OK;
  if (static_cast<int64_t>(t0) + n_steps > INT32_MAX) return fail(SN_ERANGE, "step range overflows");
  st = ensure_rows(n, static_cast<int64_t>(t0) + n_steps);
  if (st != SN_OK) return st;
  const int32_t B = n->d.B, G = n->d.G, N = n->d.N, W32 = (N + 31) / 32;
  std::vector<uint64_t> rows(static_cast<size_t>(n_steps) * B * G);
  for (int32_t b = 0; b < B; ++b) {
    for (int32_t i = 0; i < n_steps; ++i) {
      const uint32_t* src = bits + (static_cast<size_t>(b) * n_steps + i) * W32;
      uint64_t* dst = rows.data() + (static_cast<size_t>(i) * B + b) * G;
      for (int32_t g = 0; g < G; ++g) {
        const uint32_t lo = src[2 * g];
        const uint32_t hi = (2 * g + 1 < W32) ? src[2 * g + 1] : 0u;
        uint64_t v = (static_cast<uint64_t>(hi) << 32) | lo;
        const int valid = N - g * kGroup;
        if (valid < 64) v &= (1ull << valid) - 1ull;
        dst[g] = v;
      }
    }
  }
  const size_t row_bytes = static_cast<size_t>(B) * G * sizeof(uint64_t);
  SN_HIP(n, hipMemcpyAsync(const_cast<uint64_t*>(n->d.ext) + static_cast<size_t>(t0) * B * G, rows.data(),
                           rows.size() * sizeof(uint64_t), hipMemcpyHostToDevice, n->stream));
  (void)row_bytes;
  SN_HIP(n, hipStreamSynchronize(n->stream));
  return SN_OK;
}

sn_status sn_set_input_spikes_device(sn_net* n, int32_t t0, int32_t n_steps, const uint32_t* bits) {
  sn_status st = check_usable(n);
  if (st != SN_OK) return st;
  if (t0 < 0 || n_steps < 0) return fail(SN_ERANGE, "t0 and n_steps must be >= 0");
  if (n_steps > 0 && !bits) return fail(SN_EINVAL, "bits must not be NULL");
  if (n_steps == 0) return SN_OK;
  if (static_cast<int64_t>(t0) + n_steps > INT32_MAX) return fail(SN_ERANGE, "step range overflows");
  st = ensure_rows(n, static_cast<int64_t>(t0) + n_steps);
  if (st != SN_OK) return st;
  SN_HIP(n, launch_repack_input(n->d, t0, n_steps, bits, n->stream));
  return SN_OK;
}

sn_status sn_set_path(sn_net* n, int32_t path) {
  sn_status st = check_usable(n);
  if (st != SN_OK) return st;
  if ((path < SN_PATH_AUTO || path > SN_PATH_DENSE_STEP) && path != SN_PATH_DENSE_ROWS)
    return fail(SN_ERANGE, "unknown path %d", path);
  n->path = path;
  return SN_OK;
}

sn_status sn_get_progress(sn_net* n, int32_t* t, int32_t* path) {
  if (!n) return fail(SN_EINVAL, "network is NULL");
  if (t) *t = n->t;
  if (path) *path = n->last_path;
  return SN_OK;
}

sn_status sn_run(sn_net* n, int32_t n_steps) {
  sn_status st = check_usable(n);
  if (st != SN_OK) return st;
  if (!n->synapses_loaded && !n->rows_loaded) return fail(SN_ESTATE, "load synapses before sn_run");
  if (n_steps < 0) return fail(SN_ERANGE, "n_steps must be >= 0");
  if (static_cast<int64_t>(n->t) + n_steps > INT32_MAX) return fail(SN_ERANGE, "step counter overflows");
  if (n_steps == 0) return SN_OK;
  if (!on_device_ok(n)) return fail(SN_ESTATE, "the network belongs to device %d", n->device);
  st = ensure_rows(n, static_cast<int64_t>(n->t) + n_steps);
  if (st != SN_OK) return st;

  int32_t path = n->path;
  if (n->stdp_on) {  // plasticity runs with the per-step kernels
    if (path != SN_PATH_AUTO && path != SN_PATH_STEP)
      return fail(SN_ESTATE, "with plasticity on, only the per-step path runs (set SN_PATH_AUTO or SN_PATH_STEP)");
    path = SN_PATH_STEP;
  }
  if (path == SN_PATH_PUSH && n->push_stale)
    return fail(SN_ESTATE, "plasticity changed the weights: reload them before the event-driven path");
  if (n->rows_loaded != (path == SN_PATH_DENSE_ROWS) && !(n->rows_loaded && path == SN_PATH_AUTO))
    return fail(SN_ESTATE, n->rows_loaded ? "dense rows run only on SN_PATH_DENSE_ROWS"
                                          : "SN_PATH_DENSE_ROWS needs sn_load_dense_rows_i8");
  if (path == SN_PATH_AUTO) {
    // one workgroup when its records and spike ring fit in LDS, otherwise one
    // launch per step
    if (n->rows_loaded) path = SN_PATH_DENSE_ROWS;
    else if (n->dense_loaded) path = SN_PATH_DENSE;
    else if (n->small.ok && n->small.host.recs_lds && n->small.host.ring_lds) path = SN_PATH_SMALL;
    else if (n->persist.ok && n->persist.host.P > 1 && n->persist.host.recs_lds && n->persist.host.ring_lds)
      path = SN_PATH_PERSIST;
    else path = SN_PATH_STEP;
  }
  switch (path) {
    case SN_PATH_SMALL:
      if (!n->small.ok) return fail(SN_ERANGE, "network too large for the single-workgroup path");
      SN_HIP(n, launch_sim(sim_args(n, n->small), n->small.host.recs_lds, n->small.host.ring_lds, n->t, n_steps,
                           n->stream));
      break;
    case SN_PATH_PERSIST: {
      if (!n->persist.ok) return fail(SN_ERANGE, "no slice plan fits the persistent kernel");
      SN_HIP(n, launch_sim(sim_args(n, n->persist), n->persist.host.recs_lds, n->persist.host.ring_lds, n->t,
                           n_steps, n->stream));
      break;
    }
    case SN_PATH_STEP:
      SN_HIP(n, prepare_step_kernel(n->d));
      if (n->stdp_on) {  // history words of the steps before this run, from the raster
        StdpArgs a = n->stdp;
        a.n = n->d;
        SN_HIP(n, launch_hist_build(a, n->t, n->stream));
      }
      st = run_per_step(n, SN_PATH_STEP, n->t, n_steps);
      if (st != SN_OK) return st;
      if (n->stdp_on) n->push_stale = true;
      break;
    case SN_PATH_PUSH:
      st = run_push(n, n->t, n_steps);
      if (st != SN_OK) return st;
      break;
    case SN_PATH_DENSE_ROWS:
      st = run_per_step(n, SN_PATH_DENSE_ROWS, n->t, n_steps);
      if (st != SN_OK) return st;
      break;
    case SN_PATH_DENSE:
    case SN_PATH_DENSE_STEP: {
      if (!n->dense_loaded) return fail(SN_ESTATE, "the dense path needs sn_load_dense_weights");
      const int64_t wgs = static_cast<int64_t>(n->d.Npad / 16) * ((n->d.B + 63) / 64);
      if (path == SN_PATH_DENSE && wgs <= kMaxCoopGroups && dense_persist_lds_bytes(n->kpad) <= lds_limit()) {
        DenseArgs a{n->d, static_cast<const uint16_t*>(n->wt), n->kpad, static_cast<const int8_t*>(n->wt8), n->scale8};
        SN_HIP(n, launch_dense_persist(a, n->slice_flags, n->status, n->t, n_steps, n->stream));
        n->t += n_steps;
        n->last_path = n->wt8 ? kPathDensePersistI8 : kPathDensePersist;
        return SN_OK;
      }
      st = run_per_step(n, SN_PATH_DENSE, n->t, n_steps);
      if (st != SN_OK) return st;
      break;
    }
    default:
      return fail(SN_ERANGE, "path %d is not available in this build", path);
  }
  n->t += n_steps;
  n->last_path = path;
  return SN_OK;
}

sn_status sn_synchronize(sn_net* n) {
  sn_status st = check_usable(n);
  if (st != SN_OK) return st;
  SN_HIP(n, hipStreamSynchronize(n->stream));
  return check_status(n);
}

sn_status sn_read_raster(sn_net* n, int32_t t0, int32_t n_steps, uint32_t* out) {
  sn_status st = check_usable(n);
  if (st != SN_OK) return st;
  if (n_steps > 0 && !out) return fail(SN_EINVAL, "out must not be NULL");
  if (t0 < 0 || n_steps < 0 || static_cast<int64_t>(t0) + n_steps > n->t)
    return fail(SN_ERANGE, "steps [%d, %lld) not simulated (t = %d)", t0, (long long)t0 + n_steps, n->t);
  if (n_steps == 0) return SN_OK;
  const int32_t B = n->d.B, G = n->d.G, N = n->d.N, W32 = (N + 31) / 32;
  std::vector<uint64_t> rows(static_cast<size_t>(n_steps) * B * G);
  SN_HIP(n, hipMemcpyAsync(rows.data(), n->d.raster + static_cast<size_t>(t0) * B * G, rows.size() * sizeof(uint64_t),
                           hipMemcpyDeviceToHost, n->stream));
  SN_HIP(n, hipStreamSynchronize(n->stream));
  st = check_status(n);
  if (st != SN_OK) return st;
  for (int32_t b = 0; b < B; ++b) {
    for (int32_t i = 0; i < n_steps; ++i) {
      const uint64_t* src = rows.data() + (static_cast<size_t>(i) * B + b) * G;
      uint32_t* dst = out + (static_cast<size_t>(b) * n_steps + i) * W32;
      for (int32_t g = 0; g < G; ++g) {
        dst[2 * g] = static_cast<uint32_t>(src[g]);
        if (2 * g + 1 < W32) dst[2 * g + 1] = static_cast<uint32_t>(src[g] >> 32);
      }
    }
  }
  return SN_OK;
}

sn_status sn_read_state(sn_net* n, float* V, uint8_t* refractory_left) {
  sn_status st = check_usable(n);
  if (st != SN_OK) return st;
  const int32_t B = n->d.B, N = n->d.N, Npad = n->d.Npad;
  std::vector<float> hv(static_cast<size_t>(B) * Npad);
  std::vector<uint8_t> hr(static_cast<size_t>(B) * Npad);
  SN_HIP(n, hipMemcpyAsync(hv.data(), n->d.V, hv.size() * sizeof(float), hipMemcpyDeviceToHost, n->stream));
  SN_HIP(n, hipMemcpyAsync(hr.data(), n->d.ref, hr.size(), hipMemcpyDeviceToHost, n->stream));
  SN_HIP(n, hipStreamSynchronize(n->stream));
  st = check_status(n);
  if (st != SN_OK) return st;
  for (int32_t b = 0; b < B; ++b) {
    if (V) std::memcpy(V + static_cast<size_t>(b) * N, hv.data() + static_cast<size_t>(b) * Npad, N * sizeof(float));
    if (refractory_left)
      std::memcpy(refractory_left + static_cast<size_t>(b) * N, hr.data() + static_cast<size_t>(b) * Npad, N);
  }
  return SN_OK;
}

sn_status sn_read_raster_device(sn_net* n, int32_t t0, int32_t n_steps, uint32_t* out) {
  sn_status st = check_usable(n);
  if (st != SN_OK) return st;
  if (n_steps > 0 && !out) return fail(SN_EINVAL, "out must not be NULL");
  if (t0 < 0 || n_steps < 0 || static_cast<int64_t>(t0) + n_steps > n->t)
    return fail(SN_ERANGE, "steps [%d, %lld) not simulated (t = %d)", t0, (long long)t0 + n_steps, n->t);
  if (n_steps == 0) return SN_OK;
  if (!on_device_ok(n)) return fail(SN_ESTATE, "the network belongs to device %d", n->device);
  SN_HIP(n, launch_unpack_raster(n->d, t0, n_steps, out, n->stream));
  return SN_OK;
}

sn_status sn_read_state_device(sn_net* n, float* V, uint8_t* refractory_left) {
  sn_status st = check_usable(n);
  if (st != SN_OK) return st;
  if (!on_device_ok(n)) return fail(SN_ESTATE, "the network belongs to device %d", n->device);
  const size_t B = n->d.B, N = n->d.N, Npad = n->d.Npad;
  // rows of Npad on the device, rows of N in the caller's buffers
  if (V)
    SN_HIP(n, hipMemcpy2DAsync(V, N * sizeof(float), n->d.V, Npad * sizeof(float), N * sizeof(float), B,
                               hipMemcpyDeviceToDevice, n->stream));
  if (refractory_left)
    SN_HIP(n, hipMemcpy2DAsync(refractory_left, N, n->d.ref, Npad, N, B, hipMemcpyDeviceToDevice, n->stream));
  return SN_OK;
}

// Plasticity changes the weights of the 8-byte records in place; the 4-byte
// copies (compact records of the persistent and batch kernels, lane records
// of the wide kernel) keep the loaded ones.  Turning plasticity on drops them,
// so every path reads the 8-byte records from then on (reloading the synapses
// builds them again).
static sn_status drop_weight_copies(sn_net* n) {
  if (!n->crecs && !n->lrecs) return SN_OK;
  SN_HIP(n, hipStreamSynchronize(n->stream));  // queued work may still read them
  drop_graph(n);
  for (void** p : {&n->crecs, &n->lrecs, &n->lgptr, &n->lwsec}) {
    dev_free(n, *p);
    *p = nullptr;
  }
  n->d.crecs = nullptr;
  n->d.lrecs = nullptr;
  n->d.lgptr = nullptr;
  n->d.lwsec = nullptr;
  n->d.lsec = nullptr;
  n->d.held = nullptr;
  n->d.lblock = 0;
  return SN_OK;
}

sn_status sn_set_stdp(sn_net* n, const sn_stdp_desc* desc) {
  sn_status st = check_usable(n);
  if (st != SN_OK) return st;
  if (!desc) {
    n->stdp_on = false;
    return SN_OK;
  }
  if (n->rows_loaded) return fail(SN_ESTATE, "plasticity applies to synapse lists, not dense rows");
  if (!n->synapses_loaded) return fail(SN_ESTATE, "load synapses before sn_set_stdp");
  if (n->dense_loaded) return fail(SN_ESTATE, "plasticity applies to synapse lists, not dense weights");
  if (n->d.B != 1) return fail(SN_ERANGE, "plasticity needs one trial (got %d)", n->d.B);
  if (desc->window < 1 || desc->window > 16) return fail(SN_ERANGE, "window %d outside [1, 16]", desc->window);
  if (!std::isfinite(desc->w_min) || !std::isfinite(desc->w_max) || !(desc->w_min <= desc->w_max))
    return fail(SN_EINVAL, "need finite w_min <= w_max");
  for (int k = 0; k < desc->window; ++k)
    if (!std::isfinite(desc->ltp[k]) || !std::isfinite(desc->ltd[k])) return fail(SN_EINVAL, "table entry %d is not finite", k);
  StdpArgs a{};
  a.n = n->d;
  a.recs = static_cast<Rec*>(n->recs);
  a.window = desc->window;
  for (int k = 0; k < 16; ++k) {
    a.ltp[k] = k < desc->window ? desc->ltp[k] : 0.f;
    a.ltd[k] = k < desc->window ? desc->ltd[k] : 0.f;
  }
  a.w_min = desc->w_min == 0.f ? 0.f : desc->w_min;  // -0 would read as a filler mark
  a.w_max = desc->w_max == 0.f ? 0.f : desc->w_max;
  if (!n->stdp_hist) {
    n->stdp_hist = static_cast<uint64_t*>(dev_alloc(n, 2 * static_cast<size_t>(n->d.Npad) * sizeof(uint64_t)));
    if (!n->stdp_hist) return fail(SN_ENOMEM, "cannot allocate the spike-history words");
  }
  a.hist = n->stdp_hist;
  st = drop_weight_copies(n);
  if (st != SN_OK) return st;
  stdp_chunks(n->layout.max_group_records, a.chunk, a.chunks);
  SN_HIP(n, prepare_stdp_kernel());
  n->stdp = a;
  n->stdp_on = true;
  ++n->stdp_gen;
  return SN_OK;
}

sn_status sn_read_weights(sn_net* n, float* w) {
  sn_status st = check_usable(n);
  if (st != SN_OK) return st;
  if (n->rows_loaded) return fail(SN_ESTATE, "weights loaded as dense rows are not read back");
  if (!n->synapses_loaded) return fail(SN_ESTATE, "no synapses loaded");
  if (n->nnz_loaded > 0 && !w) return fail(SN_EINVAL, "w must not be NULL");
  std::vector<Rec> recs(n->layout.recs.size());
  if (!recs.empty())
    SN_HIP(n, hipMemcpyAsync(recs.data(), n->recs, recs.size() * sizeof(Rec), hipMemcpyDeviceToHost, n->stream));
  SN_HIP(n, hipStreamSynchronize(n->stream));
  for (size_t k = 0; k < recs.size(); ++k)
    if (n->layout.src[k] >= 0) w[n->layout.src[k]] = recs[k].w;
  return SN_OK;
}

sn_status sn_autotune(sn_net* n, int32_t steps, int32_t* path_out, int32_t* slices_out) {
  sn_status st = check_usable(n);
  if (st != SN_OK) return st;
  if (!n->synapses_loaded && !n->rows_loaded) return fail(SN_ESTATE, "load synapses before sn_autotune");
  if (steps < 1 || steps > 4096) return fail(SN_ERANGE, "steps %d outside [1, 4096]", steps);
  if (n->stdp_on) return fail(SN_ESTATE, "plasticity would change the weights while timing: turn it off first");
  if (!on_device_ok(n)) return fail(SN_ESTATE, "the network belongs to device %d", n->device);
  struct Cand {
    int32_t path, slices;
  };
  std::vector<Cand> cands;
  if (n->rows_loaded) {
    cands = {{SN_PATH_DENSE_ROWS, 0}};
  } else if (n->dense_loaded) {
    cands = {{SN_PATH_DENSE, 0}, {SN_PATH_DENSE_STEP, 0}};
  } else {
    if (n->small.ok) cands.push_back({SN_PATH_SMALL, 0});
    const int32_t top = std::min(n->d.G, std::max(1, kMaxCoopGroups / n->d.B));
    const int32_t least = std::max(2, (n->d.G + 127) / 128);
    int32_t last = -1;
    for (int32_t div : {1, 2, 4, 8}) {
      const int32_t s = top / div;
      if (s < least || s == last) continue;
      last = s;
      SlicePlan p = plan_persist(n->d, n->layout, s);
      if (p.P > 1) cands.push_back({SN_PATH_PERSIST, div == 1 ? 0 : s});
    }
    cands.push_back({SN_PATH_STEP, 0});
    cands.push_back({SN_PATH_PUSH, 0});
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  SN_HIP(n, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return device_error(n, hipErrorOutOfMemory, "hipEventCreate");
  }
  Cand best{SN_PATH_AUTO, 0};
  float best_ms = 0.f;
  for (const Cand& c : cands) {
    n->path = c.path;
    if (n->synapses_loaded && (c.path == SN_PATH_PERSIST || n->slices_req != c.slices)) {
      n->slices_req = c.slices;
      st = upload_plan(n, n->persist, plan_persist(n->d, n->layout, c.slices));
      if (st != SN_OK) break;
    }
    float ms = 0.f;
    for (int rep = 0; rep < 2 && st == SN_OK; ++rep) {  // untimed run, then the timed one
      st = sn_reset_state(n);
      if (st == SN_OK && hipEventRecord(e0, n->stream) != hipSuccess) st = device_error(n, hipErrorUnknown, "hipEventRecord");
      if (st == SN_OK) st = sn_run(n, steps);
      if (st == SN_OK && hipEventRecord(e1, n->stream) != hipSuccess) st = device_error(n, hipErrorUnknown, "hipEventRecord");
      if (st == SN_OK) st = sn_synchronize(n);
      if (st == SN_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = device_error(n, hipErrorUnknown, "hipEventElapsedTime");
    }
    if (st != SN_OK) {
      if (n->poisoned) break;
      st = SN_OK;  // this strategy cannot run the network (e.g. a size limit): skip it
      continue;
    }
    if (best.path == SN_PATH_AUTO || ms < best_ms) {
      best = c;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != SN_OK) return st;
  if (best.path == SN_PATH_AUTO) return fail(SN_ERANGE, "no strategy could run the network");
  n->path = best.path;
  if (n->synapses_loaded && n->slices_req != best.slices) {
    n->slices_req = best.slices;
    st = upload_plan(n, n->persist, plan_persist(n->d, n->layout, best.slices));
    if (st != SN_OK) return st;
  }
  st = sn_reset_state(n);
  if (st != SN_OK) return st;
  if (path_out) *path_out = best.path;
  if (slices_out) *slices_out = best.slices;
  return SN_OK;
}

sn_status sn_reset_state(sn_net* n) {
  sn_status st = check_usable(n);
  if (st != SN_OK) return st;
  SN_HIP(n, launch_reset_state(n->d, n->stream));
  n->t = 0;
  return SN_OK;
}

void sn_destroy_network(sn_net* n) {
  if (!n) return;
  (void)hipStreamSynchronize(n->stream);
  for (void* p : n->owned) dev_free(n, p);
  dev_free(n, n->d.raster);
  dev_free(n, const_cast<uint64_t*>(n->d.ext));
  dev_free(n, n->recs);
  dev_free(n, n->gptr);
  dev_free(n, n->gsplit);
  dev_free(n, n->wsec);
  dev_free(n, n->crecs);
  dev_free(n, n->lrecs);
  dev_free(n, n->lgptr);
  dev_free(n, n->lwsec);
  dev_free(n, n->small.wg);
  dev_free(n, n->persist.wg);
  dev_free(n, n->wt);
  dev_free(n, n->wt8);
  dev_free(n, n->rows8);
  dev_free(n, n->stdp_hist);
  dev_free(n, n->orecs);
  dev_free(n, n->optr);
  dev_free(n, n->push_wg);
  dev_free(n, n->accum);
  if (n->graph) (void)hipGraphExecDestroy(n->graph);
  if (n->capture_stream) (void)hipStreamDestroy(n->capture_stream);
  delete n;
}

}  // extern "C"
