// Host runtime behind include/sta.h: input validation, device levelization
// driver, level-sorted device layout, update sequencing and reports.
//
// Inputs follow the paper's flattened interface (§III "Heterogeneous netlist
// database", "Parasitics (RC) inputs"); outputs may go to host or device memory
// (§III "Report options").  Validation is pure host code and runs before the
// first HIP call, so malformed inputs are rejected without a device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "sta.h"
#include "sta_est.h"
#include "sta_internal.h"

using namespace sta;

namespace {

thread_local std::string g_err;

sta_status fail(sta_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

sta_status hip_fail(hipError_t e, const char *what) {
  return fail(e == hipErrorOutOfMemory ? STA_E_OOM : STA_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);   \
  } while (0)

#define STA_TRY(expr)              \
  do {                             \
    sta_status s_ = (expr);        \
    if (s_ != STA_OK) return s_;   \
  } while (0)

// Owned device allocation.
struct DevMem {
  void *p = nullptr;
  DevMem() = default;
  DevMem(const DevMem &) = delete;
  DevMem &operator=(const DevMem &) = delete;
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
};

// Host view of one input array: the caller's host memory or a host copy of
// caller device memory.
template <class T>
struct HostArr {
  const T *p = nullptr;
  std::vector<T> own;
  sta_status load(const T *src, size_t n, sta_mem mem, const char *name) {
    if (n == 0) {
      p = nullptr;
      return STA_OK;
    }
    if (!src) return fail(STA_E_ARG, "%s is NULL", name);
    if (mem == STA_HOST) {
      p = src;
      return STA_OK;
    }
    own.resize(n);
    hipError_t e = hipMemcpy(own.data(), src, n * sizeof(T), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, name);
    p = own.data();
    return STA_OK;
  }
  const T &operator[](size_t i) const { return p[i]; }
};

bool finite(float v) { return std::isfinite(v); }

}  // namespace

struct sta_ctx {
  int device = 0;
  sta_options opt{};
  int n_pins = 0, n_cells = 0, n_nets = 0, n_pi = 0, n_po = 0, n_sinks = 0, n_drv = 0, n_ep = 0;
  int n_cell_levels = 0, n_levels = 0, n_chunks = 0, n_big = 0, n_rc_chunks = 0, n_rc_adj_chunks = 0;
  int64_t n_nodes = 0;
  int n_cu = 0, sweep_grid = 1;
  bool coop = false;                   // persistent sweeps use the cooperative level-major kernels
  int coop_max = 0;                    // cooperative grid limit (blocks)
  std::vector<std::unique_ptr<DevMem>> mem;
  DevDesign D{};
  float *rc_cap = nullptr;
  const float *rc_pc = nullptr;        // the small nets' lumped pin caps (added in set_wire_caps)
  int64_t n_small_nodes = 0;           // RC nodes of the small nets (the first in RC order)
  int32_t *pin_loc = nullptr, *net_slot = nullptr, *sink_slot = nullptr, *node_src = nullptr;
  int32_t *ep_pin = nullptr, *pin_level = nullptr, *level_order = nullptr;
  int32_t *slot_drv_pin = nullptr, *slot_sink_pin = nullptr;  // slot -> caller pin (path reports)
  int max_in = 1;                      // most inputs of any library type
  int2 *rc_chunks = nullptr;
  int2 *rc_adj_chunks = nullptr;       // the RC adjoint's smaller chunks over the same net order
  BigNet *big = nullptr;
  int32_t *big_end = nullptr, *big_nsp = nullptr, *big_nsl = nullptr, *big_egp = nullptr, *big_egl = nullptr;
  WideNets wide{};
  hipStream_t side = nullptr;          // wide-net RC kernels run here, overlapping the small nets
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipStream_t side2 = nullptr;         // RC groups beside the forward sweep; WNS/TNS and the
  hipEvent_t ev_fwd = nullptr, ev_red = nullptr;  // endpoint order beside the backward sweep
  // RC pass in groups of levels: group g serves levels [rc_grp_lvl[g],
  // rc_grp_lvl[g+1]) and ends at RC chunk rc_grp_end[g]; wide nets are first
  // needed at level wide_lvl
  std::vector<int32_t> rc_grp_lvl, rc_grp_end;
  std::vector<hipEvent_t> ev_rc;
  int wide_lvl = INT32_MAX;
  float *big_pc = nullptr;
  double *big_scratch = nullptr;
  int32_t *arc_src = nullptr;
  int n_fanin = 0;
  bool updated = false;
  double *partials = nullptr, *out = nullptr;
  int32_t *vals = nullptr, *order = nullptr;
  void *sort_temp = nullptr;
  size_t sort_bytes = 0;
  std::vector<int4> ph_fwd, ph_bwd, ph_adj;  // sweep phases (kind, first item, count, level)
  std::vector<int4> lvl_reg;           // per level: first slot, end of the slots in regular chunks,
                                       // float4 granules of the largest type span of a block
  int n_pieces = 0;
  hipEvent_t ev[10]{};  // 0..6 update phases, 7..9 adjoint phases
  hipStream_t cap_stream = nullptr;   // graph schedule: capture stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int graph_overlap = -1;             // sta_options.overlap the graph was captured with
  bool flow_ok = false;               // the dataflow schedule is available
  FlowArgs flow_fwd{}, flow_bwd{};
  uint32_t *flow_err = nullptr;
  uint32_t flow_epoch = 0;
  int flow_grid = 0;
  bool bwd_timed = false;
  bool events = false, timed = false;
  hipStream_t last_stream = nullptr;
  std::vector<int32_t> h_ep_pin;       // endpoint pins (host copy)
  // batched contexts: concatenation offsets and per-design reduction buffers
  int n_designs = 1;
  bool batched = false;
  std::vector<int32_t> pin_off, ep_off;
  std::vector<int64_t> node_off;
  int32_t *d_ep_off = nullptr;
  double *b_partials = nullptr, *b_out = nullptr;
  uint64_t *keys64 = nullptr, *keys64_out = nullptr;  // [2 n_ep] endpoint sort keys
  int key_bits = 33, design_bits = 0;
  // incremental update: maps from the layout; device queues made on first use
  int32_t *inc_chunk_of = nullptr;     // [n_drv]
  int2 *inc_chunk_ph = nullptr;        // [n_chunks]
  int32_t *inc_slot_rc = nullptr;      // [n_drv] RC chunk of the slot's net, or -1 - wide-net index
  bool inc_ready = false;
  IncArgs inc{};
  uint32_t *inc_buf = nullptr;         // flags, queue lengths, recomputed-net bytes (cleared per update)
  int inc_words = 0, inc_grid = 0, inc_max_items = 0;
  int32_t *inc_stop = nullptr;         // pinned readback of the queued sweeps' stop phases
  int32_t *inc_nets = nullptr;         // device copy of the caller's net list
  int32_t *inc_host = nullptr;         // pinned staging of the list
  int inc_cap = 0;                     // capacity of both (ids)
  hipEvent_t inc_ev = nullptr;         // staging reusable once this has passed
  std::unique_ptr<DevMem> path_ws;     // path report workspace (grows, kept between reports)
  size_t path_ws_bytes = 0;

  template <class T>
  sta_status alloc(T **out_p, size_t n) {
    auto m = std::make_unique<DevMem>();
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(&m->p, n * sizeof(T));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    *out_p = static_cast<T *>(m->p);
    mem.push_back(std::move(m));
    return STA_OK;
  }
  template <class T>
  sta_status upload(T **out_p, const std::vector<T> &h) {
    STA_TRY(alloc(out_p, h.size()));
    if (!h.empty()) HIP_TRY(hipMemcpy(*out_p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return STA_OK;
  }
  ~sta_ctx() {
    if (events)
      for (auto &e : ev) (void)hipEventDestroy(e);
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_fwd) (void)hipEventDestroy(ev_fwd);
    if (ev_red) (void)hipEventDestroy(ev_red);
    for (auto &e : ev_rc) (void)hipEventDestroy(e);
    if (inc_ev) (void)hipEventDestroy(inc_ev);
    if (inc_host) (void)hipHostFree(inc_host);
    if (inc_stop) (void)hipHostFree(inc_stop);
  }
};

// The two side streams of every context on a device: made once, by the
// first context created on it, and kept until the process ends.  Streams made
// later in a process that has run a cooperative launch ran the overlapped
// per-level sequence (RC groups and the reduction beside the sweeps) at more
// than twice its in-order time, while contexts created before that launch kept
// their speed; sharing the first pair keeps every context on those.  Contexts
// used at once from several caller streams stay correct (every use is ordered
// by the context's own events) but share the pair's hardware queues.
// Two events released with their owner (an event may be destroyed while waits
// on it are still queued).
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

static hipError_t device_side_streams(int device, hipStream_t *a, hipStream_t *b);

// The estimator's tiers with the small nets beside the large nets' block
// kernel: on the current device's first side stream, forked from s and joined
// back into it (the block kernel's longest net holds a few compute units for
// most of the pass while the rest of the chip would idle).
template <class Launch>
static sta_status est_forked(hipStream_t s, Launch &&launch) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipStream_t side = nullptr, side2 = nullptr;
  HIP_TRY(device_side_streams(dev, &side, &side2));
  EventPair ev;
  HIP_TRY(hipEventCreateWithFlags(&ev.a, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&ev.b, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(ev.a, s));
  HIP_TRY(hipStreamWaitEvent(side, ev.a, 0));
  HIP_TRY(launch(side));
  HIP_TRY(hipEventRecord(ev.b, side));
  HIP_TRY(hipStreamWaitEvent(s, ev.b, 0));
  return STA_OK;
}

static hipError_t device_side_streams(int device, hipStream_t *a, hipStream_t *b) {
  static std::mutex mu;
  static std::vector<std::pair<hipStream_t, hipStream_t>> pool;
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0) return hipErrorInvalidDevice;
  if ((size_t)device >= pool.size()) pool.resize((size_t)device + 1, {nullptr, nullptr});
  auto &p = pool[(size_t)device];
  if (!p.first) {
    hipError_t e = hipStreamCreateWithFlags(&p.first, hipStreamNonBlocking);
    if (e != hipSuccess) {
      p.first = nullptr;
      return e;
    }
    e = hipStreamCreateWithFlags(&p.second, hipStreamNonBlocking);
    if (e != hipSuccess) {
      (void)hipStreamDestroy(p.first);
      p = {nullptr, nullptr};
      return e;
    }
  }
  *a = p.first;
  *b = p.second;
  return hipSuccess;
}

extern "C" {

void sta_options_default(sta_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->mode = 0;
  o->gamma_ps = 5.0f;
  o->dangling_policy = 0;
  o->sched = STA_SCHED_PER_LEVEL;
  o->big_net_nodes = 0;
  o->sort_endpoints = 1;
  o->profile = 0;
  o->device = -1;
  o->sweep_blocks = 0;
  o->delay_model = 0;
  o->overlap = 1;
}

const char *sta_status_string(sta_status s) {
  switch (s) {
    case STA_OK: return "STA_OK";
    case STA_E_ARG: return "STA_E_ARG";
    case STA_E_CYCLE: return "STA_E_CYCLE";
    case STA_E_OOM: return "STA_E_OOM";
    case STA_E_DEVICE: return "STA_E_DEVICE";
    case STA_E_STATE: return "STA_E_STATE";
    case STA_E_UNSUPPORTED: return "STA_E_UNSUPPORTED";
  }
  return "STA_E_UNKNOWN";
}

const char *sta_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

// All host-side input arrays of sta_create.
struct Inputs {
  const sta_graph_desc *g;
  const sta_rc_desc *rc;
  const sta_lib_desc *lib;
  const sta_constraints *cons;
  HostArr<int32_t> pin_kind, cell_type, cell_in_ptr, cell_in_pin, cell_out_pin;
  HostArr<int32_t> net_driver, net_sink_ptr, net_sink_pin;
  HostArr<int64_t> net_node_ptr;
  HostArr<int32_t> parent, sink_node;
  HostArr<float> res, cap;
  // derived pin maps
  std::vector<int32_t> cell_of_pin, net_of_drv, sink_idx_of_pin, drv_of_sink_pin, rank;
  // batches: design pin offsets and each design's dangling-endpoint RAT [4]
  const std::vector<int32_t> *pin_off = nullptr;
  const std::vector<float> *dang = nullptr;
  // batches with a library per design: each design's PO pin cap
  const std::vector<float> *po_caps = nullptr;
  // receiving pin cap of a PO pin p
  float po_cap(int p) const {
    if (!po_caps) return lib->po_cap_ff;
    const int d = (int)(std::upper_bound(pin_off->begin(), pin_off->end(), p) - pin_off->begin()) - 1;
    return (*po_caps)[(size_t)d];
  }
};

sta_status load_graph(Inputs &I) {
  const sta_graph_desc &g = *I.g;
  if (g.n_pins < 1 || g.n_cells < 0 || g.n_nets < 1 || g.n_pi < 1 || g.n_po < 0)
    return fail(STA_E_ARG, "bad graph sizes (pins %d cells %d nets %d pi %d po %d)", g.n_pins, g.n_cells,
                g.n_nets, g.n_pi, g.n_po);
  if (g.mem != STA_HOST && g.mem != STA_DEVICE) return fail(STA_E_ARG, "graph.mem invalid");
  STA_TRY(I.pin_kind.load(g.pin_kind, g.n_pins, g.mem, "pin_kind"));
  STA_TRY(I.cell_in_ptr.load(g.cell_in_ptr, (size_t)g.n_cells + 1, g.mem, "cell_in_ptr"));
  STA_TRY(I.net_sink_ptr.load(g.net_sink_ptr, (size_t)g.n_nets + 1, g.mem, "net_sink_ptr"));
  if (I.cell_in_ptr[0] != 0 || I.net_sink_ptr[0] != 0) return fail(STA_E_ARG, "CSR offsets must start at 0");
  const int32_t n_cin = I.cell_in_ptr[g.n_cells], n_sink = I.net_sink_ptr[g.n_nets];
  if (n_cin < 0 || n_sink < 0) return fail(STA_E_ARG, "negative CSR size");
  STA_TRY(I.cell_type.load(g.cell_type, g.n_cells, g.mem, "cell_type"));
  STA_TRY(I.cell_in_pin.load(g.cell_in_pin, n_cin, g.mem, "cell_in_pin"));
  STA_TRY(I.cell_out_pin.load(g.cell_out_pin, g.n_cells, g.mem, "cell_out_pin"));
  STA_TRY(I.net_driver.load(g.net_driver, g.n_nets, g.mem, "net_driver"));
  STA_TRY(I.net_sink_pin.load(g.net_sink_pin, n_sink, g.mem, "net_sink_pin"));
  return STA_OK;
}

sta_status validate_graph(Inputs &I) {
  const sta_graph_desc &g = *I.g;
  const sta_lib_desc &lib = *I.lib;
  const int NP = g.n_pins;
  int cnt[4] = {0, 0, 0, 0};
  I.rank.assign(NP, -1);
  for (int p = 0; p < NP; ++p) {
    const int k = I.pin_kind[p];
    if (k < 0 || k > 3) return fail(STA_E_ARG, "pin %d has kind %d", p, k);
    if (k == STA_PIN_PI || k == STA_PIN_PO) I.rank[p] = cnt[k];
    cnt[k]++;
  }
  if (cnt[STA_PIN_PI] != g.n_pi || cnt[STA_PIN_PO] != g.n_po || cnt[STA_PIN_CELL_OUT] != g.n_cells)
    return fail(STA_E_ARG, "pin kind counts (PI %d, PO %d, cell out %d) disagree with n_pi/n_po/n_cells",
                cnt[0], cnt[3], cnt[2]);
  if (g.n_nets != g.n_pi + g.n_cells)
    return fail(STA_E_ARG, "every PI and cell output drives one net: n_nets must be %d", g.n_pi + g.n_cells);
  if (I.cell_in_ptr[g.n_cells] != cnt[STA_PIN_CELL_IN])
    return fail(STA_E_ARG, "cell_in_ptr covers %d pins, design has %d cell inputs", I.cell_in_ptr[g.n_cells],
                cnt[1]);
  if (I.net_sink_ptr[g.n_nets] != cnt[STA_PIN_CELL_IN] + cnt[STA_PIN_PO])
    return fail(STA_E_ARG, "net_sink_ptr covers %d sinks, design has %d", I.net_sink_ptr[g.n_nets],
                cnt[1] + cnt[3]);
  I.cell_of_pin.assign(NP, -1);
  for (int c = 0; c < g.n_cells; ++c) {
    const int a = I.cell_in_ptr[c], b = I.cell_in_ptr[c + 1];
    if (b <= a) return fail(STA_E_ARG, "cell %d has no inputs or decreasing cell_in_ptr", c);
    const int t = I.cell_type[c];
    if (t < 0 || t >= lib.n_types) return fail(STA_E_ARG, "cell %d has type %d", c, t);
    if (lib.n_inputs[t] != b - a)
      return fail(STA_E_ARG, "cell %d has %d inputs, its type %d has %d", c, b - a, t, lib.n_inputs[t]);
    for (int k = a; k < b; ++k) {
      const int p = I.cell_in_pin[k];
      if (p < 0 || p >= NP || I.pin_kind[p] != STA_PIN_CELL_IN)
        return fail(STA_E_ARG, "cell %d input %d is pin %d, not a cell input pin", c, k - a, p);
      if (I.cell_of_pin[p] >= 0) return fail(STA_E_ARG, "pin %d is an input of two cells", p);
      I.cell_of_pin[p] = c;
    }
    const int o = I.cell_out_pin[c];
    if (o < 0 || o >= NP || I.pin_kind[o] != STA_PIN_CELL_OUT)
      return fail(STA_E_ARG, "cell %d output is pin %d, not a cell output pin", c, o);
    if (I.cell_of_pin[o] >= 0) return fail(STA_E_ARG, "pin %d is the output of two cells", o);
    I.cell_of_pin[o] = c;
  }
  I.net_of_drv.assign(NP, -1);
  I.sink_idx_of_pin.assign(NP, -1);
  I.drv_of_sink_pin.assign(NP, -1);
  for (int n = 0; n < g.n_nets; ++n) {
    const int d = I.net_driver[n];
    if (d < 0 || d >= NP || (I.pin_kind[d] != STA_PIN_PI && I.pin_kind[d] != STA_PIN_CELL_OUT))
      return fail(STA_E_ARG, "net %d driver %d is not a PI or cell output", n, d);
    if (I.net_of_drv[d] >= 0) return fail(STA_E_ARG, "pin %d drives two nets", d);
    I.net_of_drv[d] = n;
    const int a = I.net_sink_ptr[n], b = I.net_sink_ptr[n + 1];
    if (b < a) return fail(STA_E_ARG, "net_sink_ptr decreases at net %d", n);
    for (int s = a; s < b; ++s) {
      const int p = I.net_sink_pin[s];
      if (p < 0 || p >= NP || (I.pin_kind[p] != STA_PIN_CELL_IN && I.pin_kind[p] != STA_PIN_PO))
        return fail(STA_E_ARG, "net %d sink %d is pin %d, not a cell input or PO", n, s - a, p);
      if (I.sink_idx_of_pin[p] >= 0) return fail(STA_E_ARG, "pin %d is a sink of two nets", p);
      I.sink_idx_of_pin[p] = s;
      I.drv_of_sink_pin[p] = d;
    }
  }
  return STA_OK;
}

sta_status load_validate_rc(Inputs &I) {
  const sta_rc_desc &rc = *I.rc;
  const sta_graph_desc &g = *I.g;
  if (rc.mem != STA_HOST && rc.mem != STA_DEVICE) return fail(STA_E_ARG, "rc.mem invalid");
  if (rc.n_nodes < g.n_nets || rc.n_nodes >= (int64_t)INT32_MAX)
    return fail(STA_E_ARG, "rc.n_nodes %lld out of range", (long long)rc.n_nodes);
  const size_t NN = (size_t)rc.n_nodes;
  STA_TRY(I.net_node_ptr.load(rc.net_node_ptr, (size_t)g.n_nets + 1, rc.mem, "net_node_ptr"));
  STA_TRY(I.parent.load(rc.parent, NN, rc.mem, "parent"));
  STA_TRY(I.res.load(rc.res_kohm, NN, rc.mem, "res_kohm"));
  STA_TRY(I.cap.load(rc.cap_ff, NN, rc.mem, "cap_ff"));
  STA_TRY(I.sink_node.load(rc.sink_node, (size_t)I.net_sink_ptr[g.n_nets], rc.mem, "sink_node"));
  if (I.net_node_ptr[0] != 0 || I.net_node_ptr[g.n_nets] != rc.n_nodes)
    return fail(STA_E_ARG, "net_node_ptr must run from 0 to n_nodes");
  for (int n = 0; n < g.n_nets; ++n) {
    const int64_t a = I.net_node_ptr[n], b = I.net_node_ptr[n + 1];
    if (b <= a) return fail(STA_E_ARG, "net %d has no RC node (root required)", n);
    if (I.parent[a] != -1) return fail(STA_E_ARG, "net %d: root parent must be -1", n);
    for (int64_t k = a + 1; k < b; ++k) {
      const int64_t pk = I.parent[k];
      if (pk < 0 || pk >= k - a) return fail(STA_E_ARG, "net %d node %lld: parent %lld not < child", n,
                                            (long long)(k - a), (long long)pk);
    }
    for (int s = I.net_sink_ptr[n]; s < I.net_sink_ptr[n + 1]; ++s) {
      const int64_t k = I.sink_node[s];
      if (k < 0 || k >= b - a) return fail(STA_E_ARG, "sink %d: node %lld outside its net", s, (long long)k);
    }
  }
  for (size_t k = 0; k < NN; ++k) {
    if (!finite(I.res[k]) || I.res[k] < 0.0f) return fail(STA_E_ARG, "res_kohm[%zu] invalid", k);
    if (!finite(I.cap[k]) || I.cap[k] < 0.0f) return fail(STA_E_ARG, "cap_ff[%zu] invalid", k);
  }
  return STA_OK;
}

sta_status validate_lib(const sta_lib_desc &L) {
  if (L.n_types < 1 || L.n_types > kMaxTypes) return fail(STA_E_UNSUPPORTED, "n_types %d not in [1, %d]", L.n_types, kMaxTypes);
  if (L.nx < 2 || L.ny < 2 || L.nx > kMaxAxis || L.ny > kMaxAxis)
    return fail(STA_E_UNSUPPORTED, "table size %dx%d not in [2,8]x[2,8]", L.nx, L.ny);
  if (!L.n_inputs || !L.sense || !L.pin_cap_ff || !L.slew_axis || !L.load_axis || !L.tables)
    return fail(STA_E_ARG, "library array is NULL");
  if (!finite(L.po_cap_ff) || L.po_cap_ff < 0.0f) return fail(STA_E_ARG, "po_cap_ff invalid");
  for (int t = 0; t < L.n_types; ++t) {
    if (L.n_inputs[t] < 1) return fail(STA_E_ARG, "type %d has %d inputs", t, L.n_inputs[t]);
    if (L.sense[t] < 0 || L.sense[t] > 2) return fail(STA_E_ARG, "type %d sense %d", t, L.sense[t]);
    if (!finite(L.pin_cap_ff[t]) || L.pin_cap_ff[t] < 0.0f) return fail(STA_E_ARG, "type %d pin cap", t);
    for (int i = 0; i < L.nx; ++i) {
      const float v = L.slew_axis[t * L.nx + i];
      if (!finite(v) || (i > 0 && !(v > L.slew_axis[t * L.nx + i - 1])))
        return fail(STA_E_ARG, "type %d slew axis not strictly increasing", t);
    }
    for (int j = 0; j < L.ny; ++j) {
      const float v = L.load_axis[t * L.ny + j];
      if (!finite(v) || (j > 0 && !(v > L.load_axis[t * L.ny + j - 1])))
        return fail(STA_E_ARG, "type %d load axis not strictly increasing", t);
    }
    for (int k = 0; k < 4 * L.nx * L.ny; ++k)
      if (!finite(L.tables[(size_t)t * 4 * L.nx * L.ny + k])) return fail(STA_E_ARG, "type %d table value", t);
  }
  return STA_OK;
}

sta_status validate_cons(const sta_constraints &C, const sta_graph_desc &g) {
  if (!C.pi_at || !C.pi_slew || (g.n_po > 0 && !C.po_rat)) return fail(STA_E_ARG, "constraint array is NULL");
  for (int i = 0; i < g.n_pi * 4; ++i) {
    if (!finite(C.pi_at[i])) return fail(STA_E_ARG, "pi_at[%d] not finite", i);
    if (!finite(C.pi_slew[i]) || C.pi_slew[i] < 0.0f) return fail(STA_E_ARG, "pi_slew[%d] invalid", i);
  }
  for (int i = 0; i < g.n_po * 4; ++i)
    if (!finite(C.po_rat[i])) return fail(STA_E_ARG, "po_rat[%d] not finite", i);
  for (int v = 0; v < 4; ++v)
    if (!finite(C.dangling_rat[v])) return fail(STA_E_ARG, "dangling_rat not finite");
  return STA_OK;
}

// DFS preorder of one tree (children visited in increasing index); returns
// new_of_old.
std::vector<int32_t> preorder(const int32_t *par, int m) {
  std::vector<int32_t> cnt(m + 1, 0), kids(m > 0 ? m - 1 : 0), pos(m + 1, 0);
  for (int k = 1; k < m; ++k) cnt[par[k] + 1]++;
  for (int k = 0; k < m; ++k) cnt[k + 1] += cnt[k];
  for (int k = 0; k < m; ++k) pos[k] = cnt[k];
  for (int k = 1; k < m; ++k) kids[pos[par[k]]++] = k;
  std::vector<int32_t> newof(m), stack;
  stack.reserve(m);
  stack.push_back(0);
  int next = 0;
  while (!stack.empty()) {
    const int u = stack.back();
    stack.pop_back();
    newof[u] = next++;
    for (int i = cnt[u + 1] - 1; i >= cnt[u]; --i) stack.push_back(kids[i]);
  }
  return newof;
}

}  // namespace

// Levelize on the device; fills cell_level (host) and the context's pin levels
// and level order.
static sta_status levelize(sta_ctx *C, const Inputs &I, std::vector<int32_t> &cell_level) {
  const sta_graph_desc &g = *I.g;
  const int NP = g.n_pins, NC = g.n_cells;
  std::vector<int32_t> cell_nin(NC), cell_of_in(NP, -1), pis;
  for (int c = 0; c < NC; ++c) cell_nin[c] = I.cell_in_ptr[c + 1] - I.cell_in_ptr[c];
  for (int p = 0; p < NP; ++p) {
    if (I.pin_kind[p] == STA_PIN_CELL_IN) cell_of_in[p] = I.cell_of_pin[p];
    if (I.pin_kind[p] == STA_PIN_PI) pis.push_back(p);
  }
  std::vector<int32_t> h_kind(I.pin_kind.p, I.pin_kind.p + NP);
  std::vector<int32_t> h_nsp(I.net_sink_ptr.p, I.net_sink_ptr.p + g.n_nets + 1);
  std::vector<int32_t> h_nsn(I.net_sink_pin.p, I.net_sink_pin.p + h_nsp.back());
  std::vector<int32_t> h_cout(I.cell_out_pin.p, I.cell_out_pin.p + NC);
  sta_ctx tmp;  // scratch allocations released on return
  int32_t *d_kind, *d_net_of_drv, *d_nsp, *d_nsn, *d_cell_of_in, *d_cout, *d_nin, *d_cell_of_pin, *d_drv_of_sink;
  int32_t *d_pending, *d_cell_level, *d_fa, *d_fb, *d_keys, *d_keys_out, *d_vals;
  uint32_t *d_cnt;
  STA_TRY(tmp.upload(&d_kind, h_kind));
  STA_TRY(tmp.upload(&d_net_of_drv, I.net_of_drv));
  STA_TRY(tmp.upload(&d_nsp, h_nsp));
  STA_TRY(tmp.upload(&d_nsn, h_nsn));
  STA_TRY(tmp.upload(&d_cell_of_in, cell_of_in));
  STA_TRY(tmp.upload(&d_cout, h_cout));
  STA_TRY(tmp.upload(&d_nin, cell_nin));
  STA_TRY(tmp.upload(&d_cell_of_pin, I.cell_of_pin));
  STA_TRY(tmp.upload(&d_drv_of_sink, I.drv_of_sink_pin));
  STA_TRY(tmp.alloc(&d_pending, NC));
  STA_TRY(tmp.alloc(&d_cell_level, NC));
  STA_TRY(tmp.alloc(&d_fa, std::max(NP, 1)));
  STA_TRY(tmp.alloc(&d_fb, std::max(NP, 1)));
  STA_TRY(tmp.alloc(&d_cnt, 1));
  HIP_TRY(hipMemcpy(d_fa, pis.data(), pis.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(launch_level_init(d_pending, d_cell_level, d_nin, NC, nullptr));
  int n_front = (int)pis.size(), lvl = 0;
  while (n_front > 0) {
    HIP_TRY(hipMemset(d_cnt, 0, sizeof(uint32_t)));
    HIP_TRY(launch_level_step(d_fa, n_front, lvl, d_net_of_drv, d_nsp, d_nsn, d_cell_of_in, d_cout, d_pending,
                              d_cell_level, d_fb, d_cnt, nullptr));
    uint32_t nn = 0;
    HIP_TRY(hipMemcpy(&nn, d_cnt, sizeof nn, hipMemcpyDeviceToHost));
    std::swap(d_fa, d_fb);
    n_front = (int)nn;
    ++lvl;
  }
  cell_level.resize(NC);
  if (NC > 0)
    HIP_TRY(hipMemcpy(cell_level.data(), d_cell_level, NC * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int c = 0; c < NC; ++c)
    if (cell_level[c] < 0) return fail(STA_E_CYCLE, "combinational cycle through cell %d", c);
  // pin levels and the (level, pin id) order, on the device
  STA_TRY(C->alloc(&C->pin_level, NP));
  STA_TRY(C->alloc(&C->level_order, NP));
  HIP_TRY(launch_pin_levels(d_kind, d_cell_of_pin, d_cell_level, d_drv_of_sink, C->pin_level, NP, nullptr));
  STA_TRY(tmp.alloc(&d_vals, NP));
  STA_TRY(tmp.alloc(&d_keys_out, NP));
  HIP_TRY(launch_iota(d_vals, NP, nullptr));
  int maxc = 0;
  for (int c = 0; c < NC; ++c) maxc = std::max(maxc, cell_level[c]);
  const int max_pin_level = 2 * maxc + 1;
  int bits = 1;
  while ((1 << bits) <= max_pin_level) ++bits;
  const size_t tb = level_sort_temp_bytes(NP);
  void *d_temp;
  STA_TRY(tmp.alloc(reinterpret_cast<unsigned char **>(&d_temp), tb));
  d_keys = C->pin_level;
  HIP_TRY(sort_levels(d_temp, tb, d_keys, d_keys_out, d_vals, C->level_order, NP, bits, nullptr));
  HIP_TRY(hipDeviceSynchronize());
  std::vector<int32_t> pl(NP);
  HIP_TRY(hipMemcpy(pl.data(), C->pin_level, NP * sizeof(int32_t), hipMemcpyDeviceToHost));
  C->n_levels = 1 + *std::max_element(pl.begin(), pl.end());
  C->n_cell_levels = maxc;
  return STA_OK;
}

static sta_status build_layout(sta_ctx *C, const Inputs &I, const std::vector<int32_t> &cell_level) {
  const sta_graph_desc &g = *I.g;
  const sta_lib_desc &lib = *I.lib;
  const sta_constraints &cons = *I.cons;
  const int NP = g.n_pins, NC = g.n_cells, NPI = g.n_pi;
  const int L = C->n_cell_levels;
  int big_thr = C->opt.big_net_nodes > 0 ? C->opt.big_net_nodes : kSmallNetMaxNodes;
  if (big_thr > kSmallNetMaxNodes) big_thr = kSmallNetMaxNodes;

  // driver slots: PIs by pin id, then cells by (level, type, RC node count of
  // the output net, output pin id): a level's chunks then hold one or two
  // cell types each, so a level kernel stages only those types' tables, and
  // consecutive nets have near-equal RC trees, so the RC kernel can take nets
  // in slot order (its outputs fill contiguous ranges) with balanced lanes
  std::vector<int32_t> drv_pin;
  drv_pin.reserve(NPI + NC);
  std::vector<int32_t> lvl_ptr(L + 2, 0);
  for (int p = 0; p < NP; ++p)
    if (I.pin_kind[p] == STA_PIN_PI) drv_pin.push_back(p);
  lvl_ptr[1] = NPI;
  {
    std::vector<int32_t> cnt(L + 2, 0);
    for (int c = 0; c < NC; ++c) cnt[cell_level[c]]++;
    for (int l = 1; l <= L; ++l) lvl_ptr[l + 1] = lvl_ptr[l] + cnt[l];
    std::vector<int32_t> fill(lvl_ptr.begin(), lvl_ptr.end());
    drv_pin.resize(NPI + NC);
    for (int p = 0; p < NP; ++p)
      if (I.pin_kind[p] == STA_PIN_CELL_OUT) drv_pin[fill[cell_level[I.cell_of_pin[p]]]++] = p;
    const auto nodes_of = [&](int p) {
      const int n = I.net_of_drv[p];
      return n < 0 ? (int64_t)0 : I.net_node_ptr[n + 1] - I.net_node_ptr[n];
    };
    for (int l = 1; l <= L; ++l)
      std::stable_sort(drv_pin.begin() + lvl_ptr[l], drv_pin.begin() + lvl_ptr[l + 1], [&](int a, int b) {
        const int ta = I.cell_type[I.cell_of_pin[a]], tb = I.cell_type[I.cell_of_pin[b]];
        return ta != tb ? ta < tb : nodes_of(a) < nodes_of(b);
      });
  }
  // within a level, drivers with more than kSplitSinks sinks go last: the
  // other chunks of the level are then runs of kChunk slots from the level's
  // first slot, which a per-level kernel computes from its block index
  const auto fanout_of = [&](int p) {
    const int n = I.net_of_drv[p];
    return n < 0 ? 0 : I.net_sink_ptr[n + 1] - I.net_sink_ptr[n];
  };
  C->lvl_reg.assign(L + 1, make_int4(0, 0, 0, 0));
  for (int l = 0; l <= L; ++l) {
    auto b = drv_pin.begin() + lvl_ptr[l], e = drv_pin.begin() + lvl_ptr[l + 1];
    auto mid = std::stable_partition(b, e, [&](int p) { return fanout_of(p) <= kSplitSinks; });
    C->lvl_reg[l] = make_int4(lvl_ptr[l], lvl_ptr[l] + (int)(mid - b), 0, 0);
  }
  const int ND = NPI + NC;
  C->n_drv = ND;
  std::vector<int32_t> slot_of_pin(NP, -1);
  for (int x = 0; x < ND; ++x) slot_of_pin[drv_pin[x]] = x;

  // endpoints: POs, plus dangling cell outputs under dangling_policy 1
  std::vector<int32_t> ep_of_pin(NP, -1), ep_pin;
  std::vector<float4> ep_rat;
  for (int p = 0; p < NP; ++p) {
    const int k = I.pin_kind[p];
    bool is_ep = k == STA_PIN_PO;
    if (k == STA_PIN_CELL_OUT && C->opt.dangling_policy) {
      const int n = I.net_of_drv[p];
      is_ep = I.net_sink_ptr[n + 1] == I.net_sink_ptr[n];
    }
    if (!is_ep) continue;
    ep_of_pin[p] = (int)ep_pin.size();
    ep_pin.push_back(p);
    if (k == STA_PIN_PO) {
      const float *r = cons.po_rat + 4 * (size_t)I.rank[p];
      ep_rat.push_back(make_float4(r[0], r[1], r[2], r[3]));
    } else {
      const float *r = cons.dangling_rat;
      if (I.dang) {
        const size_t dsg = std::upper_bound(I.pin_off->begin(), I.pin_off->end(), p) - I.pin_off->begin() - 1;
        r = I.dang->data() + 4 * dsg;
      }
      ep_rat.push_back(make_float4(r[0], r[1], r[2], r[3]));
    }
  }
  C->n_ep = (int)ep_pin.size();
  C->h_ep_pin = ep_pin;

  // nets in slot order, sinks net-major.  RC nodes net-major in "RC order":
  // the small nets chunk by chunk (below), then the wide nets.  rc_ptr[x] is
  // the first node of net x; rc_start / rc_order list the small nets by RC
  // position.
  std::vector<int32_t> sink_ptr(ND + 1, 0), rc_ptr(ND + 1, 0), net_slot(g.n_nets), rc_m(ND);
  int64_t NN = 0;
  for (int x = 0; x < ND; ++x) {
    const int n = I.net_of_drv[drv_pin[x]];
    net_slot[n] = x;
    sink_ptr[x + 1] = sink_ptr[x] + (I.net_sink_ptr[n + 1] - I.net_sink_ptr[n]);
    const int64_t m = I.net_node_ptr[n + 1] - I.net_node_ptr[n];
    NN += m;
    if (NN >= INT32_MAX) return fail(STA_E_UNSUPPORTED, "too many RC nodes");
    rc_m[x] = (int32_t)m;
  }
  std::vector<int32_t> rc_order, rc_start, rc_chunk_slot0;
  std::vector<int2> rc_chunks, rc_adj_chunks;
  {
    std::vector<int32_t> small, wide;
    for (int x = 0; x < ND; ++x) (rc_m[x] > big_thr ? wide : small).push_back(x);
    // RC chunks (one block each): within each window of kRcSortWindow
    // consecutive slots the small nets by ascending node count (ties by slot),
    // so the 64 trees a wave walks have near-equal sizes while a block's
    // outputs stay within one window of slots; then runs of <= kRcBlock nets
    // and <= kRcChunkNodes nodes.  (Runs of consecutive slots, sorted by size
    // only inside a run, measured 3% slower.)
    std::stable_sort(small.begin(), small.end(), [&](int a, int b) {
      const int wa = a / kRcSortWindow, wb = b / kRcSortWindow;
      return wa != wb ? wa < wb : rc_m[a] < rc_m[b];
    });
    size_t j0 = 0;
    while (j0 < small.size()) {
      size_t j1 = j0;
      int64_t nodes = 0;
      int mn = INT32_MAX;
      while (j1 < small.size() && (int)(j1 - j0) < kRcBlock && nodes + rc_m[small[j1]] <= kRcChunkNodes) {
        mn = std::min(mn, small[j1]);
        nodes += rc_m[small[j1++]];
      }
      rc_chunk_slot0.push_back(mn);
      rc_chunks.push_back(make_int2((int)j0, (int)j1));
      j0 = j1;
    }
    for (size_t a = 0; a < small.size();) {  // the adjoint's chunks: same order, smaller cuts
      size_t b = a;
      int64_t nodes = 0;
      while (b < small.size() && (int)(b - a) < kRcAdjBlock && nodes + rc_m[small[b]] <= kRcAdjChunkNodes)
        nodes += rc_m[small[b++]];
      rc_adj_chunks.push_back(make_int2((int)a, (int)b));
      a = b;
    }
    int32_t pos = 0;
    rc_start.reserve(small.size() + 1);
    for (int x : small) {
      rc_start.push_back(pos);
      rc_ptr[x] = pos;
      pos += rc_m[x];
    }
    rc_start.push_back(pos);
    for (int x : wide) {
      rc_ptr[x] = pos;
      pos += rc_m[x];
    }
    rc_ptr[ND] = pos;
    rc_order = std::move(small);
  }
  const int NS = sink_ptr[ND];
  C->n_sinks = NS;
  C->n_nodes = NN;
  std::vector<int32_t> sink_drv(NS), sink_cons(NS), sink_node(NS), sink_slot(NS), pin_loc(NP), sink_pin_of_slot(NS);
  std::vector<float> sink_pincap(NS), rc_res(NN), rc_cap(NN);
  std::vector<int32_t> rc_parent(NN), node_src(NN), big_x, big_end, big_nsp, big_nsl, big_egp, big_egl;
  std::vector<float> big_pc;
  std::vector<BigNet> big;
  int64_t big_scr = 0;
  for (int x = 0; x < ND; ++x) {
    const int n = I.net_of_drv[drv_pin[x]];
    const int64_t cb = I.net_node_ptr[n];
    const int m = rc_m[x];
    const int base = rc_ptr[x];
    const bool is_big = m > big_thr;
    std::vector<int32_t> newof;
    if (is_big) {
      newof = preorder(I.parent.p + cb, m);
      big_x.push_back(x);
      BigNet bn;
      bn.x = x;
      bn.m = m;
      bn.aux = (int64_t)big_end.size();
      bn.scr = big_scr;
      bn.nsp = (int64_t)big_nsp.size();
      bn.egp = (int64_t)big_egp.size();
      bn.nblk = (m + kWideSeg - 1) / kWideSeg;
      // the blocks of one net wait for each other, so all of them must fit on
      // the device at once (2 blocks of 1024 threads per compute unit)
      if (bn.nblk > 2 * std::max(C->n_cu, 1))
        return fail(STA_E_UNSUPPORTED, "RC net of %d nodes exceeds the wide-net limit", m);
      bn.tot = big.empty() ? 0 : big.back().tot + big.back().nblk;
      big.push_back(bn);
      big_scr += kBigScratch * ((int64_t)m + 1);
    }
    for (int k = 0; k < m; ++k) {
      const int nk = is_big ? newof[k] : k;
      const int pk = I.parent[cb + k];
      rc_parent[base + nk] = pk < 0 ? -1 : (is_big ? newof[pk] : pk);
      rc_res[base + nk] = I.res[cb + k];
      rc_cap[base + nk] = I.cap[cb + k];
      node_src[base + nk] = (int32_t)(cb + k);
    }
    if (is_big) {
      // subtree end of each node in preorder, and the receiving pin caps per node
      std::vector<int32_t> size(m, 1);
      for (int k = m - 1; k >= 1; --k) size[rc_parent[base + k]] += size[k];
      std::vector<double> pcd(m, 0.0);
      for (int sc = I.net_sink_ptr[n]; sc < I.net_sink_ptr[n + 1]; ++sc) {
        const int p = I.net_sink_pin[sc];
        pcd[newof[I.sink_node[sc]]] +=
            I.pin_kind[p] == STA_PIN_PO ? I.po_cap(p) : lib.pin_cap_ff[I.cell_type[I.cell_of_pin[p]]];
      }
      for (int k = 0; k < m; ++k) {
        big_end.push_back(k + size[k]);
        big_pc.push_back((float)pcd[k]);
      }
      // Euler end-groups: for p in [0, m], the nodes a with end_a = p, found by
      // walking up from p - 1 (a chain), kept deepest first
      // (offsets local to the net; its list starts at its node offset aux,
      // since every node belongs to exactly one group)
      const int32_t *endv = big_end.data() + (big_end.size() - m);
      const size_t gbase = big_egl.size();
      big_egp.push_back(0);  // group p spans [egp[p], egp[p+1]); group 0 is empty
      big_egp.push_back(0);
      for (int p = 1; p <= m; ++p) {
        for (int a = p - 1; a >= 0 && endv[a] == p; a = rc_parent[base + a]) big_egl.push_back(a);
        big_egp.push_back((int32_t)(big_egl.size() - gbase));
      }
      // sinks of each node (local sink index, sink order) for the adjoint seeds
      std::vector<int32_t> cnt(m + 1, 0);
      const int ns = I.net_sink_ptr[n + 1] - I.net_sink_ptr[n];
      for (int j = 0; j < ns; ++j) cnt[newof[I.sink_node[I.net_sink_ptr[n] + j]] + 1]++;
      for (int k = 0; k < m; ++k) cnt[k + 1] += cnt[k];
      const int32_t lbase = (int32_t)big_nsl.size();
      for (int k = 0; k <= m; ++k) big_nsp.push_back(lbase + cnt[k]);
      big_nsl.resize(big_nsl.size() + ns);
      for (int j = 0; j < ns; ++j) big_nsl[lbase + cnt[newof[I.sink_node[I.net_sink_ptr[n] + j]]]++] = j;
    }
    int s = sink_ptr[x];
    for (int sc = I.net_sink_ptr[n]; sc < I.net_sink_ptr[n + 1]; ++sc, ++s) {
      const int p = I.net_sink_pin[sc];
      sink_slot[sc] = s;
      sink_pin_of_slot[s] = p;
      sink_drv[s] = x;
      const int k = I.sink_node[sc];
      sink_node[s] = is_big ? newof[k] : k;
      if (I.pin_kind[p] == STA_PIN_PO) {
        sink_pincap[s] = I.po_cap(p);
        sink_cons[s] = -1 - ep_of_pin[p];
      } else {
        const int c = I.cell_of_pin[p];
        sink_pincap[s] = lib.pin_cap_ff[I.cell_type[c]];
        sink_cons[s] = slot_of_pin[I.cell_out_pin[c]];
      }
      pin_loc[p] = -1 - s;
    }
    pin_loc[drv_pin[x]] = x;
  }
  C->n_big = (int)big_x.size();

  // per driver slot: cell type, fanin (sink slots of the inputs), endpoint
  std::vector<int32_t> cell_type(ND, -1), fanin_ptr(ND + 1, 0), fanin_sink, drv_ep(ND, -1), arc_src;
  fanin_sink.reserve(I.cell_in_ptr[NC]);
  arc_src.reserve(I.cell_in_ptr[NC]);
  for (int x = 0; x < ND; ++x) {
    const int p = drv_pin[x];
    drv_ep[x] = ep_of_pin[p];
    if (x >= NPI) {
      const int c = I.cell_of_pin[p];
      cell_type[x] = I.cell_type[c];
      for (int k = I.cell_in_ptr[c]; k < I.cell_in_ptr[c + 1]; ++k) {
        fanin_sink.push_back(sink_slot[I.sink_idx_of_pin[I.cell_in_pin[k]]]);
        arc_src.push_back(k);
      }
    }
    fanin_ptr[x + 1] = (int32_t)fanin_sink.size();
  }
  std::vector<int32_t> ep_loc(ep_pin.size());
  for (size_t e = 0; e < ep_pin.size(); ++e) ep_loc[e] = pin_loc[ep_pin[e]];
  C->n_fanin = (int)fanin_sink.size();
  std::vector<float4> pi_at(NPI), pi_slew(NPI);
  for (int x = 0; x < NPI; ++x) {
    const int r = I.rank[drv_pin[x]];
    const float *a = cons.pi_at + 4 * (size_t)r, *s = cons.pi_slew + 4 * (size_t)r;
    pi_at[x] = make_float4(a[0], a[1], a[2], a[3]);
    pi_slew[x] = make_float4(s[0], s[1], s[2], s[3]);
  }

  // sweep chunks: up to 64 consecutive slots of one level; a driver with more
  // than kSplitSinks sinks gets a chunk of its own, which keeps the first
  // kPieceSinks sinks, the rest going to pieces of kPieceSinks sinks.
  // Phases: forward = per level its chunks, then its pieces; backward = per
  // level (descending) its pieces, then its chunks; adjoint = chunks only.
  std::vector<int4> chunk_rec, piece_rec;
  std::vector<int2> chunk_pieces;
  std::vector<int32_t> lvl_cbeg(L + 2, 0), lvl_pbeg(L + 2, 0);
  for (int l = 0; l <= L; ++l) {
    lvl_cbeg[l] = (int)chunk_rec.size();
    lvl_pbeg[l] = (int)piece_rec.size();
    int x = lvl_ptr[l];
    while (x < lvl_ptr[l + 1]) {
      const auto fanout = [&](int y) { return sink_ptr[y + 1] - sink_ptr[y]; };
      if (fanout(x) > kSplitSinks) {
        const int c = (int)chunk_rec.size();
        const int s0 = sink_ptr[x], s1 = sink_ptr[x + 1];
        chunk_rec.push_back(make_int4(x, x + 1, s0, s0 + kPieceSinks));
        const int p0 = (int)piece_rec.size();
        for (int a = s0 + kPieceSinks; a < s1; a += kPieceSinks)
          piece_rec.push_back(make_int4(x, a, std::min(s1, a + kPieceSinks), c));
        chunk_pieces.push_back(make_int2(p0, (int)piece_rec.size() - p0));
        ++x;
        continue;
      }
      int y = x;
      while (y < lvl_ptr[l + 1] && y - x < kChunk && fanout(y) <= kSplitSinks) ++y;
      chunk_rec.push_back(make_int4(x, y, sink_ptr[x], sink_ptr[y]));
      chunk_pieces.push_back(make_int2(0, 0));
      x = y;
    }
  }
  lvl_cbeg[L + 1] = (int)chunk_rec.size();
  lvl_pbeg[L + 1] = (int)piece_rec.size();
  // library types each chunk's cells use, as (lowest, highest); (0, -1) for none
  std::vector<int2> chunk_trange(chunk_rec.size(), make_int2(0, -1));
  for (size_t c = 0; c < chunk_rec.size(); ++c) {
    int lo = INT32_MAX, hi = -1;
    for (int x = chunk_rec[c].x; x < chunk_rec[c].y; ++x)
      if (cell_type[x] >= 0) {
        lo = std::min(lo, cell_type[x]);
        hi = std::max(hi, cell_type[x]);
      }
    if (hi >= 0) chunk_trange[c] = make_int2(lo, hi);
  }
  // per level, the float4 granules of the widest type span of a block of the
  // level kernels (chunks paired from the level's first, kLevelCpb a block),
  // the LDS those kernels reserve for the tables
  {
    const int ts = TabLayout{lib.nx, lib.ny}.stride();
    for (int l = 0; l <= L; ++l) {
      int most = 0;
      for (int c = lvl_cbeg[l]; c < lvl_cbeg[l + 1]; c += kLevelCpb) {
        int lo = INT32_MAX, hi = -1;
        for (int h = c; h < std::min(c + kLevelCpb, lvl_cbeg[l + 1]); ++h)
          if (chunk_trange[h].y >= chunk_trange[h].x) {
            lo = std::min(lo, chunk_trange[h].x);
            hi = std::max(hi, chunk_trange[h].y);
          }
        if (hi >= lo) most = std::max(most, (((hi + 1) * ts + 3) >> 2) - ((lo * ts) >> 2));
      }
      C->lvl_reg[l].z = most;
    }
  }
  C->n_chunks = (int)chunk_rec.size();
  C->n_pieces = (int)piece_rec.size();
  C->ph_fwd.clear();
  C->ph_bwd.clear();
  C->ph_adj.clear();
  for (int l = 0; l <= L; ++l) {
    C->ph_fwd.push_back(make_int4(kItemChunk, lvl_cbeg[l], lvl_cbeg[l + 1] - lvl_cbeg[l], l));
    if (lvl_pbeg[l + 1] > lvl_pbeg[l])
      C->ph_fwd.push_back(make_int4(kItemPiece, lvl_pbeg[l], lvl_pbeg[l + 1] - lvl_pbeg[l], l));
  }
  for (int l = L; l >= 0; --l) {
    if (lvl_pbeg[l + 1] > lvl_pbeg[l])
      C->ph_bwd.push_back(make_int4(kItemPiece, lvl_pbeg[l], lvl_pbeg[l + 1] - lvl_pbeg[l], l));
    C->ph_bwd.push_back(make_int4(kItemChunk, lvl_cbeg[l], lvl_cbeg[l + 1] - lvl_cbeg[l], l));
    C->ph_adj.push_back(make_int4(kItemChunk, lvl_cbeg[l], lvl_cbeg[l + 1] - lvl_cbeg[l], l));
  }
  // inline fanin sink slots when every type has at most 4 inputs
  int max_in = 0;
  for (int t = 0; t < lib.n_types; ++t) max_in = std::max(max_in, (int)lib.n_inputs[t]);
  C->max_in = std::max(max_in, 1);
  C->D.max_in = C->max_in;
  std::vector<int4> fanin4;
  if (max_in <= 4) {
    fanin4.assign(ND, make_int4(-1, -1, -1, -1));
    for (int x = NPI; x < ND; ++x) {
      int v[4] = {-1, -1, -1, -1};
      for (int f = fanin_ptr[x]; f < fanin_ptr[x + 1]; ++f) v[f - fanin_ptr[x]] = fanin_sink[f];
      fanin4[x] = make_int4(v[0], v[1], v[2], v[3]);
    }
  }
  std::vector<ConsRec> cons_rec(ND);
  for (int x = 0; x < ND; ++x) {
    cons_rec[x] = ConsRec{};
    cons_rec[x].type = cell_type[x];
  }

  C->n_rc_chunks = (int)rc_chunks.size();
  // level groups of the RC pass (levels [0,2), [2,4), [4,8), [8,16), then 16
  // at a time): group g launches the RC chunks the levels before the next
  // group need.  Chunks are in window order (rc_chunk_slot0: a chunk's lowest slot).
  {
    C->rc_grp_lvl.clear();
    C->rc_grp_end.clear();
    std::vector<int32_t> bounds;
    for (int a = 0; a <= L; a = a < 2 ? 2 : (a < 16 ? 2 * a : a + 16)) bounds.push_back(a);
    bounds.push_back(L + 1);
    size_t r = 0;
    for (size_t g = 0; g + 1 < bounds.size(); ++g) {
      const int last_slot = lvl_ptr[bounds[g + 1]] - 1;
      while (r < rc_chunks.size() && rc_chunk_slot0[r] / kRcSortWindow <= last_slot / kRcSortWindow) ++r;
      C->rc_grp_lvl.push_back(bounds[g]);
      C->rc_grp_end.push_back((int32_t)r);
    }
    C->rc_grp_end.back() = (int32_t)rc_chunks.size();
    C->wide_lvl = INT32_MAX;
    for (int x : big_x) {
      const int l = (int)(std::upper_bound(lvl_ptr.begin(), lvl_ptr.end(), x) - lvl_ptr.begin()) - 1;
      C->wide_lvl = std::min(C->wide_lvl, l);
    }
  }

  // packed library
  const TabLayout lay{lib.nx, lib.ny};
  const int ts = lay.stride();
  std::vector<float> tab(((size_t)lib.n_types * ts + 3) & ~(size_t)3, 0.0f);  // padded for 16-byte staging loads
  for (int t = 0; t < lib.n_types; ++t) {
    float *o = tab.data() + (size_t)t * ts;
    const float *xa = lib.slew_axis + t * lib.nx, *ya = lib.load_axis + t * lib.ny;
    for (int i = 0; i < lib.nx; ++i) o[lay.xa() + i] = xa[i];
    for (int j = 0; j < lib.ny; ++j) o[lay.ya() + j] = ya[j];
    for (int i = 0; i + 1 < lib.nx; ++i) o[lay.rdx() + i] = 1.0f / (xa[i + 1] - xa[i]);
    for (int j = 0; j + 1 < lib.ny; ++j) o[lay.rdy() + j] = 1.0f / (ya[j + 1] - ya[j]);
    std::memcpy(o + lay.tab(0), lib.tables + (size_t)t * 4 * lib.nx * lib.ny, sizeof(float) * 4 * lib.nx * lib.ny);
  }
  std::vector<int32_t> sense(lib.sense, lib.sense + lib.n_types);

  // upload
  DevDesign &D = C->D;
  D.n_drv = ND;
  D.n_pi = NPI;
  D.n_sinks = NS;
  D.n_ep = C->n_ep;
  D.n_cell_levels = L;
  D.n_types = lib.n_types;
  D.nx = lib.nx;
  D.ny = lib.ny;
  D.tstride = ts;
  D.n_chunks = C->n_chunks;
  int32_t *p32;
  float *pf;
  float4 *p4;
  STA_TRY(C->upload(&p32, sink_ptr)); D.sink_ptr = p32;
  STA_TRY(C->upload(&p32, rc_ptr)); D.rc_ptr = p32;
  STA_TRY(C->upload(&p32, rc_order)); D.rc_order = p32;
  STA_TRY(C->upload(&p32, rc_start)); D.rc_start = p32;
  STA_TRY(C->upload(&p32, fanin_ptr)); D.fanin_ptr = p32;
  STA_TRY(C->upload(&p32, fanin_sink)); D.fanin_sink = p32;
  STA_TRY(C->upload(&p32, cell_type)); D.cell_type = p32;
  STA_TRY(C->upload(&p32, drv_ep)); D.drv_ep = p32;
  STA_TRY(C->upload(&p4, pi_at)); D.pi_at = p4;
  STA_TRY(C->upload(&p4, pi_slew)); D.pi_slew = p4;
  STA_TRY(C->upload(&p32, sink_drv)); D.sink_drv = p32;
  STA_TRY(C->upload(&p32, sink_cons)); D.sink_cons = p32;
  STA_TRY(C->upload(&p32, sink_node)); D.sink_node = p32;
  {
    // small-net parents as bytes, lumped pin caps per node, sink ranges per RC position
    std::vector<uint8_t> par8(NN, 0);
    std::vector<double> pcd(NN, 0.0);
    std::vector<int2> rc_sinks(rc_order.size());
    for (int x = 0; x < ND; ++x) {
      const int base = rc_ptr[x];
      for (int s = sink_ptr[x]; s < sink_ptr[x + 1]; ++s) pcd[base + sink_node[s]] += sink_pincap[s];
      if (rc_m[x] > big_thr) continue;
      for (int k = 1; k < rc_m[x]; ++k) par8[base + k] = (uint8_t)rc_parent[base + k];
    }
    for (size_t j = 0; j < rc_order.size(); ++j)
      rc_sinks[j] = make_int2(sink_ptr[rc_order[j]], sink_ptr[rc_order[j] + 1]);
    std::vector<float> pcf(pcd.begin(), pcd.end());
    // the small nets' C^ = wire cap + pin caps, the float sum the RC pass reads
    // (wide nets keep the wire cap; their kernels add the pin caps in FP64)
    C->n_small_nodes = rc_start.back();
    for (int64_t k = 0; k < C->n_small_nodes; ++k) rc_cap[k] = rc_cap[k] + pcf[k];
    uint8_t *p8;
    STA_TRY(C->upload(&p8, par8)); D.rc_par8 = p8;
    STA_TRY(C->upload(&pf, pcf)); D.rc_pc = pf;
    C->rc_pc = pf;
    int2 *p2;
    STA_TRY(C->upload(&p2, rc_sinks)); D.rc_sinks = p2;
  }
  STA_TRY(C->upload(&pf, rc_res)); D.rc_res = pf;
  STA_TRY(C->upload(&C->rc_cap, rc_cap)); D.rc_cap = C->rc_cap;
  STA_TRY(C->upload(&p4, ep_rat)); D.ep_rat = p4;
  STA_TRY(C->upload(&pf, tab)); D.tables = pf;
  STA_TRY(C->upload(&p32, sense)); D.sense = p32;
  {
    int4 *p4i;
    STA_TRY(C->upload(&p4i, chunk_rec)); D.chunk_rec = p4i;
    D.fanin4 = nullptr;
    if (!fanin4.empty()) {
      STA_TRY(C->upload(&p4i, fanin4));
      D.fanin4 = p4i;
    }
    ConsRec *pcr;
    STA_TRY(C->upload(&pcr, cons_rec)); D.cons_rec = pcr;
  }
  {
    std::vector<int4> ph(C->ph_fwd);
    ph.insert(ph.end(), C->ph_bwd.begin(), C->ph_bwd.end());
    ph.insert(ph.end(), C->ph_adj.begin(), C->ph_adj.end());
    int4 *p4i;
    STA_TRY(C->upload(&p4i, ph)); D.phases = p4i;
    D.n_ph_fwd = (int)C->ph_fwd.size();
    D.n_ph_bwd = (int)C->ph_bwd.size();
    D.n_ph_adj = (int)C->ph_adj.size();
    if (piece_rec.empty()) piece_rec.push_back(make_int4(0, 0, 0, 0));  // never read
    STA_TRY(C->upload(&p4i, piece_rec)); D.piece_rec = p4i;
    int2 *p2i;
    STA_TRY(C->upload(&p2i, chunk_pieces)); D.chunk_pieces = p2i;
    int2 *tr;
    STA_TRY(C->upload(&tr, chunk_trange)); D.chunk_trange = tr;
    STA_TRY(C->alloc(&D.piece_rat, std::max(C->n_pieces, 1)));
  }
  STA_TRY(C->alloc(&D.L_net, ND));
  STA_TRY(C->alloc(&D.dq, NS));
  STA_TRY(C->alloc(&D.drv_state, ND));
  STA_TRY(C->alloc(&D.sink_state, NS));
  STA_TRY(C->alloc(&D.drv_crit, ND));
  STA_TRY(C->alloc(&D.sink_rat, NS));
  STA_TRY(C->alloc(&D.drv_slack, ND));
  STA_TRY(C->alloc(&D.sink_slack, NS));
  STA_TRY(C->alloc(&D.ep_slack, C->n_ep));
  const int n_ctr = n_counters(D.n_ph_fwd + D.n_ph_bwd);
  STA_TRY(C->alloc(&D.counters, n_ctr));
  HIP_TRY(hipMemset(D.counters, 0, n_ctr * sizeof(uint32_t)));

  STA_TRY(C->upload(&C->pin_loc, pin_loc));
  STA_TRY(C->upload(&C->net_slot, net_slot));
  STA_TRY(C->upload(&C->sink_slot, sink_slot));
  STA_TRY(C->upload(&C->node_src, node_src));
  STA_TRY(C->upload(&C->ep_pin, ep_pin));
  STA_TRY(C->upload(&C->slot_drv_pin, drv_pin));
  STA_TRY(C->upload(&C->slot_sink_pin, sink_pin_of_slot));
  STA_TRY(C->upload(&C->rc_chunks, rc_chunks));
  STA_TRY(C->upload(&C->rc_adj_chunks, rc_adj_chunks));
  C->n_rc_adj_chunks = (int)rc_adj_chunks.size();
  STA_TRY(C->upload(&C->big, big));
  {
    // incremental update: chunk and phases of every driver / chunk, and the
    // host maps from a net to what recomputes it
    std::vector<int32_t> chunk_of(ND, 0);
    for (size_t c = 0; c < chunk_rec.size(); ++c)
      for (int x = chunk_rec[c].x; x < chunk_rec[c].y; ++x) chunk_of[x] = (int32_t)c;
    std::vector<int32_t> fph(L + 1, 0), bph(L + 1, 0);
    for (size_t k = 0; k < C->ph_fwd.size(); ++k)
      if (C->ph_fwd[k].x == kItemChunk) fph[C->ph_fwd[k].w] = (int32_t)k;
    for (size_t k = 0; k < C->ph_bwd.size(); ++k)
      if (C->ph_bwd[k].x == kItemChunk) bph[C->ph_bwd[k].w] = (int32_t)k;
    std::vector<int2> chunk_ph(chunk_rec.size());
    for (int l = 0; l <= L; ++l)
      for (int c = lvl_cbeg[l]; c < lvl_cbeg[l + 1]; ++c) chunk_ph[c] = make_int2(fph[l], bph[l]);
    STA_TRY(C->upload(&C->inc_chunk_of, chunk_of));
    STA_TRY(C->upload(&C->inc_chunk_ph, chunk_ph));
    // dataflow sweeps: items in sweep order, the forward item producing each
    // inline input sink (its driver's chunk, or the piece holding it) and the
    // backward item writing each sink's RAT (its consumer's chunk)
    int most_pieces = 0;
    for (const int2 &cp : chunk_pieces) most_pieces = std::max(most_pieces, cp.y);
    C->flow_ok = !fanin4.empty() && most_pieces <= kSweepBlock;
    if (C->flow_ok) {
      std::vector<int2> fi, bi;
      for (int l = 0; l <= L; ++l) {
        for (int c = lvl_cbeg[l]; c < lvl_cbeg[l + 1]; ++c) fi.push_back(make_int2(kItemChunk, c));
        for (int j = lvl_pbeg[l]; j < lvl_pbeg[l + 1]; ++j) fi.push_back(make_int2(kItemPiece, j));
      }
      for (int l = L; l >= 0; --l) {
        for (int j = lvl_pbeg[l]; j < lvl_pbeg[l + 1]; ++j) bi.push_back(make_int2(kItemPiece, j));
        for (int c = lvl_cbeg[l]; c < lvl_cbeg[l + 1]; ++c) bi.push_back(make_int2(kItemChunk, c));
      }
      const int NCH = (int)chunk_rec.size();
      auto producer = [&](int f) {  // forward item that writes sink f
        const int y = sink_drv[f], k = f - sink_ptr[y], c = chunk_of[y];
        if (chunk_pieces[c].y > 0 && k >= kPieceSinks) return NCH + chunk_pieces[c].x + (k - kPieceSinks) / kPieceSinks;
        return c;
      };
      std::vector<int4> fin(ND, make_int4(-1, -1, -1, -1));
      for (int x = NPI; x < ND; ++x) {
        const int fs[4] = {fanin4[x].x, fanin4[x].y, fanin4[x].z, fanin4[x].w};
        int o[4];
        for (int k = 0; k < 4; ++k) o[k] = fs[k] >= 0 ? producer(fs[k]) : -1;
        fin[x] = make_int4(o[0], o[1], o[2], o[3]);
      }
      std::vector<int32_t> sitem(std::max(NS, 1), -1);
      for (int f = 0; f < NS; ++f) sitem[f] = sink_cons[f] >= 0 ? chunk_of[sink_cons[f]] : -1;
      int2 *p2;
      STA_TRY(C->upload(&p2, fi));
      C->flow_fwd.items = p2;
      C->flow_fwd.n_items = (int)fi.size();
      STA_TRY(C->upload(&p2, bi));
      C->flow_bwd.items = p2;
      C->flow_bwd.n_items = (int)bi.size();
      int4 *p4;
      STA_TRY(C->upload(&p4, fin));
      int32_t *pi;
      STA_TRY(C->upload(&pi, sitem));
      const size_t nf = (size_t)NCH + std::max<size_t>(piece_rec.size(), 1);
      uint32_t *flags;
      STA_TRY(C->alloc(&flags, 2 * nf + 1));
      HIP_TRY(hipMemset(flags, 0, (2 * nf + 1) * sizeof(uint32_t)));
      for (FlowArgs *F : {&C->flow_fwd, &C->flow_bwd}) {
        F->fin_item = p4;
        F->sink_item = pi;
        F->err = flags + 2 * nf;
      }
      C->flow_fwd.flag = flags;
      C->flow_bwd.flag = flags + nf;
      C->flow_err = flags + 2 * nf;
    }
    std::vector<int32_t> slot_rc(ND, 0);
    for (size_t r = 0; r < rc_chunks.size(); ++r)
      for (int j = rc_chunks[r].x; j < rc_chunks[r].y; ++j) slot_rc[rc_order[j]] = (int32_t)r;
    for (size_t i = 0; i < big.size(); ++i) slot_rc[big[i].x] = -1 - (int32_t)i;
    STA_TRY(C->upload(&C->inc_slot_rc, slot_rc));
  }
  {
    // one launched block per (wide net, segment); per-net barrier counters
    std::vector<int2> blk;
    for (size_t i = 0; i < big.size(); ++i)
      for (int b = 0; b < big[i].nblk; ++b) blk.push_back(make_int2((int)i, b));
    const int n_tot = big.empty() ? 1 : big.back().tot + big.back().nblk;
    int2 *pb;
    STA_TRY(C->upload(&pb, blk));
    C->wide.blk = pb;
    C->wide.n_blk = (int)blk.size();
    STA_TRY(C->alloc(&C->wide.tot, n_tot));
    STA_TRY(C->alloc(&C->wide.sync, std::max<size_t>(2 * big.size(), 1)));
    HIP_TRY(hipMemset(C->wide.sync, 0, std::max<size_t>(2 * big.size(), 1) * sizeof(uint32_t)));
  }
  STA_TRY(C->upload(&C->big_end, big_end));
  STA_TRY(C->upload(&C->big_pc, big_pc));
  STA_TRY(C->upload(&C->big_nsp, big_nsp));
  STA_TRY(C->upload(&C->big_nsl, big_nsl));
  if (big_egl.size() != big_end.size()) return fail(STA_E_DEVICE, "internal: Euler group size mismatch");
  STA_TRY(C->upload(&C->big_egp, big_egp));
  STA_TRY(C->upload(&C->big_egl, big_egl));
  STA_TRY(C->upload(&C->arc_src, arc_src));
  STA_TRY(C->upload(&p32, ep_loc)); D.ep_loc = p32;
  D.gamma = C->opt.mode == 1 ? C->opt.gamma_ps : 0.0f;
  D.delay_model = C->opt.delay_model;
  if (C->opt.mode == 1) {
    STA_TRY(C->alloc(&D.g_sink, NS));
    STA_TRY(C->alloc(&D.g_dq, NS));
    STA_TRY(C->alloc(&D.g_load, ND));
    STA_TRY(C->alloc(&D.g_arc, std::max(C->n_fanin, 1)));
    STA_TRY(C->alloc(&D.g_cap, NN));
    STA_TRY(C->alloc(&D.g_res, NN));
  }
  STA_TRY(C->alloc(&C->big_scratch, (size_t)std::max<int64_t>(big_scr, 1)));
  STA_TRY(C->alloc(&C->partials, 8 * kReduceBlocks));
  STA_TRY(C->alloc(&C->out, 8));
  HIP_TRY(hipMemset(C->out, 0, 8 * sizeof(double)));
  D.norm = C->out + 4;
  const int ne = std::max(C->n_ep, 1);
  STA_TRY(C->alloc(&C->keys64, 2 * (size_t)ne));
  STA_TRY(C->alloc(&C->keys64_out, 2 * (size_t)ne));
  STA_TRY(C->alloc(&C->vals, 2 * (size_t)ne));
  STA_TRY(C->alloc(&C->order, 2 * (size_t)ne));
  C->key_bits = 33;
  C->sort_bytes = sort_temp_bytes64(2 * ne, C->key_bits);
  unsigned char *st;
  STA_TRY(C->alloc(&st, C->sort_bytes));
  C->sort_temp = st;

  C->wide.big = C->big;
  C->wide.n_big = C->n_big;
  C->wide.end = C->big_end;
  C->wide.nsp = C->big_nsp;
  C->wide.nsl = C->big_nsl;
  C->wide.egp = C->big_egp;
  C->wide.egl = C->big_egl;
  C->wide.pc = C->big_pc;
  C->wide.scratch = C->big_scratch;
  HIP_TRY(device_side_streams(C->device, &C->side, &C->side2));
  HIP_TRY(hipEventCreateWithFlags(&C->ev_fork, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&C->ev_join, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&C->ev_fwd, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&C->ev_red, hipEventDisableTiming));
  C->ev_rc.assign(C->rc_grp_lvl.size(), nullptr);
  for (auto &e : C->ev_rc) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));

  // persistent grid: every resident block slot on the device.  The level-major
  // cooperative kernels need every block resident, which the cooperative
  // launch guarantees; without cooperative launch support, or for a requested
  // grid beyond the resident limit, the ticket kernels (correct for any grid)
  // are used.
  const size_t lds = sweep_lds_bytes(D);
  if (lds > 160 * 1024) return fail(STA_E_UNSUPPORTED, "library too large for LDS (%zu bytes)", lds);
  C->sweep_grid = sweep_blocks_per_cu(lds) * C->n_cu;
  if (C->sweep_grid < 1) C->sweep_grid = 1;
  int coop_ok = 0;
  HIP_TRY(hipDeviceGetAttribute(&coop_ok, hipDeviceAttributeCooperativeLaunch, C->device));
  C->coop_max = coop_ok ? coop_blocks_per_cu(lds) * C->n_cu : 0;
  if (C->coop_max > 0) C->sweep_grid = C->coop_max;
  if (C->opt.sweep_blocks > 0) C->sweep_grid = C->opt.sweep_blocks;
  C->coop = C->sweep_grid <= C->coop_max;
  C->flow_grid = coop_ok ? flow_blocks_per_cu(D) * C->n_cu : 0;
  if (C->flow_grid <= 0) C->flow_ok = false;
  if (C->opt.sched == STA_SCHED_FLOW && !C->flow_ok)
    return fail(STA_E_UNSUPPORTED, "the dataflow schedule needs inline fanins (types of at most 4 inputs), at most "
                                   "%d sink pieces per driver and cooperative launch", kSweepBlock);
  return STA_OK;
}

// Copies n bytes of device data to dst (host or device).
static sta_status deliver(void *dst, const void *src, size_t bytes, sta_mem m, hipStream_t s) {
  if (!dst || bytes == 0) return STA_OK;
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, m == STA_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
  return STA_OK;
}

static sta_status check_options(const sta_options &o) {
  if (o.mode != 0 && o.mode != 1) return fail(STA_E_ARG, "mode must be 0 (hard) or 1 (smooth)");
  if (o.mode == 1 && !(o.gamma_ps > 0.0f && std::isfinite(o.gamma_ps)))
    return fail(STA_E_ARG, "smooth mode needs a finite gamma_ps > 0");
  if (o.sched != STA_SCHED_PERSISTENT && o.sched != STA_SCHED_PER_LEVEL && o.sched != STA_SCHED_GRAPH &&
      o.sched != STA_SCHED_FLOW)
    return fail(STA_E_ARG, "bad sched");
  if (o.big_net_nodes < 0) return fail(STA_E_ARG, "big_net_nodes < 0");
  if (o.dangling_policy != 0 && o.dangling_policy != 1) return fail(STA_E_ARG, "bad dangling_policy");
  if (o.sweep_blocks < 0) return fail(STA_E_ARG, "sweep_blocks < 0");
  if (o.delay_model != 0 && o.delay_model != 1) return fail(STA_E_ARG, "delay_model must be 0 or 1");
  if (o.delay_model == 1 && o.mode == 1)
    return fail(STA_E_UNSUPPORTED, "the reduced-order delay model has no adjoint (smooth mode)");
  return STA_OK;
}

static sta_status init_device(sta_ctx *C) {
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (ndev < 1) return fail(STA_E_DEVICE, "no HIP device");
  if (C->opt.device >= 0) {
    if (C->opt.device >= ndev) return fail(STA_E_ARG, "device %d of %d", C->opt.device, ndev);
    HIP_TRY(hipSetDevice(C->opt.device));
  }
  HIP_TRY(hipGetDevice(&C->device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, C->device));
  C->n_cu = prop.multiProcessorCount;
  return STA_OK;
}

// Levelizes the validated inputs and builds the device layout.
static sta_status build_context(sta_ctx *C, const Inputs &I) {
  const sta_graph_desc &g = *I.g;
  C->n_pins = g.n_pins;
  C->n_cells = g.n_cells;
  C->n_nets = g.n_nets;
  C->n_pi = g.n_pi;
  C->n_po = g.n_po;
  std::vector<int32_t> cell_level;
  STA_TRY(levelize(C, I, cell_level));
  STA_TRY(build_layout(C, I, cell_level));
  for (auto &e : C->ev) HIP_TRY(hipEventCreate(&e));
  C->events = true;
  return STA_OK;
}

extern "C" sta_status sta_create(const sta_graph_desc *graph, const sta_rc_desc *rc, const sta_lib_desc *lib,
                                 const sta_constraints *cons, const sta_options *opts, sta_ctx **out) {
  if (!graph || !rc || !lib || !cons || !out) return fail(STA_E_ARG, "NULL descriptor");
  sta_options o;
  sta_options_default(&o);
  if (opts) o = *opts;
  STA_TRY(check_options(o));
  STA_TRY(validate_lib(*lib));
  Inputs I;
  I.g = graph;
  I.rc = rc;
  I.lib = lib;
  I.cons = cons;
  // device memory inputs need the device before validation
  const bool dev_in = graph->mem == STA_DEVICE || rc->mem == STA_DEVICE;
  auto C = std::make_unique<sta_ctx>();
  C->opt = o;
  if (dev_in) STA_TRY(init_device(C.get()));
  STA_TRY(load_graph(I));
  STA_TRY(validate_graph(I));
  STA_TRY(load_validate_rc(I));
  STA_TRY(validate_cons(*cons, *graph));
  if (!dev_in) STA_TRY(init_device(C.get()));
  STA_TRY(build_context(C.get(), I));
  C->pin_off = {0, C->n_pins};
  C->ep_off = {0, C->n_ep};
  C->node_off = {0, C->n_nodes};
  HIP_TRY(hipDeviceSynchronize());
  *out = C.release();
  return STA_OK;
}

// ------------------------------------------------------------ batches

namespace {

// Host arrays of a concatenated batch, in the caller layout of one design.
struct Union {
  std::vector<int32_t> pin_kind, cell_type, cell_in_ptr{0}, cell_in_pin, cell_out_pin;
  std::vector<int32_t> net_driver, net_sink_ptr{0}, net_sink_pin, parent, sink_node;
  std::vector<int64_t> net_node_ptr{0};
  std::vector<float> res, cap, pi_at, pi_slew, po_rat, dang;
  std::vector<int32_t> pin_off{0};
  std::vector<int64_t> node_off{0};
  int64_t n_pins = 0, n_cells = 0, n_nets = 0, n_pi = 0, n_po = 0;
};

template <class T>
void append(std::vector<T> &dst, const T *src, size_t n, T add) {
  const size_t b = dst.size();
  dst.resize(b + n);
  for (size_t i = 0; i < n; ++i) dst[b + i] = src[i] + add;
}

sta_status prefix_design(int d, sta_status st) {
  g_err = "design " + std::to_string(d) + ": " + g_err;
  return st;
}

}  // namespace

// The union of the distinct libraries of a batch (by descriptor): their types
// one after the other, so design d's type t becomes type_off[d] + t.
struct UnionLib {
  sta_lib_desc lib{};
  std::vector<int32_t> n_inputs, sense;
  std::vector<float> pin_cap, slew_axis, load_axis, tables, po_caps;
  std::vector<int32_t> type_off;  // per design
};

static sta_status union_lib(int32_t n_designs, const sta_lib_desc *const *libs, UnionLib &U) {
  std::vector<const sta_lib_desc *> uniq;
  std::vector<int32_t> off;
  for (int d = 0; d < n_designs; ++d) {
    if (!libs[d]) return fail(STA_E_ARG, "design %d: NULL library", d);
    const auto it = std::find(uniq.begin(), uniq.end(), libs[d]);
    if (it != uniq.end()) {
      U.type_off.push_back(off[(size_t)(it - uniq.begin())]);
    } else {
      sta_status st = validate_lib(*libs[d]);
      if (st != STA_OK) return prefix_design(d, st);
      if (!uniq.empty() && (libs[d]->nx != uniq[0]->nx || libs[d]->ny != uniq[0]->ny))
        return fail(STA_E_UNSUPPORTED, "design %d: library tables of %dx%d, design 0's %dx%d", d, libs[d]->nx,
                    libs[d]->ny, uniq[0]->nx, uniq[0]->ny);
      off.push_back((int32_t)U.n_inputs.size());
      U.type_off.push_back(off.back());
      uniq.push_back(libs[d]);
      const sta_lib_desc &L = *libs[d];
      const size_t nt = (size_t)L.n_types;
      U.n_inputs.insert(U.n_inputs.end(), L.n_inputs, L.n_inputs + nt);
      U.sense.insert(U.sense.end(), L.sense, L.sense + nt);
      U.pin_cap.insert(U.pin_cap.end(), L.pin_cap_ff, L.pin_cap_ff + nt);
      U.slew_axis.insert(U.slew_axis.end(), L.slew_axis, L.slew_axis + nt * L.nx);
      U.load_axis.insert(U.load_axis.end(), L.load_axis, L.load_axis + nt * L.ny);
      U.tables.insert(U.tables.end(), L.tables, L.tables + nt * 4 * L.nx * L.ny);
    }
    U.po_caps.push_back(libs[d]->po_cap_ff);
  }
  if (U.n_inputs.size() > (size_t)kMaxTypes)
    return fail(STA_E_UNSUPPORTED, "the batch's libraries have %zu types in all (at most %d)", U.n_inputs.size(),
                kMaxTypes);
  U.lib = *uniq[0];
  U.lib.n_types = (int32_t)U.n_inputs.size();
  U.lib.n_inputs = U.n_inputs.data();
  U.lib.sense = U.sense.data();
  U.lib.pin_cap_ff = U.pin_cap.data();
  U.lib.slew_axis = U.slew_axis.data();
  U.lib.load_axis = U.load_axis.data();
  U.lib.tables = U.tables.data();
  return STA_OK;
}

static sta_status batch_create(int32_t n_designs, const sta_graph_desc *graphs, const sta_rc_desc *rcs,
                               const sta_lib_desc *const *libs, const sta_constraints *cons,
                               const sta_options *opts, sta_ctx **out) {
  sta_options o;
  sta_options_default(&o);
  if (opts) o = *opts;
  STA_TRY(check_options(o));
  if (o.mode != 0) return fail(STA_E_UNSUPPORTED, "batched contexts time hard mode (mode 0) only");
  UnionLib UL;
  STA_TRY(union_lib(n_designs, libs, UL));
  const bool one_lib = std::all_of(libs, libs + n_designs, [&](const sta_lib_desc *l) { return l == libs[0]; });
  const sta_lib_desc *lib = one_lib ? libs[0] : &UL.lib;
  auto C = std::make_unique<sta_ctx>();
  C->opt = o;
  bool dev_in = false;
  for (int d = 0; d < n_designs; ++d) dev_in |= graphs[d].mem == STA_DEVICE || rcs[d].mem == STA_DEVICE;
  if (dev_in) STA_TRY(init_device(C.get()));

  Union U;
  for (int d = 0; d < n_designs; ++d) {
    Inputs I;
    I.g = &graphs[d];
    I.rc = &rcs[d];
    I.lib = libs[d];
    I.cons = &cons[d];
    sta_status st = load_graph(I);
    if (st == STA_OK) st = validate_graph(I);
    if (st == STA_OK) st = load_validate_rc(I);
    if (st == STA_OK) st = validate_cons(cons[d], graphs[d]);
    if (st != STA_OK) return prefix_design(d, st);
    const sta_graph_desc &g = graphs[d];
    const int32_t po = (int32_t)U.n_pins;
    const int64_t no = U.node_off.back();
    if (U.n_pins + g.n_pins >= INT32_MAX || no + I.rc->n_nodes >= INT32_MAX ||
        (int64_t)U.net_sink_ptr.back() + I.net_sink_ptr[g.n_nets] >= INT32_MAX ||
        (int64_t)U.cell_in_ptr.back() + I.cell_in_ptr[g.n_cells] >= INT32_MAX)
      return fail(STA_E_UNSUPPORTED, "batch exceeds the int32 pin / sink / node limits at design %d", d);
    append(U.pin_kind, I.pin_kind.p, g.n_pins, 0);
    append(U.cell_type, I.cell_type.p, g.n_cells, one_lib ? 0 : UL.type_off[(size_t)d]);
    append(U.cell_in_ptr, I.cell_in_ptr.p + 1, g.n_cells, U.cell_in_ptr.back());
    append(U.cell_in_pin, I.cell_in_pin.p, I.cell_in_ptr[g.n_cells], po);
    append(U.cell_out_pin, I.cell_out_pin.p, g.n_cells, po);
    append(U.net_driver, I.net_driver.p, g.n_nets, po);
    append(U.net_sink_ptr, I.net_sink_ptr.p + 1, g.n_nets, U.net_sink_ptr.back());
    append(U.net_sink_pin, I.net_sink_pin.p, I.net_sink_ptr[g.n_nets], po);
    append(U.net_node_ptr, I.net_node_ptr.p + 1, g.n_nets, no);
    append(U.parent, I.parent.p, (size_t)I.rc->n_nodes, 0);
    append(U.res, I.res.p, (size_t)I.rc->n_nodes, 0.0f);
    append(U.cap, I.cap.p, (size_t)I.rc->n_nodes, 0.0f);
    append(U.sink_node, I.sink_node.p, I.net_sink_ptr[g.n_nets], 0);
    append(U.pi_at, cons[d].pi_at, 4 * (size_t)g.n_pi, 0.0f);
    append(U.pi_slew, cons[d].pi_slew, 4 * (size_t)g.n_pi, 0.0f);
    if (g.n_po > 0) append(U.po_rat, cons[d].po_rat, 4 * (size_t)g.n_po, 0.0f);
    append(U.dang, cons[d].dangling_rat, 4, 0.0f);
    U.n_pins += g.n_pins;
    U.n_cells += g.n_cells;
    U.n_nets += g.n_nets;
    U.n_pi += g.n_pi;
    U.n_po += g.n_po;
    U.pin_off.push_back((int32_t)U.n_pins);
    U.node_off.push_back(no + I.rc->n_nodes);
  }
  sta_graph_desc ug{};
  ug.n_pins = (int32_t)U.n_pins;
  ug.n_cells = (int32_t)U.n_cells;
  ug.n_nets = (int32_t)U.n_nets;
  ug.n_pi = (int32_t)U.n_pi;
  ug.n_po = (int32_t)U.n_po;
  ug.pin_kind = U.pin_kind.data();
  ug.cell_type = U.cell_type.data();
  ug.cell_in_ptr = U.cell_in_ptr.data();
  ug.cell_in_pin = U.cell_in_pin.data();
  ug.cell_out_pin = U.cell_out_pin.data();
  ug.net_driver = U.net_driver.data();
  ug.net_sink_ptr = U.net_sink_ptr.data();
  ug.net_sink_pin = U.net_sink_pin.data();
  ug.mem = STA_HOST;
  sta_rc_desc ur{};
  ur.n_nodes = U.node_off.back();
  ur.net_node_ptr = U.net_node_ptr.data();
  ur.parent = U.parent.data();
  ur.res_kohm = U.res.data();
  ur.cap_ff = U.cap.data();
  ur.sink_node = U.sink_node.data();
  ur.mem = STA_HOST;
  sta_constraints uc = cons[0];
  uc.pi_at = U.pi_at.data();
  uc.pi_slew = U.pi_slew.data();
  uc.po_rat = U.po_rat.empty() ? nullptr : U.po_rat.data();
  Inputs I;
  I.g = &ug;
  I.rc = &ur;
  I.lib = lib;
  I.cons = &uc;
  I.pin_off = &U.pin_off;
  I.dang = &U.dang;
  if (!one_lib) I.po_caps = &UL.po_caps;
  // every design passed validation; the union's derived maps are rebuilt here
  STA_TRY(load_graph(I));
  STA_TRY(validate_graph(I));
  STA_TRY(load_validate_rc(I));
  if (!dev_in) STA_TRY(init_device(C.get()));
  STA_TRY(build_context(C.get(), I));

  C->batched = true;
  C->n_designs = n_designs;
  C->pin_off = U.pin_off;
  C->node_off = U.node_off;
  C->ep_off.assign(1, 0);
  {
    size_t e = 0;
    for (int d = 0; d < n_designs; ++d) {
      while (e < C->h_ep_pin.size() && C->h_ep_pin[e] < U.pin_off[d + 1]) ++e;
      C->ep_off.push_back((int32_t)e);
    }
  }
  STA_TRY(C->upload(&C->d_ep_off, C->ep_off));
  STA_TRY(C->alloc(&C->b_partials, (size_t)n_designs * kReduceBlocks * 4));
  STA_TRY(C->alloc(&C->b_out, (size_t)n_designs * 4));
  HIP_TRY(hipMemset(C->b_out, 0, (size_t)n_designs * 4 * sizeof(double)));
  const int ne = std::max(C->n_ep, 1);
  int bits = 0;
  while ((1 << bits) < n_designs) ++bits;
  C->design_bits = bits;
  C->key_bits = 33 + bits;
  const size_t tb = sort_temp_bytes64(2 * ne, C->key_bits);
  if (tb > C->sort_bytes) {
    unsigned char *st;
    STA_TRY(C->alloc(&st, tb));
    C->sort_temp = st;
    C->sort_bytes = tb;
  }
  HIP_TRY(hipDeviceSynchronize());
  *out = C.release();
  return STA_OK;
}

extern "C" sta_status sta_batch_create(int32_t n_designs, const sta_graph_desc *graphs, const sta_rc_desc *rcs,
                                       const sta_lib_desc *lib, const sta_constraints *cons,
                                       const sta_options *opts, sta_ctx **out) {
  if (!graphs || !rcs || !lib || !cons || !out) return fail(STA_E_ARG, "NULL descriptor");
  if (n_designs < 1) return fail(STA_E_ARG, "n_designs %d < 1", n_designs);
  const std::vector<const sta_lib_desc *> libs((size_t)n_designs, lib);
  return batch_create(n_designs, graphs, rcs, libs.data(), cons, opts, out);
}

extern "C" sta_status sta_batch_create_libs(int32_t n_designs, const sta_graph_desc *graphs, const sta_rc_desc *rcs,
                                            const sta_lib_desc *const *libs, const sta_constraints *cons,
                                            const sta_options *opts, sta_ctx **out) {
  if (!graphs || !rcs || !libs || !cons || !out) return fail(STA_E_ARG, "NULL descriptor");
  if (n_designs < 1) return fail(STA_E_ARG, "n_designs %d < 1", n_designs);
  return batch_create(n_designs, graphs, rcs, libs, cons, opts, out);
}

extern "C" sta_status sta_batch_offsets(const sta_ctx *C, int32_t *n_designs, int32_t *pin_off, int32_t *ep_off,
                                        int64_t *node_off) {
  if (!C) return fail(STA_E_STATE, "NULL context");
  if (n_designs) *n_designs = C->n_designs;
  if (pin_off) std::copy(C->pin_off.begin(), C->pin_off.end(), pin_off);
  if (ep_off) std::copy(C->ep_off.begin(), C->ep_off.end(), ep_off);
  if (node_off) std::copy(C->node_off.begin(), C->node_off.end(), node_off);
  return STA_OK;
}

extern "C" void sta_destroy(sta_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  delete ctx;
}

extern "C" sta_status sta_set_wire_caps(sta_ctx *C, const float *cap_ff, sta_mem mem, void *stream) {
  if (!C) return fail(STA_E_STATE, "NULL context");
  if (!cap_ff) return fail(STA_E_ARG, "cap_ff is NULL");
  HIP_TRY(hipSetDevice(C->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (mem == STA_HOST) {
    for (int64_t k = 0; k < C->n_nodes; ++k)
      if (!finite(cap_ff[k]) || cap_ff[k] < 0.0f) return fail(STA_E_ARG, "cap_ff[%lld] invalid", (long long)k);
    float *tmp;
    sta_ctx scratch;
    STA_TRY(scratch.alloc(&tmp, C->n_nodes));
    HIP_TRY(hipMemcpyAsync(tmp, cap_ff, C->n_nodes * sizeof(float), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_permute_caps(tmp, C->node_src, C->rc_cap, C->n_nodes, C->rc_pc, C->n_small_nodes, s));
    HIP_TRY(hipStreamSynchronize(s));
  } else if (mem == STA_DEVICE) {
    HIP_TRY(launch_permute_caps(cap_ff, C->node_src, C->rc_cap, C->n_nodes, C->rc_pc, C->n_small_nodes, s));
  } else {
    return fail(STA_E_ARG, "bad mem");
  }
  return STA_OK;
}

// RC pass (or its adjoint): wide nets on the side stream, forked from and
// joined back into s around the small-net kernel, so the two overlap.
static sta_status enqueue_rc(sta_ctx *C, hipStream_t s, bool adjoint, bool res = false) {
  const DevDesign &D = C->D;
  if (C->n_big > 0) {
    HIP_TRY(hipEventRecord(C->ev_fork, s));
    HIP_TRY(hipStreamWaitEvent(C->side, C->ev_fork, 0));
    HIP_TRY(adjoint ? launch_rc_adjoint_wide(D, C->wide, C->side) : launch_rc_wide(D, C->wide, C->side));
    HIP_TRY(hipEventRecord(C->ev_join, C->side));
  }
  HIP_TRY(adjoint ? launch_rc_adjoint(D, C->rc_adj_chunks, C->n_rc_adj_chunks, res, s)
                  : launch_rc(D, C->rc_chunks, C->n_rc_chunks, s));
  if (C->n_big > 0) HIP_TRY(hipStreamWaitEvent(s, C->ev_join, 0));
  return STA_OK;
}

// WNS / TNS (and the endpoint sort keys) from the endpoint slacks.
static sta_status enqueue_reduce(sta_ctx *C, hipStream_t s) {
  const DevDesign &D = C->D;
  const bool sort = C->opt.sort_endpoints && C->n_ep > 0;
  if (C->opt.mode == 1)
    HIP_TRY(launch_reduce_smooth(D, C->partials, C->out, sort ? C->keys64 : nullptr, sort ? C->vals : nullptr, s));
  else if (C->batched)
    HIP_TRY(launch_reduce_batch(D, C->d_ep_off, C->n_designs, C->design_bits, C->b_partials, C->b_out,
                                sort ? C->keys64 : nullptr, sort ? C->vals : nullptr, s));
  else
    HIP_TRY(launch_reduce(D, C->partials, C->out, sort ? C->keys64 : nullptr, sort ? C->vals : nullptr, s));
  return STA_OK;
}

// Endpoint order per early/late from the keys the reduction wrote.
static sta_status enqueue_sort(sta_ctx *C, hipStream_t s) {
  if (!C->opt.sort_endpoints || C->n_ep <= 0) return STA_OK;
  // both orders in one sort: the early/late bit is above the (design and) slack bits
  HIP_TRY(sort_endpoints64(C->sort_temp, C->sort_bytes, C->keys64, C->keys64_out, C->vals, C->order,
                           2 * C->n_ep, C->key_bits, s));
  return STA_OK;
}

// Enqueues RC, both sweeps, the reduction and (with sort) the endpoint sort
// on s: one update.  Endpoint slacks need the arrivals only, so the reduction
// and the sort run on a second stream beside a per-level backward sweep, which
// is bound by its per-level latency; s waits for them at the end.  With prof,
// everything runs in order on s and events separate the phases.
static sta_status enqueue_update(sta_ctx *C, hipStream_t s, bool prof, bool sort) {
  const bool smooth = C->opt.mode == 1;
  if (C->opt.sched == STA_SCHED_FLOW) {  // RC, then one dataflow launch per sweep, in order on s
    C->D.rc_cons_l = 1;
    const DevDesign &D = C->D;
    if (prof) HIP_TRY(hipEventRecord(C->ev[0], s));
    STA_TRY(enqueue_rc(C, s, false));
    if (prof) HIP_TRY(hipEventRecord(C->ev[1], s));
    if (prof) HIP_TRY(hipEventRecord(C->ev[2], s));
    C->flow_fwd.epoch = C->flow_bwd.epoch = ++C->flow_epoch;
    HIP_TRY(launch_flow(D, C->flow_fwd, true, C->flow_grid, s));
    if (prof) HIP_TRY(hipEventRecord(C->ev[3], s));
    if (!smooth) HIP_TRY(launch_flow(D, C->flow_bwd, false, C->flow_grid, s));
    if (prof) HIP_TRY(hipEventRecord(C->ev[4], s));
    STA_TRY(enqueue_reduce(C, s));
    if (prof) HIP_TRY(hipEventRecord(C->ev[5], s));
    if (sort) STA_TRY(enqueue_sort(C, s));
    return STA_OK;
  }
  const bool per_level = C->opt.sched != STA_SCHED_PERSISTENT;
  // the per-level backward writes each driver's whole consumer record, so the
  // RC pass leaves its load field alone there
  C->D.rc_cons_l = per_level && !smooth ? 0 : 1;
  const DevDesign &D = C->D;
  // (not beside a persistent sweep: its blocks wait for each other, and no
  // other kernel should hold the slots they are waiting to occupy)
  const bool beside = !smooth && !prof && per_level && C->opt.overlap;
  // RC in level groups on side2 (wide nets on side) while the per-level
  // forward sweep runs: a level waits only for the groups up to its own
  const bool grouped = per_level && !prof && C->opt.overlap;
  if (prof) HIP_TRY(hipEventRecord(C->ev[0], s));
  if (grouped) {
    HIP_TRY(hipEventRecord(C->ev_fork, s));
    if (C->n_big > 0) {
      HIP_TRY(hipStreamWaitEvent(C->side, C->ev_fork, 0));
      HIP_TRY(launch_rc_wide(D, C->wide, C->side));
      HIP_TRY(hipEventRecord(C->ev_join, C->side));
    }
    HIP_TRY(hipStreamWaitEvent(C->side2, C->ev_fork, 0));
    int prev = 0;
    for (size_t g = 0; g < C->rc_grp_end.size(); ++g) {
      const int end = C->rc_grp_end[g];
      if (end > prev || g == 0) HIP_TRY(launch_rc(D, C->rc_chunks + prev, end - prev, C->side2, nullptr, g == 0));
      prev = end;
      HIP_TRY(hipEventRecord(C->ev_rc[g], C->side2));
    }
  } else {
    STA_TRY(enqueue_rc(C, s, false));
  }
  if (prof) HIP_TRY(hipEventRecord(C->ev[1], s));
  if (prof) HIP_TRY(hipEventRecord(C->ev[2], s));
  if (!per_level) {
    HIP_TRY(launch_forward(D, C->sweep_grid, C->coop, s));
  } else {
    size_t g = 0;
    bool wide_done = !grouped || C->n_big == 0;
    for (const int4 &ph : C->ph_fwd) {
      for (; grouped && g < C->rc_grp_lvl.size() && C->rc_grp_lvl[g] <= ph.w; ++g)
        HIP_TRY(hipStreamWaitEvent(s, C->ev_rc[g], 0));
      if (!wide_done && ph.w >= C->wide_lvl) {
        HIP_TRY(hipStreamWaitEvent(s, C->ev_join, 0));
        wide_done = true;
      }
      HIP_TRY(launch_forward_phase(D, ph, C->lvl_reg[ph.w], s));
    }
    for (; grouped && g < C->rc_grp_lvl.size(); ++g) HIP_TRY(hipStreamWaitEvent(s, C->ev_rc[g], 0));
    if (!wide_done) HIP_TRY(hipStreamWaitEvent(s, C->ev_join, 0));
  }
  if (prof) HIP_TRY(hipEventRecord(C->ev[3], s));
  if (beside) {
    HIP_TRY(hipEventRecord(C->ev_fwd, s));
    HIP_TRY(hipStreamWaitEvent(C->side2, C->ev_fwd, 0));
    STA_TRY(enqueue_reduce(C, C->side2));
    if (sort) STA_TRY(enqueue_sort(C, C->side2));
    HIP_TRY(hipEventRecord(C->ev_red, C->side2));
  }
  if (!smooth) {  // the smooth objective needs arrivals only; it skips the RAT sweep
    if (!per_level) {
      HIP_TRY(launch_backward(D, C->sweep_grid, C->coop, s));
    } else {
      for (const int4 &ph : C->ph_bwd) HIP_TRY(launch_backward_phase(D, ph, C->lvl_reg[ph.w], s));
    }
  }
  if (prof) HIP_TRY(hipEventRecord(C->ev[4], s));
  if (beside) {
    HIP_TRY(hipStreamWaitEvent(s, C->ev_red, 0));
  } else {
    STA_TRY(enqueue_reduce(C, s));
  }
  if (prof) HIP_TRY(hipEventRecord(C->ev[5], s));
  if (sort && !beside) STA_TRY(enqueue_sort(C, s));
  return STA_OK;
}

// Graph schedule: the per-level launch sequence of one update is captured once
// and replayed; it holds kernel nodes only (counters are cleared by a kernel,
// never by a memset node).
static sta_status ensure_graph(sta_ctx *C) {
  if (C->graph_exec && C->graph_overlap != C->opt.overlap) {  // captured with the other stream layout
    (void)hipGraphExecDestroy(C->graph_exec);
    (void)hipGraphDestroy(C->graph);
    C->graph_exec = nullptr;
    C->graph = nullptr;
  }
  if (C->graph_exec) return STA_OK;
  C->graph_overlap = C->opt.overlap;
  if (!C->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&C->cap_stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(C->cap_stream, hipStreamCaptureModeThreadLocal));
  sta_status st = enqueue_update(C, C->cap_stream, false, false);  // the sort stays outside the graph
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(C->cap_stream, &g);
  if (st != STA_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  C->graph = g;
  HIP_TRY(hipGraphInstantiate(&C->graph_exec, g, nullptr, nullptr, 0));
  return STA_OK;
}

extern "C" sta_status sta_update_timing(sta_ctx *C, void *stream) {
  if (!C) return fail(STA_E_STATE, "NULL context");
  HIP_TRY(hipSetDevice(C->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool prof = C->opt.profile != 0;
  if (C->opt.sched == STA_SCHED_GRAPH) {
    STA_TRY(ensure_graph(C));
    if (prof) {
      for (int i = 0; i < 5; ++i) HIP_TRY(hipEventRecord(C->ev[i], s));  // phases not separable in a graph
    }
    HIP_TRY(hipGraphLaunch(C->graph_exec, s));
    if (prof) HIP_TRY(hipEventRecord(C->ev[5], s));
    STA_TRY(enqueue_sort(C, s));
  } else {
    STA_TRY(enqueue_update(C, s, prof, true));
  }
  if (prof) HIP_TRY(hipEventRecord(C->ev[6], s));
  C->timed = prof;
  C->last_stream = s;
  C->updated = true;
  return STA_OK;
}

// The phase where a queued incremental sweep stopped (waits for it).
// Incremental updates of more than kIncMinFull nets and more than one net in
// kIncFullShare run as full updates
// (10M-pin design: 100 nets took 0.87 and 10,000 nets 1.01 of a full update).
constexpr int64_t kIncFullShare = 1024;
constexpr int32_t kIncMinFull = 256;  // (and of more than this many nets)

static sta_status read_stop(sta_ctx *C, int which, int *stop, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(C->inc_stop + which, C->inc.stop + which, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *stop = C->inc_stop[which];
  return STA_OK;
}

// Device queues and staging of the incremental update, made on first use.
static sta_status inc_prepare(sta_ctx *C) {
  if (C->inc_ready) return STA_OK;
  const int n_ph = (int)(C->ph_fwd.size() + C->ph_bwd.size());
  const int64_t n_big = std::max(C->n_big, 1);
  const int64_t words =
      2 * (int64_t)C->n_chunks + n_ph + ((int64_t)C->n_drv + 3) / 4 + 2 + C->n_rc_chunks + n_big;
  if (words >= INT32_MAX) return fail(STA_E_UNSUPPORTED, "design too large for the incremental queues");
  STA_TRY(C->alloc(&C->inc_buf, (size_t)words));
  C->inc_words = (int)words;
  IncArgs &I = C->inc;
  I.flag = C->inc_buf;
  I.cnt = I.flag + 2 * (size_t)C->n_chunks;
  I.rcd = reinterpret_cast<uint8_t *>(I.cnt + n_ph);
  I.stop = reinterpret_cast<int32_t *>(C->inc_buf + words - 2 - C->n_rc_chunks - n_big);
  I.rc_flag = C->inc_buf + words - C->n_rc_chunks - n_big;
  I.wide_flag = I.rc_flag + C->n_rc_chunks;
  I.net_slot = C->net_slot;
  I.slot_rc = C->inc_slot_rc;
  STA_TRY(C->alloc(&I.wl_c, 2 * (size_t)C->n_chunks));
  STA_TRY(C->alloc(&I.wl_p, 2 * (size_t)std::max(C->n_pieces, 1)));
  I.chunk_of = C->inc_chunk_of;
  I.chunk_ph = C->inc_chunk_ph;
  int32_t *scc;
  int4 *fcc = nullptr;
  STA_TRY(C->alloc(&scc, (size_t)std::max(C->n_sinks, 1)));
  if (C->D.fanin4) STA_TRY(C->alloc(&fcc, (size_t)C->n_drv));
  HIP_TRY(launch_inc_maps(C->D, C->inc_chunk_of, scc, fcc, nullptr));
  HIP_TRY(hipDeviceSynchronize());
  I.sink_cc = scc;
  I.fanin_cc = fcc;
  I.n_chunks = C->n_chunks;
  I.n_pieces = C->n_pieces;
  HIP_TRY(hipEventCreateWithFlags(&C->inc_ev, hipEventDisableTiming));
  HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&C->inc_stop), 2 * sizeof(int32_t), hipHostMallocDefault));
  // queued sweeps: few blocks (the per-phase wait is cheaper with fewer
  // pollers, and a small cone has little work per phase), within the
  // cooperative limit; sweep_blocks overrides.  They hand over to per-phase
  // launches at the first phase with more than kIncMaxItems items: a non-empty
  // phase costs about as much either way, an empty one far less queued.
  const int per_cu = inc_blocks_per_cu(sweep_lds_bytes(C->D));
  const int cap = per_cu * std::max(C->n_cu, 1);
  C->inc_grid = !C->coop ? 0 : C->opt.sweep_blocks > 0 ? std::min(C->opt.sweep_blocks, cap) : std::min(kIncBlocks, cap);
  C->inc_max_items = kIncMaxItems;
  C->inc_ready = true;
  return STA_OK;
}

extern "C" sta_status sta_update_timing_incremental(sta_ctx *C, const int32_t *nets, int32_t n_nets, sta_mem mem,
                                                    void *stream) {
  if (!C) return fail(STA_E_STATE, "NULL context");
  if (n_nets < 0) return fail(STA_E_ARG, "n_nets < 0");
  if (n_nets > 0 && !nets) return fail(STA_E_ARG, "nets is NULL");
  if (mem != STA_HOST && mem != STA_DEVICE) return fail(STA_E_ARG, "bad mem");
  if (C->batched) return fail(STA_E_UNSUPPORTED, "incremental update of a batched context");
  if (!C->updated) return fail(STA_E_STATE, "incremental update before a full sta_update_timing");
  HIP_TRY(hipSetDevice(C->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  STA_TRY(inc_prepare(C));
  HIP_TRY(hipEventSynchronize(C->inc_ev));  // the staging buffer's previous upload has been read
  if (n_nets > C->inc_cap) {  // grows geometrically; the old device buffer stays with the context
    const int cap = std::max(n_nets, 2 * C->inc_cap);
    if (C->inc_host) HIP_TRY(hipHostFree(C->inc_host));
    C->inc_host = nullptr;
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&C->inc_host), (size_t)cap * sizeof(int32_t),
                          hipHostMallocDefault));
    STA_TRY(C->alloc(&C->inc_nets, (size_t)cap));
    C->inc_cap = cap;
  }
  // ids are checked on the host (a device list is read back first); the
  // device then takes the list as it is (a device list in place)
  const int32_t *h = nets;
  if (mem == STA_DEVICE && n_nets > 0) {
    HIP_TRY(hipMemcpyAsync(C->inc_host, nets, (size_t)n_nets * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    h = C->inc_host;
  }
  for (int32_t i = 0; i < n_nets; ++i)
    if (h[i] < 0 || h[i] >= C->n_nets) return fail(STA_E_ARG, "nets[%d] = %d out of range", i, h[i]);
  // Beyond about one net in kIncFullShare the cones cover most of the design
  // and a full update is cheaper than walking them (the results are the same
  // bits either way; the list needs no device copy then).
  if (n_nets > kIncMinFull && (int64_t)n_nets * kIncFullShare > (int64_t)C->n_nets) return sta_update_timing(C, stream);
  const int32_t *d_nets = nets;
  if (mem == STA_HOST && n_nets > 0) {
    std::memcpy(C->inc_host, nets, (size_t)n_nets * sizeof(int32_t));
    HIP_TRY(hipMemcpyAsync(C->inc_nets, C->inc_host, (size_t)n_nets * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(C->inc_ev, s));
    d_nets = C->inc_nets;
  }
  C->D.rc_cons_l = 1;  // the incremental backward reads consumer records, whose loads it does not write
  const DevDesign &D = C->D;
  HIP_TRY(launch_reset_counters(C->inc_buf, C->inc_words, s));
  HIP_TRY(launch_reset_counters(D.counters, n_counters(D.n_ph_fwd + D.n_ph_bwd), s));
  HIP_TRY(launch_inc_seed(D, C->inc, d_nets, n_nets, s));
  // the RC chunks and wide nets holding a listed net (the others return at once)
  if (C->n_rc_chunks > 0) HIP_TRY(launch_rc(D, C->rc_chunks, C->n_rc_chunks, s, C->inc.rc_flag));
  if (C->n_big > 0) HIP_TRY(launch_rc_wide(D, C->wide, s, C->inc.wide_flag));
  // queued forward sweep while the cone is small, then per-phase launches
  int stop = 0;
  if (C->inc_grid > 0) {
    HIP_TRY(launch_inc_queues(D, C->inc, false, s));
    HIP_TRY(launch_inc_forward(D, C->inc, C->inc_grid, C->inc_max_items, s));
    STA_TRY(read_stop(C, 0, &stop, s));
  }
  for (int k = stop; k < (int)C->ph_fwd.size(); ++k)
    HIP_TRY(launch_inc_forward_phase(D, C->inc, C->ph_fwd[k], C->lvl_reg[C->ph_fwd[k].w], s));
  if (C->opt.mode != 1) {
    stop = 0;
    if (C->inc_grid > 0) {
      HIP_TRY(launch_inc_queues(D, C->inc, true, s));
      HIP_TRY(launch_inc_backward(D, C->inc, C->inc_grid, C->inc_max_items, s));
      STA_TRY(read_stop(C, 1, &stop, s));
    }
    for (int k = stop; k < (int)C->ph_bwd.size(); ++k) HIP_TRY(launch_inc_backward_phase(D, C->inc, C->ph_bwd[k], s));
  }
  STA_TRY(enqueue_reduce(C, s));
  STA_TRY(enqueue_sort(C, s));
  C->timed = false;
  C->last_stream = s;
  return STA_OK;
}

namespace {
// Device buffers of a call that has no context, freed when it returns.
struct CallScratch {
  std::vector<std::unique_ptr<DevMem>> mem;
  template <typename T>
  sta_status alloc(T **out_p, size_t n) {
    auto m = std::make_unique<DevMem>();
    hipError_t e = hipMalloc(&m->p, std::max<size_t>(n, 1) * sizeof(T));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    *out_p = static_cast<T *>(m->p);
    mem.push_back(std::move(m));
    return STA_OK;
  }
};
}  // namespace

// RC trees from pin positions (no context; see sta.h).  Host inputs go up to
// scratch buffers, every input is checked by one device pass whose result the
// host reads before the estimation kernels start, host outputs come back.
extern "C" sta_status sta_estimate_rc(const sta_graph_desc *g, const float *pin_x, const float *pin_y,
                                      const sta_wire_params *w, int64_t *net_node_ptr, int32_t *parent,
                                      float *res_kohm, float *cap_ff, int32_t *sink_node, sta_mem mem,
                                      void *stream) {
  if (!g || !w) return fail(STA_E_ARG, "NULL graph or wire parameters");
  if (mem != STA_HOST && mem != STA_DEVICE) return fail(STA_E_ARG, "bad mem");
  if (g->mem != STA_HOST && g->mem != STA_DEVICE) return fail(STA_E_ARG, "bad graph mem");
  if (g->n_nets < 0 || g->n_pins < 0) return fail(STA_E_ARG, "negative sizes");
  for (float v : {w->r_x, w->r_y, w->c_x, w->c_y})
    if (!std::isfinite(v) || v < 0.0f) return fail(STA_E_ARG, "wire parameters must be finite and >= 0");
  const int NN = g->n_nets, NP = g->n_pins;
  if (!net_node_ptr || !g->net_sink_ptr || (NN > 0 && !g->net_driver) || (NP > 0 && (!pin_x || !pin_y)))
    return fail(STA_E_ARG, "NULL array");
  hipStream_t s = static_cast<hipStream_t>(stream);
  CallScratch tmp;  // freed on return, after the final synchronization or an error
  int32_t n_sinks = 0;
  if (g->mem == STA_HOST) {
    n_sinks = g->net_sink_ptr[NN];
  } else {
    HIP_TRY(hipMemcpyAsync(&n_sinks, g->net_sink_ptr + NN, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  if (n_sinks < 0) return fail(STA_E_ARG, "net_sink_ptr[n_nets] < 0");
  if (n_sinks > 0 && !g->net_sink_pin) return fail(STA_E_ARG, "NULL net_sink_pin");
  const int64_t n_nodes = (int64_t)NN + 3 * (int64_t)n_sinks;
  if (n_nodes > 0 && (!parent || !res_kohm || !cap_ff)) return fail(STA_E_ARG, "NULL RC output array");
  if (n_sinks > 0 && !sink_node) return fail(STA_E_ARG, "NULL sink_node");
  EstArgs A{};
  A.n_nets = NN;
  A.rx = w->r_x;
  A.ry = w->r_y;
  A.cx = w->c_x;
  A.cy = w->c_y;
  auto up = [&](auto **dst, const auto *src, size_t n) -> sta_status {
    STA_TRY(tmp.alloc(dst, std::max<size_t>(n, 1)));
    if (n > 0) HIP_TRY(hipMemcpyAsync(*dst, src, n * sizeof(*src), hipMemcpyHostToDevice, s));
    return STA_OK;
  };
  if (g->mem == STA_HOST) {
    int32_t *d_drv, *d_nsp, *d_pin;
    STA_TRY(up(&d_drv, g->net_driver, (size_t)NN));
    STA_TRY(up(&d_nsp, g->net_sink_ptr, (size_t)NN + 1));
    STA_TRY(up(&d_pin, g->net_sink_pin, (size_t)n_sinks));
    A.driver = d_drv;
    A.sink_ptr = d_nsp;
    A.sink_pin = d_pin;
  } else {
    A.driver = g->net_driver;
    A.sink_ptr = g->net_sink_ptr;
    A.sink_pin = g->net_sink_pin;
  }
  if (mem == STA_HOST) {
    float *dx, *dy;
    STA_TRY(up(&dx, pin_x, (size_t)NP));
    STA_TRY(up(&dy, pin_y, (size_t)NP));
    A.x = dx;
    A.y = dy;
    STA_TRY(tmp.alloc(&A.node_ptr, (size_t)NN + 1));
    STA_TRY(tmp.alloc(&A.parent, (size_t)std::max<int64_t>(n_nodes, 1)));
    STA_TRY(tmp.alloc(&A.res, (size_t)std::max<int64_t>(n_nodes, 1)));
    STA_TRY(tmp.alloc(&A.cap, (size_t)std::max<int64_t>(n_nodes, 1)));
    STA_TRY(tmp.alloc(&A.sink_node, (size_t)std::max(n_sinks, 1)));
  } else {
    A.x = pin_x;
    A.y = pin_y;
    A.node_ptr = net_node_ptr;
    A.parent = parent;
    A.res = res_kohm;
    A.cap = cap_ff;
    A.sink_node = sink_node;
  }
  int32_t *mid, *big;
  uint32_t *st;
  STA_TRY(tmp.alloc(&mid, (size_t)NN));
  STA_TRY(tmp.alloc(&big, (size_t)NN));
  STA_TRY(tmp.alloc(&st, 6));
  const uint32_t st0[6] = {0u, 0u, 0u, ~0u, ~0u, ~0u};
  HIP_TRY(hipMemcpyAsync(st, st0, sizeof st0, hipMemcpyHostToDevice, s));
  HIP_TRY(launch_est_check(A, NP, n_sinks, mid, big, st, s));
  uint32_t h[6];
  HIP_TRY(hipMemcpyAsync(h, st, sizeof h, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h[3] != ~0u) return fail(STA_E_ARG, "net %u: bad net_sink_ptr or net_driver", h[3]);
  if (h[4] != ~0u) return fail(STA_E_ARG, "net_sink_pin[%u] out of range", h[4]);
  if (h[5] != ~0u) return fail(STA_E_ARG, "pin %u: position not finite or beyond 1e18 in magnitude", h[5]);
  if (h[1] > 0 && (int64_t)h[2] + 1 > kEstMaxPins)
    return fail(STA_E_UNSUPPORTED, "a net has %u sinks (at most %d)", h[2], kEstMaxPins - 1);
  if (NN == 0) {
    const int64_t zero = 0;
    HIP_TRY(hipMemcpyAsync(A.node_ptr, &zero, sizeof zero, hipMemcpyHostToDevice, s));
  }
  // the large nets' per-pin scratch
  unsigned long long tot = 0;
  int64_t *off;
  unsigned long long *total;
  STA_TRY(tmp.alloc(&off, (size_t)std::max(NN, 1)));
  STA_TRY(tmp.alloc(&total, 1));
  if (h[1] > 0) {
    HIP_TRY(launch_est_acc_offsets(A, big, st, off, total, s));
    HIP_TRY(hipMemcpyAsync(&tot, total, sizeof tot, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  STA_TRY(tmp.alloc(&A.big_tmp, (size_t)std::max<unsigned long long>(16 * tot, 1)));
  A.acc_off = off;
  STA_TRY(est_forked(s, [&](hipStream_t side) { return launch_est(A, mid, big, st, h[0], h[1], s, side); }));
  if (mem == STA_HOST) {
    HIP_TRY(hipMemcpyAsync(net_node_ptr, A.node_ptr, ((size_t)NN + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (n_nodes > 0) {
      HIP_TRY(hipMemcpyAsync(parent, A.parent, n_nodes * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(res_kohm, A.res, n_nodes * sizeof(float), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(cap_ff, A.cap, n_nodes * sizeof(float), hipMemcpyDeviceToHost, s));
    }
    if (n_sinks > 0)
      HIP_TRY(hipMemcpyAsync(sink_node, A.sink_node, n_sinks * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  return STA_OK;
}

// Copy bandwidth of a plain vector copy kernel (see sta.h).
extern "C" sta_status sta_measure_copy(const void *src, void *dst, int64_t bytes, int32_t reps, void *stream,
                                       float *ms) {
  if (!src || !dst || !ms) return fail(STA_E_ARG, "NULL argument");
  if (bytes <= 0 || bytes % 16 != 0) return fail(STA_E_ARG, "bytes must be a positive multiple of 16");
  if (reps < 1) return fail(STA_E_ARG, "reps %d < 1", reps);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e, "hipEventCreate");
  }
  e = launch_copy4(src, dst, bytes / 16, s);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch_copy4(src, dst, bytes / 16, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "copy timing");
  *ms = t / (float)reps;
  return STA_OK;
}

// Latency floor of a level-synchronous sweep (see sta.h).
extern "C" sta_status sta_measure_level_floor(int32_t levels, int32_t items, int64_t records, int32_t reps,
                                              void *stream, float *ms) {
  if (!ms) return fail(STA_E_ARG, "NULL ms");
  if (levels < 1 || items < 1 || reps < 1 || records < items || records > INT32_MAX)
    return fail(STA_E_ARG, "bad sizes (levels %d, items %d, records %lld, reps %d)", levels, items,
                (long long)records, reps);
  hipStream_t s = static_cast<hipStream_t>(stream);
  CallScratch tmp;
  int32_t *idx;
  PinState *src, *dst;
  STA_TRY(tmp.alloc(&idx, (size_t)records));
  STA_TRY(tmp.alloc(&src, (size_t)records));
  STA_TRY(tmp.alloc(&dst, (size_t)records));
  {  // a fixed pseudo-random permutation-free index: SplitMix64 draws
    std::vector<int32_t> h((size_t)records);
    uint64_t z = 0x9e3779b97f4a7c15ull;
    for (int64_t i = 0; i < records; ++i) {
      uint64_t x = (z += 0x9e3779b97f4a7c15ull);
      x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
      x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
      x ^= x >> 31;
      h[(size_t)i] = (int32_t)(x % (uint64_t)records);
    }
    HIP_TRY(hipMemcpy(idx, h.data(), h.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(src, 0, (size_t)records * sizeof(PinState)));
  }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e, "hipEventCreate");
  }
  const int64_t span = records - items;
  auto sweep = [&]() {
    hipError_t r = hipSuccess;
    for (int l = 0; l < levels && r == hipSuccess; ++l)
      r = launch_level_floor(idx, src, dst, items, (int)(span > 0 ? ((int64_t)l * items) % span : 0), s);
    return r;
  };
  e = sweep();  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int i = 0; i < reps && e == hipSuccess; ++i) e = sweep();
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "level floor timing");
  *ms = t / (float)reps;
  return STA_OK;
}

// The same trees with no allocation (see sta.h): every array in device memory,
// the check words and net lists in the library's fixed device scratch.
extern "C" sta_status sta_estimate_rc_noalloc(const sta_graph_desc *g, const float *pin_x, const float *pin_y,
                                              const sta_wire_params *w, int64_t *net_node_ptr, int32_t *parent,
                                              float *res_kohm, float *cap_ff, int32_t *sink_node, void *stream) {
  if (!g || !w) return fail(STA_E_ARG, "NULL graph or wire parameters");
  if (g->mem != STA_DEVICE) return fail(STA_E_ARG, "the allocation-free estimator takes the net CSR in device memory");
  if (g->n_nets < 0 || g->n_pins < 0) return fail(STA_E_ARG, "negative sizes");
  for (float v : {w->r_x, w->r_y, w->c_x, w->c_y})
    if (!std::isfinite(v) || v < 0.0f) return fail(STA_E_ARG, "wire parameters must be finite and >= 0");
  const int NN = g->n_nets, NP = g->n_pins;
  if (!net_node_ptr || !g->net_sink_ptr || (NN > 0 && !g->net_driver) || (NP > 0 && (!pin_x || !pin_y)))
    return fail(STA_E_ARG, "NULL array");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  unsigned char *scr = nullptr;
  HIP_TRY(est_noalloc_scratch(dev, &scr));
  int32_t n_sinks = 0;
  HIP_TRY(hipMemcpyAsync(&n_sinks, g->net_sink_ptr + NN, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (n_sinks < 0) return fail(STA_E_ARG, "net_sink_ptr[n_nets] < 0");
  if (n_sinks > 0 && !g->net_sink_pin) return fail(STA_E_ARG, "NULL net_sink_pin");
  const int64_t n_nodes = (int64_t)NN + 3 * (int64_t)n_sinks;
  if (n_nodes > 0 && (!parent || !res_kohm || !cap_ff)) return fail(STA_E_ARG, "NULL RC output array");
  if (n_sinks > 0 && !sink_node) return fail(STA_E_ARG, "NULL sink_node");
  EstArgs A{};
  A.n_nets = NN;
  A.rx = w->r_x;
  A.ry = w->r_y;
  A.cx = w->c_x;
  A.cy = w->c_y;
  A.driver = g->net_driver;
  A.sink_ptr = g->net_sink_ptr;
  A.sink_pin = g->net_sink_pin;
  A.x = pin_x;
  A.y = pin_y;
  A.node_ptr = net_node_ptr;
  A.parent = parent;
  A.res = res_kohm;
  A.cap = cap_ff;
  A.sink_node = sink_node;
  uint32_t *st = reinterpret_cast<uint32_t *>(scr);
  int32_t *mid = reinterpret_cast<int32_t *>(scr + 256);
  int32_t *big = mid + kEstNoallocMid;
  const uint32_t st0[6] = {0u, 0u, 0u, ~0u, ~0u, ~0u};  // the last call's words are overwritten
  HIP_TRY(hipMemcpyAsync(st, st0, sizeof st0, hipMemcpyHostToDevice, s));
  HIP_TRY(launch_est_check(A, NP, n_sinks, mid, big, st, s, kEstNoallocMid, kEstNoallocBig));
  uint32_t h[6];
  HIP_TRY(hipMemcpyAsync(h, st, sizeof h, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h[3] != ~0u) return fail(STA_E_ARG, "net %u: bad net_sink_ptr or net_driver", h[3]);
  if (h[4] != ~0u) return fail(STA_E_ARG, "net_sink_pin[%u] out of range", h[4]);
  if (h[5] != ~0u) return fail(STA_E_ARG, "pin %u: position not finite or beyond 1e18 in magnitude", h[5]);
  if (h[1] > 0 && (int64_t)h[2] + 1 > kEstMaxPins)
    return fail(STA_E_UNSUPPORTED, "a net has %u sinks (at most %d)", h[2], kEstMaxPins - 1);
  if (h[0] > kEstNoallocMid || h[1] > kEstNoallocBig)
    return fail(STA_E_UNSUPPORTED,
                "%u nets of 9-64 pins and %u of more than 64 pins exceed the fixed scratch (at most %u and %u)", h[0],
                h[1], kEstNoallocMid, kEstNoallocBig);
  int64_t *off = reinterpret_cast<int64_t *>(big + kEstNoallocBig);
  uint32_t *big_tmp = reinterpret_cast<uint32_t *>(off + kEstNoallocBig);
  uint64_t tot = 0;
  if (h[1] > 0) {  // the big nets' pin total, into the check words' spare slots
    unsigned long long *total = reinterpret_cast<unsigned long long *>(scr + 64);
    HIP_TRY(launch_est_acc_offsets(A, big, st, off, total, s));
    HIP_TRY(hipMemcpyAsync(&tot, total, sizeof tot, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  if (tot > kEstNoallocBigPins)
    return fail(STA_E_UNSUPPORTED, "the nets of more than 64 pins hold %llu pins, beyond the fixed scratch (%u)",
                (unsigned long long)tot, kEstNoallocBigPins);
  A.big_tmp = big_tmp;
  A.acc_off = off;
  if (NN == 0) {
    const int64_t zero = 0;
    HIP_TRY(hipMemcpyAsync(A.node_ptr, &zero, sizeof zero, hipMemcpyHostToDevice, s));
  }
  HIP_TRY(launch_est(A, mid, big, st, h[0], h[1], s));
  HIP_TRY(hipStreamSynchronize(s));
  return STA_OK;
}

// Gradient to pin positions through estimated trees (no context; see sta.h).
extern "C" sta_status sta_estimate_rc_backward(const sta_graph_desc *g, const float *pin_x, const float *pin_y,
                                               const sta_wire_params *w, const int32_t *parent,
                                               const int32_t *sink_node, const float *grad_res,
                                               const float *grad_cap, float *grad_x, float *grad_y, sta_mem mem,
                                               void *stream) {
  if (!g || !w) return fail(STA_E_ARG, "NULL graph or wire parameters");
  if (mem != STA_HOST && mem != STA_DEVICE) return fail(STA_E_ARG, "bad mem");
  if (g->mem != STA_HOST && g->mem != STA_DEVICE) return fail(STA_E_ARG, "bad graph mem");
  if (g->n_nets < 0 || g->n_pins < 0) return fail(STA_E_ARG, "negative sizes");
  for (float v : {w->r_x, w->r_y, w->c_x, w->c_y})
    if (!std::isfinite(v) || v < 0.0f) return fail(STA_E_ARG, "wire parameters must be finite and >= 0");
  const int NN = g->n_nets, NP = g->n_pins;
  if (!g->net_sink_ptr || (NN > 0 && !g->net_driver) || (NP > 0 && (!pin_x || !pin_y || !grad_x || !grad_y)))
    return fail(STA_E_ARG, "NULL array");
  hipStream_t s = static_cast<hipStream_t>(stream);
  CallScratch tmp;
  int32_t n_sinks = 0;
  if (g->mem == STA_HOST) {
    n_sinks = g->net_sink_ptr[NN];
  } else {
    HIP_TRY(hipMemcpyAsync(&n_sinks, g->net_sink_ptr + NN, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  if (n_sinks < 0) return fail(STA_E_ARG, "net_sink_ptr[n_nets] < 0");
  if (n_sinks > 0 && (!g->net_sink_pin || !sink_node)) return fail(STA_E_ARG, "NULL sink array");
  const int64_t n_nodes = (int64_t)NN + 3 * (int64_t)n_sinks;
  if (n_nodes > 0 && (!parent || !grad_res || !grad_cap)) return fail(STA_E_ARG, "NULL node array");
  auto up = [&](auto **dst, const auto *src, size_t n) -> sta_status {
    STA_TRY(tmp.alloc(dst, std::max<size_t>(n, 1)));
    if (n > 0) HIP_TRY(hipMemcpyAsync(*dst, src, n * sizeof(*src), hipMemcpyHostToDevice, s));
    return STA_OK;
  };
  EstArgs A{};
  A.n_nets = NN;
  A.rx = w->r_x;
  A.ry = w->r_y;
  A.cx = w->c_x;
  A.cy = w->c_y;
  if (g->mem == STA_HOST) {
    int32_t *d_drv, *d_nsp, *d_pin;
    STA_TRY(up(&d_drv, g->net_driver, (size_t)NN));
    STA_TRY(up(&d_nsp, g->net_sink_ptr, (size_t)NN + 1));
    STA_TRY(up(&d_pin, g->net_sink_pin, (size_t)n_sinks));
    A.driver = d_drv;
    A.sink_ptr = d_nsp;
    A.sink_pin = d_pin;
  } else {
    A.driver = g->net_driver;
    A.sink_ptr = g->net_sink_ptr;
    A.sink_pin = g->net_sink_pin;
  }
  if (mem == STA_HOST) {
    float *dx, *dy, *gr, *gc, *ox, *oy;
    int32_t *par, *snode;
    STA_TRY(up(&dx, pin_x, (size_t)NP));
    STA_TRY(up(&dy, pin_y, (size_t)NP));
    STA_TRY(up(&par, parent, (size_t)n_nodes));
    STA_TRY(up(&snode, sink_node, (size_t)n_sinks));
    STA_TRY(up(&gr, grad_res, (size_t)n_nodes));
    STA_TRY(up(&gc, grad_cap, (size_t)n_nodes));
    STA_TRY(tmp.alloc(&ox, (size_t)std::max(NP, 1)));
    STA_TRY(tmp.alloc(&oy, (size_t)std::max(NP, 1)));
    A.x = dx;
    A.y = dy;
    A.g_parent = par;
    A.g_sink_node = snode;
    A.g_res = gr;
    A.g_cap = gc;
    A.gx = ox;
    A.gy = oy;
  } else {
    A.x = pin_x;
    A.y = pin_y;
    A.g_parent = parent;
    A.g_sink_node = sink_node;
    A.g_res = grad_res;
    A.g_cap = grad_cap;
    A.gx = grad_x;
    A.gy = grad_y;
  }
  if (NP > 0) {
    HIP_TRY(hipMemsetAsync(A.gx, 0, NP * sizeof(float), s));
    HIP_TRY(hipMemsetAsync(A.gy, 0, NP * sizeof(float), s));
  }
  // checks of the net CSR and positions, as for the estimation
  int32_t *mid, *big;
  int64_t *off;
  uint32_t *st;
  unsigned long long *total;
  STA_TRY(tmp.alloc(&mid, (size_t)NN));
  STA_TRY(tmp.alloc(&big, (size_t)NN));
  STA_TRY(tmp.alloc(&off, (size_t)std::max(NN, 1)));
  STA_TRY(tmp.alloc(&st, 7));
  STA_TRY(tmp.alloc(&total, 1));
  STA_TRY(tmp.alloc(&A.step_src, (size_t)std::max(n_sinks, 1)));
  const uint32_t st0[7] = {0u, 0u, 0u, ~0u, ~0u, ~0u, ~0u};
  HIP_TRY(hipMemcpyAsync(st, st0, sizeof st0, hipMemcpyHostToDevice, s));
  HIP_TRY(launch_est_check(A, NP, n_sinks, mid, big, st, s));
  uint32_t h[7];
  HIP_TRY(hipMemcpyAsync(h, st, 6 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h[3] != ~0u) return fail(STA_E_ARG, "net %u: bad net_sink_ptr or net_driver", h[3]);
  if (h[4] != ~0u) return fail(STA_E_ARG, "net_sink_pin[%u] out of range", h[4]);
  if (h[5] != ~0u) return fail(STA_E_ARG, "pin %u: position not finite or beyond 1e18 in magnitude", h[5]);
  if (h[1] > 0 && (int64_t)h[2] + 1 > kEstMaxPins)
    return fail(STA_E_UNSUPPORTED, "a net has %u sinks (at most %d)", h[2], kEstMaxPins - 1);
  // the large nets' integer accumulators
  unsigned long long tot = 0;
  if (h[1] > 0) {
    HIP_TRY(launch_est_acc_offsets(A, big, st, off, total, s));
    HIP_TRY(hipMemcpyAsync(&tot, total, sizeof tot, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  STA_TRY(tmp.alloc(&A.acc, (size_t)std::max<unsigned long long>(2 * tot, 1)));
  STA_TRY(tmp.alloc(&A.big_tmp, (size_t)std::max<unsigned long long>(16 * tot, 1)));
  if (tot > 0) HIP_TRY(hipMemsetAsync(A.acc, 0, 2 * tot * sizeof(unsigned long long), s));
  A.acc_off = off;
  A.err = st + 6;
  // the trees rebuilt from the positions, checked against the caller's, and differentiated
  STA_TRY(est_forked(s, [&](hipStream_t side) { return launch_est_grad(A, mid, big, st, h[0], h[1], s, side); }));
  HIP_TRY(hipMemcpyAsync(h + 6, st + 6, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h[6] != ~0u)
    return fail(STA_E_ARG, "net %u: parent / sink_node are not the trees these positions give", h[6]);
  if (mem == STA_HOST && NP > 0) {
    HIP_TRY(hipMemcpyAsync(grad_x, A.gx, NP * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(grad_y, A.gy, NP * sizeof(float), hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  return STA_OK;
}

extern "C" sta_status sta_backward(sta_ctx *C, float g_tns, float g_wns, float *grad_wire_cap,
                                   float *grad_wire_res, float *grad_pin_load, float *grad_arc_delay, sta_mem dst,
                                   void *stream) {
  if (!C) return fail(STA_E_STATE, "NULL context");
  if (C->opt.mode != 1) return fail(STA_E_STATE, "sta_backward needs a context created with mode 1 (smooth)");
  if (!C->updated) return fail(STA_E_STATE, "sta_backward before sta_update_timing");
  if (!std::isfinite(g_tns) || !std::isfinite(g_wns)) return fail(STA_E_ARG, "non-finite seed");
  if (dst != STA_HOST && dst != STA_DEVICE) return fail(STA_E_ARG, "bad dst");
  HIP_TRY(hipSetDevice(C->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool prof = C->opt.profile != 0;
  const DevDesign &D = C->D;
  if (prof) HIP_TRY(hipEventRecord(C->ev[7], s));
  // the reverse sweep runs one launch per level in every schedule, then the
  // RC adjoint (run beside the sweep in level groups, it slowed both: 0.90 ->
  // 1.01 ms on the 1M-pin design)
  for (const int4 &ph : C->ph_adj) HIP_TRY(launch_adjoint_phase(D, g_tns, g_wns, ph, C->lvl_reg[ph.w].z, s));
  if (prof) HIP_TRY(hipEventRecord(C->ev[8], s));
  STA_TRY(enqueue_rc(C, s, true, grad_wire_res != nullptr));
  if (prof) HIP_TRY(hipEventRecord(C->ev[9], s));
  C->bwd_timed = prof;
  if (!grad_wire_cap && !grad_wire_res && !grad_pin_load && !grad_arc_delay) return STA_OK;
  if (dst == STA_DEVICE) {
    HIP_TRY(launch_scatter_grads(D, C->node_src, C->n_nodes, grad_wire_cap, grad_wire_res, C->pin_loc, C->n_pins,
                                 grad_pin_load, C->arc_src, C->n_fanin, reinterpret_cast<float4 *>(grad_arc_delay),
                                 s));
    return STA_OK;
  }
  sta_ctx tmp;
  float *gc = nullptr, *gr = nullptr, *gl = nullptr;
  float4 *ga = nullptr;
  if (grad_wire_cap) STA_TRY(tmp.alloc(&gc, (size_t)C->n_nodes));
  if (grad_wire_res) STA_TRY(tmp.alloc(&gr, (size_t)C->n_nodes));
  if (grad_pin_load) STA_TRY(tmp.alloc(&gl, C->n_pins));
  if (grad_arc_delay) STA_TRY(tmp.alloc(&ga, std::max(C->n_fanin, 1)));
  HIP_TRY(launch_scatter_grads(D, C->node_src, C->n_nodes, gc, gr, C->pin_loc, C->n_pins, gl, C->arc_src,
                               C->n_fanin, ga, s));
  STA_TRY(deliver(grad_wire_cap, gc, (size_t)C->n_nodes * 4, STA_HOST, s));
  STA_TRY(deliver(grad_wire_res, gr, (size_t)C->n_nodes * 4, STA_HOST, s));
  STA_TRY(deliver(grad_pin_load, gl, (size_t)C->n_pins * 4, STA_HOST, s));
  STA_TRY(deliver(grad_arc_delay, ga, (size_t)C->n_fanin * 16, STA_HOST, s));
  HIP_TRY(hipStreamSynchronize(s));
  return STA_OK;
}

extern "C" sta_status sta_get_phase_times(sta_ctx *C, float *ms, int32_t *n) {
  if (!C || !ms || !n) return fail(STA_E_ARG, "NULL argument");
  if (!C->timed) return fail(STA_E_STATE, "no profiled update (set options.profile = 1)");
  HIP_TRY(hipSetDevice(C->device));
  HIP_TRY(hipEventSynchronize(C->ev[6]));
  for (int i = 0; i < 6; ++i) HIP_TRY(hipEventElapsedTime(&ms[i], C->ev[i], C->ev[i + 1]));
  ms[6] = ms[7] = 0.0f;
  if (C->bwd_timed) {
    HIP_TRY(hipEventSynchronize(C->ev[9]));
    HIP_TRY(hipEventElapsedTime(&ms[6], C->ev[7], C->ev[8]));
    HIP_TRY(hipEventElapsedTime(&ms[7], C->ev[8], C->ev[9]));
  }
  *n = 8;
  return STA_OK;
}

// A dataflow sweep whose wait gave up leaves a raised error word (its
// results are invalid); reports surface it.
static sta_status check_flow(sta_ctx *C, hipStream_t s) {
  if (!C->flow_err || C->flow_epoch == 0) return STA_OK;
  uint32_t e = 0;
  HIP_TRY(hipMemcpyAsync(&e, C->flow_err, sizeof e, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (e) return fail(STA_E_DEVICE, "a dataflow sweep wait timed out; results are invalid");
  return STA_OK;
}

extern "C" sta_status sta_report_timing(sta_ctx *C, float *at, float *slew, float *rat, int8_t *crit,
                                        sta_mem dst, void *stream) {
  if (!C) return fail(STA_E_STATE, "NULL context");
  if (dst != STA_HOST && dst != STA_DEVICE) return fail(STA_E_ARG, "bad dst");
  if (rat && C->opt.mode == 1) return fail(STA_E_STATE, "smooth mode computes no required times");
  HIP_TRY(hipSetDevice(C->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  STA_TRY(check_flow(C, s));
  const size_t n4 = (size_t)C->n_pins * sizeof(float4);
  if (dst == STA_DEVICE) {
    HIP_TRY(launch_report_pins(C->D, C->pin_loc, C->n_pins, reinterpret_cast<float4 *>(at),
                               reinterpret_cast<float4 *>(slew), reinterpret_cast<float4 *>(rat),
                               reinterpret_cast<uint32_t *>(crit), nullptr, s));
    return STA_OK;
  }
  sta_ctx tmp;
  float4 *a = nullptr, *sl = nullptr, *r = nullptr;
  uint32_t *cr = nullptr;
  if (at) STA_TRY(tmp.alloc(&a, C->n_pins));
  if (slew) STA_TRY(tmp.alloc(&sl, C->n_pins));
  if (rat) STA_TRY(tmp.alloc(&r, C->n_pins));
  if (crit) STA_TRY(tmp.alloc(&cr, C->n_pins));
  HIP_TRY(launch_report_pins(C->D, C->pin_loc, C->n_pins, a, sl, r, cr, nullptr, s));
  STA_TRY(deliver(at, a, n4, STA_HOST, s));
  STA_TRY(deliver(slew, sl, n4, STA_HOST, s));
  STA_TRY(deliver(rat, r, n4, STA_HOST, s));
  STA_TRY(deliver(crit, cr, (size_t)C->n_pins * 4, STA_HOST, s));
  HIP_TRY(hipStreamSynchronize(s));
  return STA_OK;
}

extern "C" sta_status sta_report_slack(sta_ctx *C, float *pin_slack, float *ep_slack, int32_t *ep_order,
                                       double *wns, double *tns, sta_mem dst, void *stream) {
  if (!C) return fail(STA_E_STATE, "NULL context");
  if (dst != STA_HOST && dst != STA_DEVICE) return fail(STA_E_ARG, "bad dst");
  if (ep_order && !C->opt.sort_endpoints) return fail(STA_E_STATE, "endpoint sorting is disabled");
  if (pin_slack && C->opt.mode == 1) return fail(STA_E_STATE, "smooth mode computes no pin slacks");
  HIP_TRY(hipSetDevice(C->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  STA_TRY(check_flow(C, s));
  sta_ctx tmp;
  if (pin_slack) {
    float4 *ps = reinterpret_cast<float4 *>(pin_slack);
    if (dst == STA_HOST) STA_TRY(tmp.alloc(&ps, C->n_pins));
    HIP_TRY(launch_report_pins(C->D, C->pin_loc, C->n_pins, nullptr, nullptr, nullptr, nullptr, ps, s));
    if (dst == STA_HOST) STA_TRY(deliver(pin_slack, ps, (size_t)C->n_pins * sizeof(float4), STA_HOST, s));
  }
  STA_TRY(deliver(ep_slack, C->D.ep_slack, (size_t)C->n_ep * sizeof(float2), dst, s));
  STA_TRY(deliver(ep_order, C->order, (size_t)C->n_ep * 2 * sizeof(int32_t), dst, s));
  double h[4] = {0, 0, 0, 0};
  std::vector<double> hb;
  if ((wns || tns) && C->batched) {
    hb.resize((size_t)C->n_designs * 4);
    HIP_TRY(hipMemcpyAsync(hb.data(), C->b_out, hb.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  } else if (wns || tns) {
    HIP_TRY(hipMemcpyAsync(h, C->out, sizeof h, hipMemcpyDeviceToHost, s));
  }
  if (dst == STA_HOST || wns || tns) HIP_TRY(hipStreamSynchronize(s));
  for (int d = 0; d < (int)hb.size() / 4; ++d) {  // batch: min of WNS, sum of TNS in design order
    h[0] = std::min(h[0], hb[4 * d + 0]);
    h[1] = std::min(h[1], hb[4 * d + 1]);
    h[2] += hb[4 * d + 2];
    h[3] += hb[4 * d + 3];
  }
  if (wns) { wns[0] = h[0]; wns[1] = h[1]; }
  if (tns) { tns[0] = h[2]; tns[1] = h[3]; }
  return STA_OK;
}

extern "C" sta_status sta_report_levels(sta_ctx *C, int32_t *pin_level, int32_t *level_order, sta_mem dst,
                                        void *stream) {
  if (!C) return fail(STA_E_STATE, "NULL context");
  HIP_TRY(hipSetDevice(C->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  STA_TRY(deliver(pin_level, C->pin_level, (size_t)C->n_pins * 4, dst, s));
  STA_TRY(deliver(level_order, C->level_order, (size_t)C->n_pins * 4, dst, s));
  if (dst == STA_HOST) HIP_TRY(hipStreamSynchronize(s));
  return STA_OK;
}

extern "C" sta_status sta_report_rc(sta_ctx *C, float *net_load, float *sink_delay, float *sink_spread,
                                    sta_mem dst, void *stream) {
  if (!C) return fail(STA_E_STATE, "NULL context");
  HIP_TRY(hipSetDevice(C->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dst == STA_DEVICE) {
    HIP_TRY(launch_report_rc(C->D, C->net_slot, C->n_nets, C->sink_slot, C->n_sinks, net_load, sink_delay,
                             sink_spread, s));
    return STA_OK;
  }
  sta_ctx tmp;
  float *l = nullptr, *d = nullptr, *q = nullptr;
  if (net_load) STA_TRY(tmp.alloc(&l, C->n_nets));
  if (sink_delay) STA_TRY(tmp.alloc(&d, C->n_sinks));
  if (sink_spread) STA_TRY(tmp.alloc(&q, C->n_sinks));
  HIP_TRY(launch_report_rc(C->D, C->net_slot, C->n_nets, C->sink_slot, C->n_sinks, l, d, q, s));
  STA_TRY(deliver(net_load, l, (size_t)C->n_nets * 4, STA_HOST, s));
  STA_TRY(deliver(sink_delay, d, (size_t)C->n_sinks * 4, STA_HOST, s));
  STA_TRY(deliver(sink_spread, q, (size_t)C->n_sinks * 4, STA_HOST, s));
  HIP_TRY(hipStreamSynchronize(s));
  return STA_OK;
}

extern "C" sta_status sta_report_endpoints(sta_ctx *C, int32_t *ep_pin, sta_mem dst, void *stream) {
  if (!C) return fail(STA_E_STATE, "NULL context");
  HIP_TRY(hipSetDevice(C->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  STA_TRY(deliver(ep_pin, C->ep_pin, (size_t)C->n_ep * 4, dst, s));
  if (dst == STA_HOST) HIP_TRY(hipStreamSynchronize(s));
  return STA_OK;
}

extern "C" sta_status sta_get_info(const sta_ctx *C, sta_info *info) {
  if (!C || !info) return fail(STA_E_ARG, "NULL argument");
  info->n_pins = C->n_pins;
  info->n_cells = C->n_cells;
  info->n_nets = C->n_nets;
  info->n_pi = C->n_pi;
  info->n_po = C->n_po;
  info->n_sinks = C->n_sinks;
  info->n_nodes = C->n_nodes;
  info->n_levels = C->n_levels;
  info->n_cell_levels = C->n_cell_levels;
  info->n_endpoints = C->n_ep;
  info->n_big_nets = C->n_big;
  info->n_chunks = C->n_chunks;
  info->device = C->device;
  return STA_OK;
}

extern "C" sta_status sta_batch_report(sta_ctx *C, double *wns, double *tns, void *stream) {
  if (!C) return fail(STA_E_STATE, "NULL context");
  if (!C->updated) return fail(STA_E_STATE, "sta_batch_report before sta_update_timing");
  HIP_TRY(hipSetDevice(C->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<double> h((size_t)C->n_designs * 4);
  HIP_TRY(hipMemcpyAsync(h.data(), C->batched ? C->b_out : C->out, h.size() * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int d = 0; d < C->n_designs; ++d) {
    if (wns) { wns[2 * d] = h[4 * d + 0]; wns[2 * d + 1] = h[4 * d + 1]; }
    if (tns) { tns[2 * d] = h[4 * d + 2]; tns[2 * d + 1] = h[4 * d + 3]; }
  }
  return STA_OK;
}

extern "C" sta_status sta_autotune(sta_ctx *C, int32_t reps, sta_tune_result *best, void *stream) {
  if (!C) return fail(STA_E_STATE, "NULL context");
  if (reps < 1) return fail(STA_E_ARG, "reps %d < 1", reps);
  HIP_TRY(hipSetDevice(C->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  struct Cand { int sched, grid, overlap; };
  std::vector<Cand> cands;
  const int max_per_cu = std::max(1, C->coop_max > 0 ? C->coop_max / std::max(1, C->n_cu)
                                                    : sweep_blocks_per_cu(sweep_lds_bytes(C->D)));
  const int max_grid = max_per_cu * C->n_cu;
  for (int k = 1; k <= max_per_cu; ++k) cands.push_back({STA_SCHED_PERSISTENT, k * C->n_cu, 0});
  for (int ov = 0; ov <= 1; ++ov) {
    cands.push_back({STA_SCHED_PER_LEVEL, max_grid, ov});
    cands.push_back({STA_SCHED_GRAPH, max_grid, ov});
  }
  if (C->flow_ok) cands.push_back({STA_SCHED_FLOW, max_grid, 0});
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const sta_options saved = C->opt;
  C->opt.profile = 0;
  sta_tune_result r{saved.sched, C->sweep_grid, 0.0f, 0, saved.overlap};
  float best_ms = INFINITY;
  sta_status st = STA_OK;
  for (const Cand &c : cands) {
    C->opt.sched = c.sched;
    C->opt.overlap = c.overlap;
    C->sweep_grid = c.grid;
    C->coop = c.grid <= C->coop_max;
    st = sta_update_timing(C, s);  // warm-up (builds the graph once)
    if (st != STA_OK) break;
    hipError_t e = hipEventRecord(e0, s);
    for (int i = 0; i < reps && st == STA_OK && e == hipSuccess; ++i) st = sta_update_timing(C, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      st = hip_fail(e, "autotune timing");
      break;
    }
    if (st != STA_OK) break;
    ms /= (float)reps;
    r.n_tried++;
    if (ms < best_ms) {
      best_ms = ms;
      r.sched = c.sched;
      r.sweep_blocks = c.grid;
      r.overlap = c.overlap;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  C->opt = saved;
  if (st != STA_OK) {
    C->sweep_grid = max_grid;
    C->coop = max_grid <= C->coop_max;
    return st;
  }
  C->opt.sched = r.sched;
  C->opt.overlap = r.overlap;
  C->sweep_grid = r.sweep_blocks;
  C->coop = r.sweep_blocks <= C->coop_max;
  r.ms = best_ms;
  if (best) *best = r;
  return STA_OK;
}

// Pieces of one device buffer, each 256-byte aligned: a first pass with no
// base only adds up the size.
struct Carve {
  unsigned char *base = nullptr;
  size_t off = 0;
  template <class T>
  T *take(size_t n) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += std::max<size_t>(n, 1) * sizeof(T);
    return p;
  }
};

// The path workspace holds at least `bytes` (its old contents are dropped;
// every report ends synchronized, so nothing still uses them).
static sta_status path_ws_reserve(sta_ctx *C, size_t bytes) {
  if (C->path_ws && C->path_ws_bytes >= bytes) return STA_OK;
  C->path_ws.reset();
  C->path_ws_bytes = 0;
  auto m = std::make_unique<DevMem>();
  const hipError_t e = hipMalloc(&m->p, bytes);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc");
  C->path_ws = std::move(m);
  C->path_ws_bytes = bytes;
  return STA_OK;
}

extern "C" sta_status sta_report_paths(sta_ctx *C, const sta_path_query *q, int32_t *n_paths, int32_t *path_ptr,
                                       int32_t *path_pin, int8_t *path_rf, float *path_slack, int32_t *path_endpoint,
                                       sta_mem dst, void *stream) {
  if (!C) return fail(STA_E_STATE, "NULL context");
  if (!q || !n_paths) return fail(STA_E_ARG, "NULL query or n_paths");
  if (q->k < 1 || q->per_endpoint < 1 || q->per_endpoint > 64 || (q->el != 0 && q->el != 1) ||
      std::isnan(q->slack_below))
    return fail(STA_E_ARG, "bad path query (k %d, per_endpoint %d, el %d)", q->k, q->per_endpoint, q->el);
  if (dst != STA_HOST && dst != STA_DEVICE) return fail(STA_E_ARG, "bad dst");
  if (C->opt.mode != 0) return fail(STA_E_STATE, "path reports need a hard-mode context");
  if (!C->opt.sort_endpoints) return fail(STA_E_STATE, "path reports need endpoint sorting");
  if (!C->updated) return fail(STA_E_STATE, "sta_report_paths before sta_update_timing");
  HIP_TRY(hipSetDevice(C->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  *n_paths = 0;
  const int ne = C->n_ep, el = q->el, m = q->per_endpoint;
  // endpoints that can hold a reported path: the first k in ascending endpoint
  // slack (each holds a path of its own slack), and only those below the
  // threshold (no path of an endpoint is better than its slack)
  const int cand = std::min(q->k, ne);
  int n_sel = 0;
  if (cand > 0) {  // counted on the device: the leading endpoints below the threshold
    STA_TRY(path_ws_reserve(C, 256));
    int32_t *cnt = static_cast<int32_t *>(C->path_ws->p);
    HIP_TRY(launch_paths_count(C->D, C->order + (size_t)el * ne, cand, el, q->slack_below, cnt, s));
    HIP_TRY(hipMemcpyAsync(&n_sel, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  if (n_sel == 0) {
    const int32_t zero = 0;
    if (path_ptr && dst == STA_HOST) path_ptr[0] = 0;
    if (path_ptr && dst == STA_DEVICE) {
      HIP_TRY(hipMemcpyAsync(path_ptr, &zero, sizeof zero, hipMemcpyHostToDevice, s));
      HIP_TRY(hipStreamSynchronize(s));
    }
    return STA_OK;
  }
  const int lmax = C->n_levels;
  // each endpoint keeps at most m pending items (in LDS when they fit beside
  // the library), its m paths of at most lmax nodes, their lengths and slacks;
  // then the global selection and the output, all in the kept workspace
  // (STA_PATH_QUEUES_GLOBAL set in the environment forces the global-memory
  // queues, so that both forms can be compared)
  const bool q_lds = paths_queue_lds_bytes(C->D, m) <= 160 * 1024 && !std::getenv("STA_PATH_QUEUES_GLOBAL");
  const int nc = n_sel * m, top = std::min(q->k, nc);
  const size_t sb = sort_temp_bytes(nc);
  size_t xb = 0;
  HIP_TRY(exclusive_sum(nullptr, xb, nullptr, nullptr, top + 1, s));
  PathArgs A{};
  uint32_t *keys, *keys_out;
  int32_t *vals, *vals_out, *len, *ptr, *pin, *pe;
  unsigned char *stemp, *xtemp;
  int8_t *prf;
  float *psl;
  for (int pass = 0; pass < 2; ++pass) {
    Carve cv;
    if (pass == 1) cv.base = static_cast<unsigned char *>(C->path_ws->p);
    A.items = q_lds ? nullptr : cv.take<int4>((size_t)n_sel * m);
    A.nodes = cv.take<int32_t>((size_t)n_sel * m * lmax);
    A.plen = cv.take<int32_t>((size_t)nc);
    A.pkey = cv.take<float>((size_t)nc);
    keys = cv.take<uint32_t>(nc);
    keys_out = cv.take<uint32_t>(nc);
    vals = cv.take<int32_t>(nc);
    vals_out = cv.take<int32_t>(nc);
    stemp = cv.take<unsigned char>(sb);
    len = cv.take<int32_t>((size_t)top + 1);
    ptr = cv.take<int32_t>((size_t)top + 1);
    xtemp = cv.take<unsigned char>(xb);
    pin = cv.take<int32_t>((size_t)top * lmax);
    prf = cv.take<int8_t>((size_t)top * lmax);
    psl = cv.take<float>((size_t)top);
    pe = cv.take<int32_t>((size_t)top);
    if (pass == 0) {
      if ((double)cv.off > 16e9) return fail(STA_E_UNSUPPORTED, "path search needs %.1f GB of scratch", cv.off / 1e9);
      STA_TRY(path_ws_reserve(C, cv.off));
    }
  }
  A.eps = C->order + (size_t)el * ne;
  A.n_eps = n_sel;
  A.el = el;
  A.m = m;
  A.lmax = lmax;
  A.thr = q->slack_below;
  A.drv_pin = C->slot_drv_pin;
  A.sink_pin = C->slot_sink_pin;
  HIP_TRY(launch_paths_enum(C->D, A, s));
  // global selection: ascending slack over every found path (ties in
  // endpoint order, then path order)
  HIP_TRY(launch_paths_keys(A, keys, vals, s));
  HIP_TRY(sort_endpoints(stemp, sb, keys, keys_out, vals, vals_out, nc, s));
  std::vector<uint32_t> hk(top);
  HIP_TRY(hipMemcpyAsync(hk.data(), keys_out, top * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  int n_out = 0;
  while (n_out < top && hk[n_out] != 0xffffffffu) ++n_out;
  HIP_TRY(hipMemsetAsync(len, 0, (n_out + 1) * sizeof(int32_t), s));
  HIP_TRY(launch_paths_lengths(A, vals_out, n_out, len, s));
  HIP_TRY(exclusive_sum(xtemp, xb, len, ptr, n_out + 1, s));  // (scratch sized for top + 1 items)
  int32_t total = 0;
  HIP_TRY(hipMemcpyAsync(&total, ptr + n_out, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(launch_paths_emit(C->D, A, vals_out, n_out, ptr, pin, prf, psl, pe, s));
  STA_TRY(deliver(path_ptr, ptr, (size_t)(n_out + 1) * 4, dst, s));
  STA_TRY(deliver(path_pin, pin, (size_t)total * 4, dst, s));
  STA_TRY(deliver(path_rf, prf, (size_t)total, dst, s));
  STA_TRY(deliver(path_slack, psl, (size_t)n_out * 4, dst, s));
  STA_TRY(deliver(path_endpoint, pe, (size_t)n_out * 4, dst, s));
  HIP_TRY(hipStreamSynchronize(s));
  *n_paths = n_out;
  return STA_OK;
}
