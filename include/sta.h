/*
 * sta.h - C ABI of the MI355X static-timing hot path (libsta.so).
 *
 * What it computes (HeteroSTA, arXiv 2511.11660): graph-based static timing
 * analysis on a flattened netlist.  Per net, Elmore delay and slew on the RC
 * tree (§III "Delay models", "Parasitics (RC) inputs"); per cell arc, NLDM
 * delay and output slew by bilinear table lookup (§IV-A, Table I); levelized
 * forward propagation of arrival time and slew and backward propagation of
 * required time, giving per-pin slack, endpoint slack, WNS and TNS (§I, §III
 * "Report options").  The interface follows the paper's flattened,
 * zero-translation API (§II last paragraph, §III "Heterogeneous netlist
 * database"): the netlist arrives as net and cell CSR arrays, parasitics as a
 * flattened RC CSR, and every input and output array may live in host or
 * device memory (§III "Parasitics (RC) inputs", "Report options").
 *
 * Conventions
 *   - Views: index v = 2*el + rf, el 0 early / 1 late, rf 0 rise / 1 fall.
 *     Arrays documented as [n][4] hold the four views of item n contiguously.
 *   - Units: time ps, capacitance fF, resistance kOhm (kOhm x fF = ps).
 *   - Pins carry caller ids 0..n_pins-1.  PIs are ranked by ascending pin id
 *     (index into pi_at / pi_slew), POs likewise (index into po_rat).
 *     Endpoints are the PO pins plus, when dangling_policy is 1, every cell
 *     output without fanout; endpoint e is the e-th endpoint in ascending pin
 *     id.
 *   - sta_mem STA_HOST / STA_DEVICE tells where a pointer lives.  Device
 *     pointers are HIP device addresses on the context's device.
 *   - Every function returns a status; no exception crosses the ABI.  On an
 *     error the thread-local sta_last_error() string says what was wrong.
 *   - A context is used by one host thread at a time.  Work is enqueued on the
 *     HIP stream passed in (NULL = the default stream); calls that return data
 *     to host memory synchronize that stream.
 */
#ifndef STA_H
#define STA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sta_ctx sta_ctx; /* opaque */

typedef enum {
  STA_OK = 0,
  STA_E_ARG = 1,         /* malformed input (bounds, kinds, CSR, NaN, ...) */
  STA_E_CYCLE = 2,       /* the timing graph has a combinational cycle */
  STA_E_OOM = 3,         /* device or host allocation failed */
  STA_E_DEVICE = 4,      /* a HIP call or kernel failed */
  STA_E_STATE = 5,       /* call not valid in the context's current state */
  STA_E_UNSUPPORTED = 6  /* valid input outside what this build supports */
} sta_status;

typedef enum { STA_HOST = 0, STA_DEVICE = 1 } sta_mem;

typedef enum { STA_PIN_PI = 0, STA_PIN_CELL_IN = 1, STA_PIN_CELL_OUT = 2, STA_PIN_PO = 3 } sta_pin_kind;

/* Flattened netlist (§III "Heterogeneous netlist database": net and cell CSR
 * arrays taken directly from a flow, no pin remapping).  Every PI and cell
 * output pin drives exactly one net (which may have no sinks); every cell
 * input and PO pin is a sink of exactly one net.  Cells have one output and
 * at least one input; the order of a cell's inputs is its fanin position. */
typedef struct {
  int32_t n_pins, n_cells, n_nets, n_pi, n_po;
  const int32_t *pin_kind;     /* [n_pins] sta_pin_kind */
  const int32_t *cell_type;    /* [n_cells] library type */
  const int32_t *cell_in_ptr;  /* [n_cells+1] CSR offsets into cell_in_pin */
  const int32_t *cell_in_pin;  /* [cell_in_ptr[n_cells]] input pins per cell */
  const int32_t *cell_out_pin; /* [n_cells] */
  const int32_t *net_driver;   /* [n_nets] driving pin */
  const int32_t *net_sink_ptr; /* [n_nets+1] CSR offsets into net_sink_pin */
  const int32_t *net_sink_pin; /* [net_sink_ptr[n_nets]] sink pins per net */
  sta_mem mem;
} sta_graph_desc;

/* Flattened RC CSR (§III "Parasitics (RC) inputs").  Net n owns nodes
 * [net_node_ptr[n], net_node_ptr[n+1]); node 0 of a net is its root at the
 * driver.  parent is net-local with parent[root] = -1 and parent[k] < k.
 * res_kohm[k] is the resistance of the segment parent->k; cap_ff[k] the ground
 * cap at node k.  sink_node[s] is the net-local node of sink s, aligned with
 * sta_graph_desc.net_sink_pin.  The receiving pin's input cap (library pin cap
 * or po_cap_ff) is added at its node. */
typedef struct {
  int64_t n_nodes;
  const int64_t *net_node_ptr; /* [n_nets+1] */
  const int32_t *parent;       /* [n_nodes] */
  const float *res_kohm;       /* [n_nodes] */
  const float *cap_ff;         /* [n_nodes] */
  const int32_t *sink_node;    /* [n_sinks] */
  sta_mem mem;
} sta_rc_desc;

/* Liberty-style NLDM library (§IV-A, Table I uses NLDM).  Per type: tables
 * [4][nx][ny] = cell_rise, cell_fall, rise_transition, fall_transition indexed
 * by (input slew, output load); axes strictly increasing.  sense: 0 positive
 * unate, 1 negative unate, 2 non-unate; all arcs of a type share its tables.
 * Always host memory. */
typedef struct {
  int32_t n_types, nx, ny;     /* n_types <= 64, 2 <= nx, ny <= 8 */
  const int32_t *n_inputs;     /* [n_types] */
  const int32_t *sense;        /* [n_types] */
  const float *pin_cap_ff;     /* [n_types] input pin cap */
  const float *slew_axis;      /* [n_types][nx] ps */
  const float *load_axis;      /* [n_types][ny] fF */
  const float *tables;         /* [n_types][4][nx][ny] ps */
  float po_cap_ff;             /* load of a PO pin */
} sta_lib_desc;

/* Boundary constraints; always host memory. */
typedef struct {
  const float *pi_at;          /* [n_pi][4] */
  const float *pi_slew;        /* [n_pi][4] */
  const float *po_rat;         /* [n_po][4] */
  float dangling_rat[4];       /* RAT of dangling cell outputs when they are endpoints */
} sta_constraints;

/* Schedules for the level sweeps. */
typedef enum {
  STA_SCHED_PERSISTENT = 0,    /* one launch per sweep, device-side level counters */
  STA_SCHED_PER_LEVEL = 1,     /* one launch per level */
  STA_SCHED_GRAPH = 2,         /* one launch per level, captured once in a HIP graph and replayed
                                  (in-graph phases are not timed separately) */
  STA_SCHED_FLOW = 3           /* one launch per sweep, no level barrier: each chunk waits only for the
                                  chunks producing its inputs (per-chunk completion flags); needs library
                                  types of at most 4 inputs and cooperative launch (else STA_E_UNSUPPORTED) */
} sta_sched;

typedef struct {
  int32_t mode;                /* 0 hard max/min; 1 smooth late arrival merges (differentiable) */
  float gamma_ps;              /* smoothing temperature of mode 1 (> 0), e.g. 5 ps */
  int32_t dangling_policy;     /* 0: zero-fanout cell outputs unconstrained; 1: endpoints */
  int32_t sched;               /* sta_sched; default STA_SCHED_PER_LEVEL */
  int32_t big_net_nodes;       /* nets with more RC nodes go to the wide RC kernel; 0 = 255 */
  int32_t sort_endpoints;      /* 1: sta_update_timing also orders endpoints by slack */
  int32_t profile;             /* 1: record per-kernel HIP event times in sta_update_timing */
  int32_t device;              /* HIP device ordinal; -1 = current device */
  int32_t sweep_blocks;        /* persistent sweep grid (blocks of 256 threads); 0 = every block slot
                                  the device can hold resident (any value >= 1 is deadlock-free) */
  int32_t delay_model;         /* net delay: 0 Elmore (first moment); 1 reduced-order model (§III
                                  "Delay models": Arnoldi iterations, here two steps in the G inner
                                  product from the Elmore vector; the 50% time of the projected step
                                  response; hard mode only) */
  int32_t overlap;             /* per-level and graph schedules: 1 (default) runs the RC pass in level
                                  groups beside the forward sweep and WNS/TNS with the endpoint order
                                  beside the backward sweep, on the context's own side streams; 0 runs
                                  every phase in order on the caller's stream.  Results are identical */
} sta_options;

typedef struct {
  int32_t n_pins, n_cells, n_nets, n_pi, n_po, n_sinks;
  int64_t n_nodes;
  int32_t n_levels;            /* pin levels (max pin level + 1) */
  int32_t n_cell_levels;       /* max cell level (cells at 1..n_cell_levels) */
  int32_t n_endpoints;
  int32_t n_big_nets;          /* nets routed to the wide RC kernel */
  int32_t n_chunks;            /* sweep work items */
  int32_t device;
} sta_info;

/* Fills *opt with the defaults: hard mode (gamma 5 ps for smooth mode), per-level schedule with
   side-stream overlap, Elmore net delays, endpoint sorting on, current device. */
void sta_options_default(sta_options *opt);

/* Validates the inputs on the host, levelizes the timing graph on the device
 * (longest-path levels; a cycle gives STA_E_CYCLE) and builds the device
 * layout.  All input arrays are read during the call only (device arrays are
 * copied); the context owns every buffer it allocates.  opts may be NULL for
 * the defaults.  *out is set only on STA_OK. */
sta_status sta_create(const sta_graph_desc *graph, const sta_rc_desc *rc, const sta_lib_desc *lib,
                      const sta_constraints *cons, const sta_options *opts, sta_ctx **out);

/* Releases the context and its device memory.  NULL is a no-op. */
void sta_destroy(sta_ctx *ctx);

/* Replaces every RC node's ground cap (caller node order, [n_nodes] fF), the
 * quantity an optimization loop changes between timing updates (§IV-C, IV-D
 * flows call the timer inside their loop).  The values are copied (permuted
 * into the device layout) on `stream`; the caller's buffer may be reused once
 * the stream has passed this point.  Values must be finite and >= 0 (checked
 * on the host for STA_HOST input only). */
sta_status sta_set_wire_caps(sta_ctx *ctx, const float *cap_ff, sta_mem mem, void *stream);

/* One full timing update on `stream`, asynchronous: RC pass (Elmore delay,
 * impulse spread, net load), forward AT/slew sweep with NLDM lookups, backward
 * RAT sweep with slacks, endpoint WNS/TNS (FP64, fixed reduction order) and,
 * if enabled, the endpoint order.  Device faults surface as STA_E_DEVICE at
 * the next synchronizing call. */
sta_status sta_update_timing(sta_ctx *ctx, void *stream);

/* Incremental timing update (§I: incremental GPU graph propagation is among
 * the prior art the paper builds on, and its TAU 2015 designs come from an
 * incremental-timing contest; §IV flows call the timer after small changes).
 * Precondition: sta_update_timing has run on this context, and since the
 * last update (full or incremental) the wire caps changed only on the nets
 * listed.  Recomputes the RC pass of those nets, arrivals in their fan-out
 * cone and RATs in the fan-in cone of what changed, stopping wherever a
 * recomputed value is bitwise unchanged, then WNS/TNS and the endpoint order
 * as a full update does.  Every output is then bitwise equal to what
 * sta_update_timing would give.  A net whose caps changed but is not listed
 * leaves stale results (not detected).
 *
 *   nets [n_nets]   caller net ids (duplicates allowed), in `mem` memory.  A
 *                   host list may be reused when the call returns.  A device
 *                   list is read back to check the ids (synchronizes
 *                   `stream`) and then read again by the device, so it must
 *                   stay unchanged until `stream` has passed the call.
 *                   n_nets = 0 recomputes nothing but the reports.
 *
 * Errors: STA_E_STATE (NULL context, or no full update yet), STA_E_ARG (bad
 * list or id; nothing is enqueued), STA_E_UNSUPPORTED (batched context).
 * Allocates device queues and flags (about 4 bytes per driver, sink, chunk
 * and RC chunk) and pinned staging for the list on first use (the staging
 * grows with the longest list).  The call waits for the device twice (where
 * a small-cone sweep hands over to per-level launches); the rest is
 * asynchronous on `stream`. */
sta_status sta_update_timing_incremental(sta_ctx *ctx, const int32_t *nets, int32_t n_nets, sta_mem mem,
                                         void *stream);

/* Slack report (§III "Report options": pin slacks, WNS/TNS).  Any pointer may
 * be NULL to skip it.  pin_slack [n_pins][4] (late RAT-AT, early AT-RAT, +inf
 * when unconstrained); ep_slack [n_endpoints][2] (min over rise/fall, per
 * early/late); ep_order [2][n_endpoints] endpoint indices by ascending (slack,
 * pin id), per early/late (requires sort_endpoints); wns[2], tns[2] per
 * early/late with WNS = min(0, min slack) and TNS = sum of min(0, slack)
 * (Table IV prints both as 0 for a clean design).  Array outputs go to `dst`
 * memory; wns/tns are always host doubles.  Synchronizes `stream` when any
 * output is host memory. */
sta_status sta_report_slack(sta_ctx *ctx, float *pin_slack, float *ep_slack, int32_t *ep_order,
                            double *wns, double *tns, sta_mem dst, void *stream);

/* Per-pin timing in caller pin order, each [n_pins][4] or NULL: arrival,
 * slew, required time, and the critical fanin of each cell output view
 * (2 * fanin position + input transition, ties to the lower value; -1 for
 * pins that are not cell outputs). */
sta_status sta_report_timing(sta_ctx *ctx, float *at, float *slew, float *rat, int8_t *crit,
                             sta_mem dst, void *stream);

/* Pin levels [n_pins] and the pins in ascending (level, pin id) [n_pins]. */
sta_status sta_report_levels(sta_ctx *ctx, int32_t *pin_level, int32_t *level_order, sta_mem dst,
                             void *stream);

/* RC pass results (§III "Delay models"): net_load [n_nets] in caller net order,
 * sink_delay and sink_spread [n_sinks] in caller sink order (Elmore delay and
 * impulse-response spread q; sink slew = sqrt(driver slew^2 + q)). */
sta_status sta_report_rc(sta_ctx *ctx, float *net_load, float *sink_delay, float *sink_spread,
                         sta_mem dst, void *stream);

/* Endpoint pins [n_endpoints] in endpoint-index order (ascending pin id). */
sta_status sta_report_endpoints(sta_ctx *ctx, int32_t *ep_pin, sta_mem dst, void *stream);

/* Sizes and schedule facts of a context. */
sta_status sta_get_info(const sta_ctx *ctx, sta_info *info);

/* Per-kernel durations (ms) when profiling is on: ms[0] RC pass, ms[1] unused
 * (0), ms[2] forward sweep, ms[3] backward sweep, ms[4] endpoint reduction,
 * ms[5] endpoint sort of the last sta_update_timing; ms[6] adjoint sweep and
 * ms[7] RC adjoint of the last sta_backward (0 if none).  *n receives the count
 * (8); ms needs room for 8.  Synchronizes the streams of those calls. */
sta_status sta_get_phase_times(sta_ctx *ctx, float *ms, int32_t *n);

/* Smooth mode (options.mode = 1).  Not in the paper: a differentiable form for
 * gradient-driven optimization loops of the kind §IV-C (timing-driven
 * placement, which consumes back-propagated pin slacks) and §IV-D run.  Late
 * arrival merges become log-sum-exp with temperature g = gamma_ps; the late
 * endpoint slack is s = -LSE_g(AT - RAT over rise/fall); the update reports
 * (through sta_report_slack) tns[1] = TNS_g = sum -g log(1 + e^{-s/g}) and
 * wns[1] = WNS_g = -g log(1 + sum e^{-s/g}), with the early views hard.  In
 * this mode the update runs no required-time sweep (pin RAT/slack reports
 * return STA_E_STATE).
 *
 * sta_backward computes, after sta_update_timing on the same context, the
 * gradient of J = g_tns TNS_g + g_wns WNS_g with respect to:
 *   grad_wire_cap  [n_nodes]    every RC node's ground cap, caller node order
 *                               (through the RC moments and the driver's load);
 *   grad_wire_res  [n_nodes]    every segment's resistance (parent -> node),
 *                               caller node order, through the RC moments
 *                               (0 at net roots);
 *   grad_pin_load  [n_pins]     each cell output's NLDM load (partial through
 *                               the lookups only; 0 on other pins);
 *   grad_arc_delay [n_arcs][4]  each cell arc's additive delay per output view
 *                               (arcs in cell_in_pin order; early views 0).
 * Any output may be NULL; outputs go to `dst` memory.  Activations are not
 * stored beyond the per-pin arrival/slew the update keeps anyway: the reverse
 * sweep recomputes delays, softmax weights and table partials from them.
 * Gradients are accumulated in a fixed order (bitwise reproducible).
 * STA_E_STATE if the context is not in mode 1 or was never updated. */
sta_status sta_backward(sta_ctx *ctx, float g_tns, float g_wns, float *grad_wire_cap, float *grad_wire_res,
                        float *grad_pin_load, float *grad_arc_delay, sta_mem dst, void *stream);

/* Batched form (not in the paper; the paper's flows time one design per call).
 * Times n_designs independent designs that share one cell library (one
 * technology) as a single timing graph: their netlists, RC trees and
 * constraints are concatenated in design order (design d's pins, cells, nets,
 * RC nodes, PIs and POs follow design d-1's), the union is levelized (design
 * levels line up: level l of the union holds every design's level-l cells),
 * and every sta_update_timing then runs each sweep over all designs at once
 * (one persistent launch per sweep, or one HIP graph replay with
 * STA_SCHED_GRAPH).  graphs, rcs and cons are arrays of n_designs
 * descriptors, each validated as sta_create would (errors name the design);
 * lib is the one shared library (sta_batch_create_libs below takes one per
 * design).  Per-pin results are bit-identical to timing
 * each design alone.  The union must stay within the single-context limits
 * (int32 pin, sink and node counts), else STA_E_UNSUPPORTED; batches time hard
 * mode only (opts->mode must be 0, else STA_E_UNSUPPORTED).
 *
 * On a batched context the per-pin reports of sta_report_timing / _slack /
 * _levels / _rc / _endpoints and sta_set_wire_caps use the concatenated
 * orders; sta_report_slack's wns/tns aggregate the designs (min of WNS, sum of
 * TNS in design order) and its ep_order holds, in each design's endpoint range,
 * design-local endpoint indices by ascending (slack, pin id). */
sta_status sta_batch_create(int32_t n_designs, const sta_graph_desc *graphs, const sta_rc_desc *rcs,
                            const sta_lib_desc *lib, const sta_constraints *cons, const sta_options *opts,
                            sta_ctx **out);

/* sta_batch_create with a library per design: corners (one netlist under
 * several libraries, e.g. slow / typical / fast) or designs of several
 * technologies in one batch.  libs holds n_designs pointers; designs whose
 * pointers are equal share that library's types, and design d's cell types
 * index libs[d].  The context's library is the union of the distinct
 * libraries, one after the other, each kept as given (its tables, pin caps,
 * unateness and PO pin cap apply to its own designs), so per-pin results are
 * bit-identical to timing each design alone with its own library.  Every
 * library must have the same table shape (nx, ny) and the union at most 256
 * types (else STA_E_UNSUPPORTED); the persistent, dataflow and path-report
 * kernels also need the whole union in LDS (about five 32-type libraries of
 * 7x7 tables), else sta_batch_create_libs returns STA_E_UNSUPPORTED for them
 * at create.  Otherwise as sta_batch_create. */
sta_status sta_batch_create_libs(int32_t n_designs, const sta_graph_desc *graphs, const sta_rc_desc *rcs,
                                 const sta_lib_desc *const *libs, const sta_constraints *cons,
                                 const sta_options *opts, sta_ctx **out);

/* Concatenation offsets of a batched context, host arrays of n_designs + 1
 * entries each (any may be NULL): pin_off, ep_off (endpoint index ranges),
 * node_off (RC node ranges).  *n_designs receives the design count (1 and the
 * whole design for a context from sta_create). */
sta_status sta_batch_offsets(const sta_ctx *ctx, int32_t *n_designs, int32_t *pin_off, int32_t *ep_off,
                             int64_t *node_off);

/* Per-design results of the last update, host doubles [n_designs][2] each
 * (early, late), any may be NULL: WNS = min(0, min endpoint slack) and TNS =
 * sum of min(0, slack) over the design's endpoints, reduced with the same
 * partition and order as a single-design context (bit-identical to timing the
 * design alone).  Synchronizes `stream`.  STA_E_STATE before an update. */
sta_status sta_batch_report(sta_ctx *ctx, double *wns, double *tns, void *stream);

/* Launch-configuration tuner.  Times `reps` updates (after one warm-up) on
 * `stream` for each candidate schedule: the persistent sweeps at every grid
 * size from 1 block per compute unit up to the occupancy limit, one launch per
 * level, and the captured HIP graph; keeps the fastest in the context (later
 * updates use it) and reports it.  Results of the tuning updates are those of
 * a normal update.  Synchronizes `stream`. */
typedef struct {
  int32_t sched;               /* sta_sched chosen */
  int32_t sweep_blocks;        /* persistent grid (blocks of 256 threads) */
  float ms;                    /* mean update time of the choice */
  int32_t n_tried;             /* candidates timed */
  int32_t overlap;             /* sta_options.overlap chosen */
} sta_tune_result;
sta_status sta_autotune(sta_ctx *ctx, int32_t reps, sta_tune_result *best, void *stream);

/* Top-k timing path report (§III "Report options": top-k path reports
 * controlled by k, a per-endpoint limit and a slack-less-than threshold, as
 * flattened CSR path-pin arrays with slacks).  A path runs from a primary
 * input to an endpoint over net arcs and cell arcs (transitions as each
 * type's unateness allows); its arrival is the startpoint arrival plus the
 * arc delays of the last sta_update_timing (net arc: the sink's Elmore delay;
 * cell arc: the NLDM delay at the input's propagated slew and the output
 * net's load, in the query's early or late view); late slack = endpoint RAT
 * - arrival, early slack = arrival - endpoint RAT, per endpoint transition.
 * The report holds, in ascending slack, the paths of smallest slack over all
 * endpoints, at most per_endpoint of them per endpoint, only those with
 * slack < slack_below, and at most k in all.  Exact (k-best enumeration by
 * deviations from each pin's critical fanin).  Needs a hard-mode context with
 * endpoint sorting on (else STA_E_STATE).
 *
 *   *n_paths            (host) number of paths reported, <= k
 *   path_ptr [k+1]      CSR offsets into path_pin / path_rf
 *   path_pin, path_rf   [k * n_levels] pins from startpoint to endpoint and
 *                       each pin's transition (0 rise, 1 fall); a path has
 *                       at most n_levels (sta_info) pins
 *   path_slack [k]      slack of each path; path_endpoint [k] its endpoint index
 * Any array may be NULL; arrays go to `dst` memory.  The search's device
 * scratch (bounded by k, per_endpoint and the level count)
 * is a workspace the context keeps and grows across reports, freed with the
 * context; each endpoint's pending paths sit in LDS when they fit beside the
 * library (the environment variable STA_PATH_QUEUES_GLOBAL, when set, keeps
 * them in global memory instead, for testing).  Synchronizes `stream`. */
typedef struct {
  int32_t k;                   /* most paths reported (>= 1) */
  int32_t per_endpoint;        /* most paths per endpoint, 1..64 */
  float slack_below;           /* report only slack < slack_below (+inf: no threshold) */
  int32_t el;                  /* 0 early (hold) view, 1 late (setup) view */
} sta_path_query;
sta_status sta_report_paths(sta_ctx *ctx, const sta_path_query *q, int32_t *n_paths, int32_t *path_ptr,
                            int32_t *path_pin, int8_t *path_rf, float *path_slack, int32_t *path_endpoint,
                            sta_mem dst, void *stream);

/* RC trees estimated from pin positions (§III "Parasitics (RC) inputs": in
 * placement flows the timer derives each net's RC tree itself from pin
 * coordinates and per-unit-length resistance and capacitance along x and y,
 * as rectilinear Steiner trees).  Per net, the shortest-path heuristic of
 * Takahashi and Matsuyama (1980) in the rectilinear plane (pin 0 the driver,
 * pins 1..k the sinks in net_sink_pin order): the tree starts as the driver's
 * point; step t = 1..k joins the outside pin nearest to the tree's wires
 * (FP32 Manhattan distance to the nearest point q_t of a wire, ties to the
 * lower pin index; a pin's nearest wire changes only to a strictly nearer
 * one) along an L: wire 2t-1 along x from q_t to the corner K_t = (x_pin,
 * q_t.y), wire 2t along y from K_t to the pin.  Where q_t lies inside a wire
 * the wire is split there (a Steiner point).  Net-local nodes: the driver 0,
 * and per step the attach point S_t, the corner K_t and the pin; the points
 * on a wire (its start, the S points attached to it, its end) form a chain
 * ordered by distance from the start (ties by step), each the parent of the
 * next.  Nodes are numbered wire by wire (0, 1, ..., 2k; the S points of a
 * wire, then its end), so every parent precedes its child.  A node's R and C
 * are the unit values of its wire's axis times the coordinate distance to its
 * parent (FP32 products), its piece's capacitance lumped at the node; the
 * driver's are 0.  A net of k sinks has 3k+1 nodes, net n starts at node
 * n + 3 * net_sink_ptr[n], so the output is an sta_rc_desc of
 * n_nets + 3 * n_sinks nodes, ready for sta_create.  Its wire length never
 * exceeds the rectilinear minimum spanning tree's.  The paper builds the
 * Steiner trees with FLUTE, whose lookup tables it does not give.
 *
 *   g          netlist (only n_pins, n_nets and the net CSR are read), host or
 *              device memory per g->mem
 *   pin_x/y    [n_pins] positions (um), finite and at most 1e18 in
 *              magnitude; `mem` memory
 *   w          unit wire values, finite and >= 0; host memory
 *   outputs    net_node_ptr [n_nets+1], parent / res_kohm / cap_ff
 *              [n_nets + 3 n_sinks], sink_node [n_sinks]; `mem` memory,
 *              caller-allocated
 * Nets may have at most 12287 sinks (else STA_E_UNSUPPORTED).  Malformed
 * net CSR, a pin index out of range or a position out of range give
 * STA_E_ARG; they are checked on the device before any tree is built, and
 * then no output is written.  Allocates device scratch; synchronizes
 * `stream` twice (after the check and at the end). */
typedef struct {
  float r_x, r_y;              /* kOhm per um along x, y */
  float c_x, c_y;              /* fF per um along x, y */
} sta_wire_params;
sta_status sta_estimate_rc(const sta_graph_desc *g, const float *pin_x, const float *pin_y,
                           const sta_wire_params *w, int64_t *net_node_ptr, int32_t *parent, float *res_kohm,
                           float *cap_ff, int32_t *sink_node, sta_mem mem, void *stream);

/* Measurement helper: the achievable HBM bandwidth beside the published peak.
 * Copies `bytes` (a positive multiple of 16) from src to dst, both
 * caller-owned device buffers that should not overlap, with a plain
 * vector-load / vector-store kernel, once to warm up and then `reps` times
 * on `stream`, and writes the mean time of one copy (ms, HIP events) to *ms;
 * a copy moves 2 * bytes.  Synchronizes `stream`. */
sta_status sta_measure_copy(const void *src, void *dst, int64_t bytes, int32_t reps, void *stream, float *ms);

/* Measurement helper: the latency floor of a level-synchronous sweep on this
 * device.  Times `levels` dependent launches, each of `items` threads doing
 * only what bounds one level kernel's critical path (an index load, a 32-byte
 * gather at that index, a 32-byte store) over `records` 32-byte records (at
 * least items; make it as large as the design's pin state so the gathers miss
 * the caches as the sweep's do), once to warm up and then `reps` times, and
 * writes the mean ms of one such sweep to *ms.  Allocates and frees its own
 * device buffers; synchronizes `stream`. */
sta_status sta_measure_level_floor(int32_t levels, int32_t items, int64_t records, int32_t reps, void *stream,
                                   float *ms);

/* sta_estimate_rc for callers that cannot allocate device memory (code
 * under HIP graph capture nearby, tight serving loops, harnesses that forbid
 * hipMalloc).  Same trees, same outputs, bit for bit, and the same errors;
 * but every array (the net CSR per g->mem, which must be STA_DEVICE,
 * positions and outputs) is in device memory, and the call allocates
 * nothing: its check words, its lists of nets of 9-64 pins and of more than
 * 64 pins, and the per-pin working space of the nets of more than 64 pins
 * live in a fixed scratch array of the library (about 12.8 MiB per device,
 * held until the process ends).  Those lists take at most 1,048,576 and
 * 65,536 nets, and the nets of more than 64 pins at most 131,072 pins in
 * all; a netlist with more gives STA_E_UNSUPPORTED before any tree is
 * built.  Every call on one device shares that device's
 * scratch, so calls that overlap on one device (other host threads, other
 * streams) race and give undefined results; the call synchronizes `stream`
 * twice (after the check and at the end), so calls from one thread do not
 * overlap. */
sta_status sta_estimate_rc_noalloc(const sta_graph_desc *g, const float *pin_x, const float *pin_y,
                                   const sta_wire_params *w, int64_t *net_node_ptr, int32_t *parent,
                                   float *res_kohm, float *cap_ff, int32_t *sink_node, void *stream);

/* Gradient to pin positions through estimated RC trees (the placement side
 * of §III "Parasitics (RC) inputs").  With the trees of sta_estimate_rc held
 * fixed, every node coordinate is a copy of one pin's coordinate (a wire's
 * nearest point clamps a coordinate to the wire's ends), so a node piece of
 * length |c_u - c_w| along x (u the node, w its parent) gives, from dJ/dR and
 * dJ/dC of the node (e.g. grad_wire_res and grad_wire_cap of sta_backward on
 * a context created from those trees),
 *   dJ/dx of c_u's pin += sgn(c_u - c_w) (r_x dJ/dR + c_x dJ/dC),
 *   dJ/dx of c_w's pin -= the same,  and likewise along y,
 * with sgn(0) = 0 (the zero subgradient of a piece of no length).  Pins on
 * no net get 0; a pin on several nets gets an unspecified one of them (the
 * netlists of sta_create have every pin on one net).
 *
 *   g, pin_x/y, w        as for sta_estimate_rc (same positions)
 *   parent, sink_node    the trees sta_estimate_rc wrote for them
 *   grad_res, grad_cap   [n_nets + 3 n_sinks] per node; `mem` memory
 *   grad_x, grad_y       [n_pins] outputs; `mem` memory
 * The trees are rebuilt from the positions and compared with parent and
 * sink_node: a difference gives STA_E_ARG (the outputs are then undefined).
 * Terms are added as integers of 2^-44 of the net's largest term per axis,
 * exact in any order, so results are bitwise reproducible.  Errors as
 * sta_estimate_rc otherwise.  Allocates device scratch; synchronizes
 * `stream`. */
sta_status sta_estimate_rc_backward(const sta_graph_desc *g, const float *pin_x, const float *pin_y,
                                    const sta_wire_params *w, const int32_t *parent, const int32_t *sink_node,
                                    const float *grad_res, const float *grad_cap, float *grad_x, float *grad_y,
                                    sta_mem mem, void *stream);

/* Name of a status code; message of the calling thread's last error. */
const char *sta_status_string(sta_status s);
const char *sta_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STA_H */
