// Device layout shared by the host runtime (sta_host.cpp) and the kernels
// (sta_kernels.hip).  Everything is level-sorted once at create time:
//
//   driver slots  [0, n_drv): the PIs (ascending pin id), then the cells in
//                 ascending (cell level, type, output pin id), a level's
//                 high-fanout drivers last.  Slot x drives net x.
//                 Level l occupies [lvl_ptr[l], lvl_ptr[l+1]); level 0 = PIs.
//   sink slots    [0, n_sinks): net-major, sinks of net x in
//                 [sink_ptr[x], sink_ptr[x+1]) in the caller's sink order.
//   RC nodes      net-major in driver-slot order; node order inside a net is
//                 the caller's (small nets) or DFS preorder (big nets).
//
// Pin state is an AoS record of the four views: at[4] then slew[4] (32 B), so a
// fanin gather is one 32-byte access.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sta {

constexpr int kWave = 64;
constexpr int kMaxTypes = 256;
constexpr int kMaxAxis = 8;
constexpr int kSweepBlock = 256;            // 4 waves, each wave owns one chunk at a time
constexpr int kChunk = kWave;               // driver slots per sweep chunk
constexpr int kRcBlock = 256;               // one small net per thread
constexpr int kRcChunkNodes = 2048;         // RC nodes staged in LDS per block
constexpr int kRcAdjBlock = 128;            // the RC adjoint's blocks: nets and
constexpr int kRcAdjChunkNodes = 1024;      // nodes (its LDS holds eight arrays)
constexpr int kRcSortWindow = 4096;         // slots within which small nets are ordered by size
constexpr int kSmallNetMaxNodes = 255;      // parents fit in a byte
constexpr int kReduceBlocks = 128;
constexpr int kLevelCpb = 1;                // chunks per block of the full-update level kernels

struct alignas(32) PinState {
  float4 at;
  float4 slew;
};

// counters[] layout: kCtrReduce, then kDoneGroups completion counters per
// sweep phase (forward phases, then backward phases; the adjoint reuses the
// forward ones), then one ticket counter per phase
constexpr int kCtrReduce = 2;
constexpr int kCtrPhases = 4;
constexpr int kDoneGroups = 8;  // completion counters per phase (block b bumps group b % 8)
__host__ __device__ inline int n_counters(int n_phases) { return kCtrPhases + n_phases * (kDoneGroups + 1); }

// Sweep phases: int4 (kind, first item, item count, level); items are chunks
// or sink pieces of high-fanout drivers.
constexpr int kItemChunk = 0, kItemPiece = 1;
constexpr int kSplitSinks = 1024;  // a driver with more sinks gets its own chunk and sink pieces
constexpr int kPieceSinks = 512;   // sinks per piece (the chunk keeps the first piece)

// What the backward sweep gathers about a consumer cell, in one 32-byte record:
// its output RAT (written by the sweep), NLDM load (written by the RC pass) and
// library type (fixed).
struct __align__(32) ConsRec {
  float4 rat;
  float L;
  int32_t type;
  float pad0, pad1;
};

struct DevDesign {
  int32_t n_drv, n_pi, n_sinks, n_ep, n_cell_levels;
  int32_t n_types, nx, ny, tstride;
  int32_t n_chunks;
  int32_t max_in;             // most inputs of any library type

  // driver slots
  const int32_t *sink_ptr;    // [n_drv+1]
  const int32_t *rc_ptr;      // [n_drv] first RC node of each net (RC order, not monotone in slot)
  const int32_t *rc_order;    // [small nets] slot at each RC position
  const int32_t *rc_start;    // [small nets + 1] first node at each RC position (monotone)
  const int32_t *fanin_ptr;   // [n_drv+1] (empty for PIs)
  const int32_t *fanin_sink;  // sink slot of each cell input, fanin order
  const int32_t *cell_type;   // [n_drv] (-1 for PIs)
  const int32_t *drv_ep;      // [n_drv] endpoint index of a dangling endpoint, else -1
  const float4 *pi_at;        // [n_pi]
  const float4 *pi_slew;      // [n_pi]

  // sink slots
  const int32_t *sink_drv;    // [n_sinks] driver slot
  const int32_t *sink_cons;   // [n_sinks] consumer driver slot, or -1 - endpoint
  const int32_t *sink_node;   // [n_sinks] net-local RC node

  // RC nodes
  const uint8_t *rc_par8;     // net-local parent of a small-net node (root: 0, unused); 0 on wide nets
  const float *rc_pc;         // receiving pin caps lumped at each small-net node (fixed), summed in sink
                              // order; added into rc_cap whenever the wire caps are set
  const int2 *rc_sinks;       // [small nets] sink-slot range at each RC position
  const float *rc_res;
  const float *rc_cap;        // small nets: wire cap + rc_pc (one float sum); wide nets: the wire cap

  // endpoints
  const float4 *ep_rat;       // [n_ep]

  // library, packed per type: xa[nx] ya[ny] rdx[nx-1] rdy[ny-1] T[4][nx][ny]
  const float *tables;
  const int32_t *sense;

  // state written by the update
  float *L_net;               // [n_drv]
  float2 *dq;                 // [n_sinks] (Elmore delay, spread)
  PinState *drv_state;        // [n_drv]
  PinState *sink_state;       // [n_sinks]
  uint32_t *drv_crit;         // [n_drv] four int8 critical-fanin codes
  ConsRec *cons_rec;          // [n_drv] RAT / load / type per driver slot
  float4 *sink_rat;
  float4 *drv_slack, *sink_slack;
  float2 *ep_slack;           // [n_ep] (early, late)

  // smooth (differentiable) mode: gamma > 0 turns late arrival merges into
  // log-sum-exp; the adjoint writes the g_* arrays
  float gamma;
  int delay_model;              // 0 Elmore, 1 reduced-order (Arnoldi, two poles)
  int rc_cons_l;                // 1: the RC kernels also write cons_rec[].L (0 where the per-level
                                // backward writes each driver's whole record)
  const int32_t *ep_loc;        // [n_ep] endpoint pin: driver slot (>= 0) or -1 - sink slot
  float4 *g_sink;               // [n_sinks] dJ/d(late AT R, F), dJ/d(late slew R, F)
  float2 *g_dq;                 // [n_sinks] dJ/d(Elmore delay), dJ/d(spread q)
  float *g_load;                // [n_drv] dJ/d(NLDM load) of each cell output
  float2 *g_arc;                // [n_fanin] dJ/d(arc delay), late rise / fall output view
  float *g_cap;                 // [n_nodes] dJ/d(node cap), layout order
  float *g_res;                 // [n_nodes] dJ/d(segment resistance), layout order
  double *norm;                 // [2] WNS_g normalisation (max shift M, denominator)

  // sweep schedule
  const int4 *chunk_rec;        // [n_chunks] (first slot, end slot, first sink, end sink)
  const int4 *fanin4;           // [n_drv] input sink slots of each cell, -1 padded; NULL if a type has > 4 inputs
  const int4 *phases;           // forward, then backward, then adjoint phase lists
  int32_t n_ph_fwd, n_ph_bwd, n_ph_adj;
  const int4 *piece_rec;        // [n_pieces] (driver slot, first sink, end sink, owner chunk)
  const int2 *chunk_pieces;     // [n_chunks] (first piece, count) of a high-fanout driver's chunk
  const int2 *chunk_trange;     // [n_chunks] (lowest, highest) library type of the chunk's cells; (0, -1): none
  float4 *piece_rat;            // [n_pieces] each piece's merge of RAT_s - d
  uint32_t *counters;
};

// A wide RC net (more nodes than one lane handles), nodes in DFS preorder.
struct BigNet {
  int32_t x, m;       // driver slot, node count
  int64_t aux;        // offset into big_end / big_pc (one entry per node)
  int64_t scr;        // offset into the FP64 scratch (kBigScratch * (m + 1) doubles)
  int64_t nsp;        // offset into big_nsp (m + 1 entries: sinks of each node, CSR)
  int64_t egp;        // offset into big_egp (m + 2 entries): nodes whose subtree ends at p,
                      // listed in big_egl (aux-indexed, m entries) deepest first
  int32_t nblk;       // blocks sharing the net (segments of kWideSeg preorder nodes)
  int32_t tot;        // offset into the per-block scan totals
};
constexpr int kWideBlock = 1024;            // threads per wide-net block
constexpr int kWideSeg = 8192;              // preorder nodes per wide-net block
constexpr int kBigScratch = 11;

// Packed-table offsets for one type.
struct TabLayout {
  int nx, ny;
  __host__ __device__ int xa() const { return 0; }
  __host__ __device__ int ya() const { return nx; }
  __host__ __device__ int rdx() const { return nx + ny; }
  __host__ __device__ int rdy() const { return nx + ny + nx - 1; }
  __host__ __device__ int tab(int k) const { return 2 * nx + 2 * ny - 2 + k * nx * ny; }
  __host__ __device__ int stride() const { return 2 * nx + 2 * ny - 2 + 4 * nx * ny; }
};

// Launch wrappers (sta_kernels.hip).  All return hipError_t of the launch.
// Wide-net arrays handed to the RC kernels.
struct WideNets {
  const BigNet *big;
  int n_big;
  const int2 *blk;       // [n_blk] (net, segment) of each launched block
  int n_blk;
  const int32_t *end, *nsp, *nsl, *egp, *egl;
  const float *pc;
  double *scratch;
  double *tot;           // per-block scan totals
  uint32_t *sync;        // [2 n_big] barrier arrivals and departures per net
};

// incremental update: per-sweep queues of the chunks and pieces to recompute
constexpr int kIncBlocks = 64;    // default grid of the queued sweeps
constexpr int kIncMaxItems = 16;  // a queued sweep hands over at the first phase with more items
struct IncArgs {
  uint32_t *flag;            // [2 n_chunks] queued for the forward / backward sweep
  uint32_t *cnt;             // [n_ph_fwd + n_ph_bwd] queue length of each phase
  int32_t *wl_c;             // [2 n_chunks] queued chunks, each phase's at its first chunk id
  int32_t *wl_p;             // [2 n_pieces] queued pieces, likewise
  const int32_t *chunk_of;   // [n_drv] chunk of each driver slot
  const int32_t *sink_cc;    // [n_sinks] chunk of the sink's consumer, -1 at an endpoint
  const int4 *fanin_cc;      // [n_drv] chunks of the cell's inline input sinks' drivers; NULL without inline fanins
  const int2 *chunk_ph;      // [n_chunks] (forward phase, backward phase index) of each chunk
  uint8_t *rcd;              // [n_drv] 1: the driver's net was recomputed
  uint32_t *rc_flag;         // [n_rc_chunks] 1: the RC chunk holds a changed net
  uint32_t *wide_flag;       // [n_big] 1: the wide net changed
  const int32_t *net_slot;   // [n_nets] caller net id -> driver slot
  const int32_t *slot_rc;    // [n_drv] RC chunk of the slot's net, or -1 - wide-net index
  int32_t *stop;             // [2] phase where the queued forward / backward sweep stopped
  int n_chunks, n_pieces;
};
hipError_t launch_inc_maps(const DevDesign &D, const int32_t *chunk_of, int32_t *sink_cc, int4 *fanin_cc,
                           hipStream_t s);
hipError_t launch_inc_seed(const DevDesign &D, const IncArgs &I, const int32_t *nets, int n, hipStream_t s);
// queued sweeps: stop (and record the phase) at the first phase with more than max_items items
hipError_t launch_inc_forward(const DevDesign &D, const IncArgs &I, int grid, int max_items, hipStream_t s);
hipError_t launch_inc_backward(const DevDesign &D, const IncArgs &I, int grid, int max_items, hipStream_t s);
hipError_t launch_inc_queues(const DevDesign &D, const IncArgs &I, bool backward, hipStream_t s);
// flagged per-phase continuation (one launch per phase; unflagged chunks return at once)
hipError_t launch_inc_forward_phase(const DevDesign &D, const IncArgs &I, int4 phase, int4 reg, hipStream_t s);
hipError_t launch_inc_backward_phase(const DevDesign &D, const IncArgs &I, int4 phase, hipStream_t s);
int inc_blocks_per_cu(size_t lds_bytes);
// only: optional per-chunk / per-wide-net flags, unflagged ones skipped;
// the first block also clears the sweep and reduction counters unless
// clear_counters is false (a later launch of one update's RC pass in parts)
hipError_t launch_rc(const DevDesign &D, const int2 *chunks, int n_chunks, hipStream_t s,
                     const uint32_t *only = nullptr, bool clear_counters = true);
hipError_t launch_rc_wide(const DevDesign &D, const WideNets &W, hipStream_t s, const uint32_t *only = nullptr);
hipError_t launch_rc_adjoint_wide(const DevDesign &D, const WideNets &W, hipStream_t s);
// Persistent sweeps: with coop, the level-major static schedule on a
// cooperative (co-resident) grid; otherwise the ticket schedule.
hipError_t launch_forward(const DevDesign &D, int persistent_grid, bool coop, hipStream_t s);
// reg: the level's first slot and the end of its slots in regular (kChunk-slot) chunks
hipError_t launch_forward_phase(const DevDesign &D, int4 phase, int4 reg, hipStream_t s);
hipError_t launch_backward(const DevDesign &D, int persistent_grid, bool coop, hipStream_t s);
// Dataflow sweeps (one cooperative launch per sweep, per-item completion
// flags instead of level barriers): the items of one sweep in order and the
// producer items each item waits for.
struct FlowArgs {
  const int2 *items;         // [n_items] (kind, chunk or piece id) in sweep order
  int n_items;
  uint32_t *flag;            // [n_chunks + n_pieces] this sweep's flags: chunk c at c, piece j at n_chunks + j
  const int4 *fin_item;      // [n_drv] forward item producing each inline input sink (-1: none)
  const int32_t *sink_item;  // [n_sinks] backward item writing each sink's RAT (-1: an endpoint)
  uint32_t epoch;            // the value a published item's flag holds in this update
  uint32_t *err;             // raised if a wait gave up (results then invalid)
};
hipError_t launch_flow(const DevDesign &D, const FlowArgs &F, bool fwd, int grid, hipStream_t s);
int flow_blocks_per_cu(const DevDesign &D);  // co-resident blocks of the flow kernels per CU

// per-level backward (RATs pushed to the inputs by their consumers); reg as
// for the forward: the level's first slot and the end of its regular chunks
hipError_t launch_backward_phase(const DevDesign &D, int4 phase, int4 reg, hipStream_t s);
hipError_t launch_reset_counters(uint32_t *counters, int n, hipStream_t s);
// plain copy of n16 16-byte elements (bandwidth measurement)
hipError_t launch_copy4(const void *src, void *dst, int64_t n16, hipStream_t s);
// one level-shaped launch: dst[off + i] = src[idx[off + i]] (+1 on one field)
// for i < n, 32-byte records (latency floor measurement)
hipError_t launch_level_floor(const int32_t *idx, const void *src, void *dst, int n, int off, hipStream_t s);
// keys (when not NULL): [2 n_ep] endpoint sort keys, (early/late, slack) with
// early/late above the slack bits, and their endpoint indices in vals
hipError_t launch_reduce_smooth(const DevDesign &D, double *partials, double *out, uint64_t *keys,
                                int32_t *vals, hipStream_t s);
hipError_t launch_adjoint_phase(const DevDesign &D, float g_tns, float g_wns, int4 phase, int lib_f4, hipStream_t s);
// res: also dJ/dR (D.g_res) for the small nets; the wide nets always write it
hipError_t launch_rc_adjoint(const DevDesign &D, const int2 *chunks, int n_chunks, bool res, hipStream_t s);
hipError_t launch_scatter_grads(const DevDesign &D, const int32_t *node_src, int64_t n_nodes, float *grad_cap,
                                float *grad_res, const int32_t *pin_loc, int n_pins, float *grad_load,
                                const int32_t *arc_src, int n_arcs, float4 *grad_arc, hipStream_t s);
hipError_t launch_reduce(const DevDesign &D, double *partials, double *out, uint64_t *keys,
                         int32_t *vals, hipStream_t s);
hipError_t sort_endpoints(void *temp, size_t temp_bytes, const uint32_t *keys_in,
                          uint32_t *keys_out, const int32_t *vals_in, int32_t *vals_out, int n,
                          hipStream_t s);
size_t sort_temp_bytes(int n);
// batches: per-design reductions (out[d][4] = early WNS, late WNS, early TNS,
// late TNS) and the endpoint sort keys (early/late, design, slack), the design
// in dbits bits above the slack
hipError_t launch_reduce_batch(const DevDesign &D, const int32_t *ep_off, int n_designs, int dbits,
                               double *partials, double *out, uint64_t *keys, int32_t *vals, hipStream_t s);
size_t sort_temp_bytes64(int n, int end_bit);
hipError_t sort_endpoints64(void *temp, size_t temp_bytes, const uint64_t *keys_in, uint64_t *keys_out,
                            const int32_t *vals_in, int32_t *vals_out, int n, int end_bit, hipStream_t s);
int sweep_blocks_per_cu(size_t lds_bytes);
int coop_blocks_per_cu(size_t lds_bytes);
size_t sweep_lds_bytes(const DevDesign &D, int chunks_per_block = 1);

// levelization
hipError_t launch_level_init(int32_t *pending, int32_t *cell_level, const int32_t *cell_nin,
                             int n_cells, hipStream_t s);
hipError_t launch_level_step(const int32_t *frontier, int n_front, int lvl,
                             const int32_t *net_of_drv_pin, const int32_t *net_sink_ptr,
                             const int32_t *net_sink_pin, const int32_t *cell_of_in_pin,
                             const int32_t *cell_out_pin, int32_t *pending, int32_t *cell_level,
                             int32_t *next, uint32_t *next_count, hipStream_t s);
hipError_t launch_pin_levels(const int32_t *pin_kind, const int32_t *cell_of_pin,
                             const int32_t *cell_level, const int32_t *drv_of_sink_pin,
                             int32_t *pin_level, int n_pins, hipStream_t s);
hipError_t sort_levels(void *temp, size_t temp_bytes, const int32_t *keys_in, int32_t *keys_out,
                       const int32_t *vals_in, int32_t *vals_out, int n, int key_bits,
                       hipStream_t s);
size_t level_sort_temp_bytes(int n);
hipError_t launch_iota(int32_t *a, int n, hipStream_t s);

// top-k path report: per selected endpoint, a best-first search over
// deviations from the critical fanins (one thread per endpoint)
struct PathArgs {
  const int32_t *eps;   // [n_eps] endpoint indices, ascending endpoint slack
  int n_eps, el, m, lmax;
  float thr;
  int4 *items;          // [m][n_eps] queue items (key bits, sequence, parent << 24 | position, node), or
                        // null: the queues are in LDS
  int32_t *nodes;       // [n_eps * m * lmax] path nodes, endpoint first
  int32_t *plen;        // [n_eps * m] path lengths (0: none)
  float *pkey;          // [n_eps * m] path slacks
  const int32_t *drv_pin, *sink_pin;  // slot -> caller pin
};
size_t paths_queue_lds_bytes(const DevDesign &D, int m);  // library + LDS queues of one block
hipError_t launch_paths_count(const DevDesign &D, const int32_t *ord, int cand, int el, float thr, int32_t *out,
                              hipStream_t s);
hipError_t launch_paths_enum(const DevDesign &D, const PathArgs &A, hipStream_t s);
hipError_t launch_paths_keys(const PathArgs &A, uint32_t *keys, int32_t *vals, hipStream_t s);
hipError_t launch_paths_emit(const DevDesign &D, const PathArgs &A, const int32_t *sel, int n_sel,
                             const int32_t *ptr, int32_t *pin, int8_t *rf, float *slack, int32_t *ep,
                             hipStream_t s);
hipError_t launch_paths_lengths(const PathArgs &A, const int32_t *sel, int n_sel, int32_t *len, hipStream_t s);
hipError_t exclusive_sum(void *temp, size_t &temp_bytes, const int32_t *in, int32_t *out, int n, hipStream_t s);

// reports and inputs
hipError_t launch_report_pins(const DevDesign &D, const int32_t *pin_loc, int n_pins, float4 *at,
                              float4 *slew, float4 *rat, uint32_t *crit, float4 *slack,
                              hipStream_t s);
hipError_t launch_report_rc(const DevDesign &D, const int32_t *net_slot, int n_nets,
                            const int32_t *sink_slot, int n_sinks, float *net_load,
                            float *sink_delay, float *sink_spread, hipStream_t s);
hipError_t launch_permute_caps(const float *src, const int32_t *node_src, float *dst, int64_t n,
                               const float *pc, int64_t n_small, hipStream_t s);

}  // namespace sta
