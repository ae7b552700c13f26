// HIP kernels of the static-timing hot path, written for CDNA4 (gfx950, wave64).
//
//   k_rc           Elmore delay / impulse spread / net load (§III "Delay models"):
//                  small nets one per lane with the block's nodes staged in LDS,
//                  wide nets one per block with FP64 preorder scans
//   k_forward      levelized AT/slew sweep with NLDM lookups from LDS tables
//                  (§I graph-based STA; Table I NLDM)
//   k_backward     levelized RAT sweep, per-pin slack     (§III "Report options")
//   k_reduce       endpoint WNS/TNS in FP64, fixed reduction order
//
// A sweep work item ("chunk") is one wavefront over 64 consecutive driver slots
// of one level: lanes compute the drivers, then the wave walks the contiguous
// range of the drivers' sinks.  In the persistent schedule waves take chunks
// from a ticket counter in level order and wait on per-level completion
// counters, so any grid size is deadlock-free (a ticket holder is running).
#include <hipcub/hipcub.hpp>

#include "sta_internal.h"

namespace sta {

namespace {

constexpr float kInf = __builtin_inff();

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Monotone float <-> int map for integer atomic min/max (signed compare).
__device__ __forceinline__ int f2key(float f) {
  int k = __float_as_int(f);
  return k ^ ((k >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float key2f(int k) { return __int_as_float(k ^ ((k >> 31) & 0x7fffffff)); }
// Monotone float -> unsigned map for radix sorting ascending.
__device__ __forceinline__ uint32_t f2ukey(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ bool arc_maps(int sense, int ri, int ro) {
  return sense == 2 || (sense == 0 ? ri == ro : ri != ro);
}

struct AxisPos {
  int i;
  float t;
};

// Segment = largest i with ax[i] <= X, kept in [0, n-2] (off-table points
// extrapolate along the boundary segment); t = (X - ax[i]) / (ax[i+1] - ax[i]).
__device__ __forceinline__ AxisPos axis_find(const float *ax, const float *rd, int n, float X) {
  int i = 0;
#pragma unroll
  for (int m = 1; m < kMaxAxis - 1; ++m)
    if (m <= n - 2 && ax[m] <= X) i = m;
  return {i, (X - ax[i]) * rd[i]};
}

__device__ __forceinline__ float bilerp(const float *T, int ny, AxisPos px, AxisPos py) {
  const float *r0 = T + px.i * ny + py.i;
  const float *r1 = r0 + ny;
  float a = r0[0] + px.t * (r1[0] - r0[0]);
  float b = r0[1] + px.t * (r1[1] - r0[1]);
  return a + py.t * (b - a);
}

__device__ __forceinline__ float4 slack4(float4 at, float4 rat) {
  return make_float4(at.x - rat.x, at.y - rat.y, rat.z - at.z, rat.w - at.w);
}

__device__ __forceinline__ float2 ep_slack2(float4 at, float4 rat) {
  return make_float2(fminf(at.x - rat.x, at.y - rat.y), fminf(rat.z - at.z, rat.w - at.w));
}

// LDS image of the library: packed tables then the sense codes.
struct LdsLib {
  const float *tab;
  const int *sense;
};

__device__ LdsLib load_lib(const DevDesign &D, unsigned char *smem) {
  float *tab = reinterpret_cast<float *>(smem);
  const int ntab = D.n_types * D.tstride;
  for (int i = threadIdx.x; i < ntab; i += blockDim.x) tab[i] = D.tables[i];
  int *sense = reinterpret_cast<int *>(tab + ntab);
  for (int i = threadIdx.x; i < D.n_types; i += blockDim.x) sense[i] = D.sense[i];
  return {tab, sense};
}

__host__ __device__ inline size_t lib_lds_bytes(int n_types, int tstride) {
  size_t b = (size_t)n_types * tstride * 4 + (size_t)n_types * 4;
  return (b + 31) & ~(size_t)31;
}

// ------------------------------------------------------------ forward

// Arrival/slew of one cell output: merge over fanin arcs of AT_in + delay
// (late max, early min), slew merged the same way independent of the AT
// winner; the critical code is 2*fanin + input transition of the AT winner,
// ties kept by the earlier candidate.
__device__ __forceinline__ void cell_forward(const DevDesign &D, const LdsLib &lib, int x,
                                             PinState &out, uint32_t &crit) {
  const int t = D.cell_type[x];
  const int sense = lib.sense[t];
  const float L = D.L_net[x];
  const TabLayout lay{D.nx, D.ny};
  const float *tb = lib.tab + t * D.tstride;
  const AxisPos py = axis_find(tb + lay.ya(), tb + lay.rdy(), D.ny, L);
  float at[4] = {kInf, kInf, -kInf, -kInf};
  float sl[4] = {kInf, kInf, -kInf, -kInf};
  int cr[4] = {-1, -1, -1, -1};
  const int f0 = D.fanin_ptr[x], f1 = D.fanin_ptr[x + 1];
  for (int f = f0; f < f1; ++f) {
    const PinState in = D.sink_state[D.fanin_sink[f]];
    const float ia[4] = {in.at.x, in.at.y, in.at.z, in.at.w};
    const float is[4] = {in.slew.x, in.slew.y, in.slew.z, in.slew.w};
    const int k2 = (f - f0) * 2;
#pragma unroll
    for (int el = 0; el < 2; ++el) {
#pragma unroll
      for (int ri = 0; ri < 2; ++ri) {
        const int vi = el * 2 + ri;
        const AxisPos px = axis_find(tb + lay.xa(), tb + lay.rdx(), D.nx, is[vi]);
#pragma unroll
        for (int ro = 0; ro < 2; ++ro) {
          if (!arc_maps(sense, ri, ro)) continue;
          const int vo = el * 2 + ro;
          const float dl = bilerp(tb + lay.tab(ro), D.ny, px, py);
          const float os = bilerp(tb + lay.tab(2 + ro), D.ny, px, py);
          const float cand = ia[vi] + dl;
          if (el ? cand > at[vo] : cand < at[vo]) {
            at[vo] = cand;
            cr[vo] = k2 + ri;
          }
          sl[vo] = el ? fmaxf(sl[vo], os) : fminf(sl[vo], os);
        }
      }
    }
  }
  out.at = make_float4(at[0], at[1], at[2], at[3]);
  out.slew = make_float4(sl[0], sl[1], sl[2], sl[3]);
  crit = (uint32_t)(cr[0] & 0xff) | ((uint32_t)(cr[1] & 0xff) << 8) |
         ((uint32_t)(cr[2] & 0xff) << 16) | ((uint32_t)(cr[3] & 0xff) << 24);
}

// One chunk: the 64 drivers, then every sink of their nets
// (AT_s = AT_drv + d, slew_s = sqrt(slew_drv^2 + q)).
__device__ void fwd_chunk(const DevDesign &D, const LdsLib &lib, PinState *wst, int c) {
  const int lane = lane_id();
  const int x0 = D.chunk_start[c], x1 = D.chunk_start[c + 1];
  const int x = x0 + lane;
  if (x < x1) {
    PinState st;
    uint32_t crit = 0xffffffffu;
    if (x < D.n_pi) {
      st.at = D.pi_at[x];
      st.slew = D.pi_slew[x];
    } else {
      cell_forward(D, lib, x, st, crit);
    }
    D.drv_state[x] = st;
    D.drv_crit[x] = crit;
    wst[lane] = st;
  }
  wave_sync();
  const int s0 = D.sink_ptr[x0], s1 = D.sink_ptr[x1];
  for (int s = s0 + lane; s < s1; s += kWave) {
    const PinState ds = wst[D.sink_drv[s] - x0];
    const float2 w = D.dq[s];
    PinState o;
    o.at = make_float4(ds.at.x + w.x, ds.at.y + w.x, ds.at.z + w.x, ds.at.w + w.x);
    o.slew = make_float4(sqrtf(ds.slew.x * ds.slew.x + w.y), sqrtf(ds.slew.y * ds.slew.y + w.y),
                         sqrtf(ds.slew.z * ds.slew.z + w.y), sqrtf(ds.slew.w * ds.slew.w + w.y));
    D.sink_state[s] = o;
  }
  wave_sync();
}

// The persistent loops contain no lane-divergent branch: every lane issues the
// counter atomics (lane 0 adds 1, the others 0, which the compiler folds into
// one wave-level atomic) and the ticket / polled count are broadcast with
// readfirstlane, so every loop exit is a scalar branch and the 64 lanes always
// iterate together.  (With `if (lane == 0) atomic` at both ends of the loop,
// jump threading merged the two regions into a lane-0-only path and the
// other lanes re-entered the loop without a ticket.)
__device__ __forceinline__ void wait_count(uint32_t *ctr, uint32_t target) {
  for (;;) {
    const uint32_t v = __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__builtin_amdgcn_readfirstlane(v) >= target) break;
    __builtin_amdgcn_s_sleep(1);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ __forceinline__ int take_ticket(uint32_t *ctr) {
  const uint32_t old = atomicAdd(ctr, lane_id() == 0 ? 1u : 0u);
  return (int)__builtin_amdgcn_readfirstlane(old);
}

__device__ __forceinline__ void signal_done(uint32_t *ctr) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __hip_atomic_fetch_add(ctr, lane_id() == 0 ? 1u : 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kSweepBlock) void k_forward(DevDesign D, int c0, int c1, int persistent) {
  extern __shared__ __align__(32) unsigned char smem[];
  const LdsLib lib = load_lib(D, smem);
  PinState *wst = reinterpret_cast<PinState *>(smem + lib_lds_bytes(D.n_types, D.tstride)) +
                  (threadIdx.x / kWave) * kWave;
  __syncthreads();
  if (persistent) {
    uint32_t *done = D.counters + kCtrLevels;
    for (;;) {
      const int c = take_ticket(D.counters + kCtrFwdTicket);
      if (c >= D.n_chunks) break;
      const int lvl = D.chunk_level[c];
      if (lvl > 0) wait_count(done + lvl - 1, (uint32_t)D.level_nchunks[lvl - 1]);
      fwd_chunk(D, lib, wst, c);
      signal_done(done + lvl);
    }
  } else {
    const int c = c0 + blockIdx.x * (kSweepBlock / kWave) + threadIdx.x / kWave;
    if (c < c1) fwd_chunk(D, lib, wst, c);
  }
}

// ------------------------------------------------------------ backward

// One chunk: every sink of the 64 drivers gets RAT from its consumer (the
// consumer cell's output RAT minus the recomputed arc delay, min for late and
// max for early over the output transitions the input reaches) or from its
// endpoint constraint; the drivers merge RAT_s - d over their sinks.
__device__ void bwd_chunk(const DevDesign &D, const LdsLib &lib, int *wacc, int c) {
  const int lane = lane_id();
  const int x0 = D.chunk_start[c], x1 = D.chunk_start[c + 1];
  const int x = x0 + lane;
  if (x < x1) {
    float4 init = make_float4(-kInf, -kInf, kInf, kInf);
    const int e = D.drv_ep[x];
    if (e >= 0) init = D.ep_rat[e];
    wacc[lane * 4 + 0] = f2key(init.x);
    wacc[lane * 4 + 1] = f2key(init.y);
    wacc[lane * 4 + 2] = f2key(init.z);
    wacc[lane * 4 + 3] = f2key(init.w);
  }
  wave_sync();
  const TabLayout lay{D.nx, D.ny};
  const int s0 = D.sink_ptr[x0], s1 = D.sink_ptr[x1];
  for (int s = s0 + lane; s < s1; s += kWave) {
    const PinState ss = D.sink_state[s];
    const int cons = D.sink_cons[s];
    float4 R;
    if (cons < 0) {
      const int e = -1 - cons;
      R = D.ep_rat[e];
      D.ep_slack[e] = ep_slack2(ss.at, R);
    } else {
      const int t = D.cell_type[cons];
      const int sense = lib.sense[t];
      const float L = D.L_net[cons];
      const float4 Ro4 = D.drv_rat[cons];
      const float Ro[4] = {Ro4.x, Ro4.y, Ro4.z, Ro4.w};
      const float is[4] = {ss.slew.x, ss.slew.y, ss.slew.z, ss.slew.w};
      const float *tb = lib.tab + t * D.tstride;
      const AxisPos py = axis_find(tb + lay.ya(), tb + lay.rdy(), D.ny, L);
      float r[4];
#pragma unroll
      for (int el = 0; el < 2; ++el) {
#pragma unroll
        for (int ri = 0; ri < 2; ++ri) {
          const int vi = el * 2 + ri;
          const AxisPos px = axis_find(tb + lay.xa(), tb + lay.rdx(), D.nx, is[vi]);
          float best = el ? kInf : -kInf;
#pragma unroll
          for (int ro = 0; ro < 2; ++ro) {
            if (!arc_maps(sense, ri, ro)) continue;
            const float cand = Ro[el * 2 + ro] - bilerp(tb + lay.tab(ro), D.ny, px, py);
            best = el ? fminf(best, cand) : fmaxf(best, cand);
          }
          r[vi] = best;
        }
      }
      R = make_float4(r[0], r[1], r[2], r[3]);
    }
    D.sink_rat[s] = R;
    D.sink_slack[s] = slack4(ss.at, R);
    const float d = D.dq[s].x;
    int *acc = wacc + (D.sink_drv[s] - x0) * 4;
    atomicMax(acc + 0, f2key(R.x - d));
    atomicMax(acc + 1, f2key(R.y - d));
    atomicMin(acc + 2, f2key(R.z - d));
    atomicMin(acc + 3, f2key(R.w - d));
  }
  wave_sync();
  if (x < x1) {
    const float4 R = make_float4(key2f(wacc[lane * 4 + 0]), key2f(wacc[lane * 4 + 1]),
                                 key2f(wacc[lane * 4 + 2]), key2f(wacc[lane * 4 + 3]));
    const float4 A = D.drv_state[x].at;
    D.drv_rat[x] = R;
    D.drv_slack[x] = slack4(A, R);
    const int e = D.drv_ep[x];
    if (e >= 0) D.ep_slack[e] = ep_slack2(A, R);
  }
  wave_sync();
}

__global__ __launch_bounds__(kSweepBlock) void k_backward(DevDesign D, int c0, int c1, int persistent) {
  extern __shared__ __align__(32) unsigned char smem[];
  const LdsLib lib = load_lib(D, smem);
  int *wacc = reinterpret_cast<int *>(smem + lib_lds_bytes(D.n_types, D.tstride)) +
              (threadIdx.x / kWave) * kWave * 4;
  __syncthreads();
  if (persistent) {
    uint32_t *done = D.counters + kCtrLevels + D.n_cell_levels + 1;
    for (;;) {
      const int t = take_ticket(D.counters + kCtrBwdTicket);
      if (t >= D.n_chunks) break;
      const int c = D.n_chunks - 1 - t;
      const int lvl = D.chunk_level[c];
      if (lvl < D.n_cell_levels) wait_count(done + lvl + 1, (uint32_t)D.level_nchunks[lvl + 1]);
      bwd_chunk(D, lib, wacc, c);
      signal_done(done + lvl);
    }
  } else {
    const int c = c0 + blockIdx.x * (kSweepBlock / kWave) + threadIdx.x / kWave;
    if (c < c1) bwd_chunk(D, lib, wacc, c);
  }
}

// ------------------------------------------------------------------ RC

// Elmore recursions on one tree held in LDS (nodes b..b+m-1, parent < child):
//   load = subtree sum of C^ (bottom-up), d = d(parent) + R load (top-down),
//   ld = subtree sum of C^ d (bottom-up), m2 = m2(parent) + R ld (top-down).
// On return A holds m2 and B holds d; the result is the root load.
__device__ __forceinline__ float rc_tree_lds(const uint8_t *par, const float *R, const float *C,
                                             float *A, float *B, int b, int m) {
  for (int k = 0; k < m; ++k) A[b + k] = C[b + k];
  for (int k = m - 1; k >= 1; --k) A[b + par[b + k]] += A[b + k];
  const float load = A[b];
  B[b] = 0.0f;
  for (int k = 1; k < m; ++k) B[b + k] = B[b + par[b + k]] + R[b + k] * A[b + k];
  for (int k = 0; k < m; ++k) A[b + k] = C[b + k] * B[b + k];
  for (int k = m - 1; k >= 1; --k) A[b + par[b + k]] += A[b + k];
  A[b] = 0.0f;
  for (int k = 1; k < m; ++k) A[b + k] = A[b + par[b + k]] + R[b + k] * A[b + k];
  return load;
}

// ---- wide nets: block per net, FP64 scans over the DFS preorder ----------
//
// In preorder the subtree of node k is the index range [k, end_k), so
//   load_k = sum of C^ over [k, end_k)           = P[end_k] - P[k]   (P = exclusive scan of C^)
//   ld_k   = sum of C^ d over [k, end_k)         (same with C^ d)
// and a path sum over the ancestors-or-self of k (the a with a <= k < end_a) is
//   sum_{p <= k} (w_p - E_p),   E_p = sum of w_a over the nodes a with end_a = p,
// which gives d (w = R load) and m2 (w = R ld).  The nodes with end_a = p form a
// chain upward from p - 1, so E_p is gathered by walking that chain (each node is
// visited once overall) in a fixed order.  FP64 keeps the prefix differences
// exact to far below FP32 resolution.

// Block-wide scan of in[0, n) into out (may alias in): inclusive, or exclusive
// with out[n] = total.  Tiles of kScanPer consecutive elements per thread.
constexpr int kScanPer = 8;

__device__ void block_scan(const double *in, double *out, int n, bool exclusive, double *s_w) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int nw = blockDim.x / kWave;
  const int tile = blockDim.x * kScanPer;
  double carry = 0.0;
  for (int base = 0; base < n; base += tile) {
    const int i0 = base + tid * kScanPer;
    double x[kScanPer];
    double run = 0.0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      x[j] = (i0 + j < n) ? in[i0 + j] : 0.0;
      run += x[j];
    }
    double incl = run;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const double y = __shfl_up(incl, off);
      if (lane >= off) incl += y;
    }
    double excl = __shfl_up(incl, 1);
    if (lane == 0) excl = 0.0;
    if (lane == kWave - 1) s_w[wid] = incl;
    __syncthreads();
    if (tid == 0) {
      double acc = 0.0;
      for (int w = 0; w < nw; ++w) {
        const double t = s_w[w];
        s_w[w] = acc;
        acc += t;
      }
      s_w[nw] = acc;
    }
    __syncthreads();
    double pre = carry + s_w[wid] + excl;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      if (i0 + j < n) out[i0 + j] = exclusive ? pre : pre + x[j];
      pre += x[j];
    }
    carry += s_w[nw];
    __syncthreads();
  }
  if (exclusive && threadIdx.x == 0) out[n] = carry;
  __syncthreads();
}

// Y[p] = X[p] - sum of X[a] over the nodes a whose subtree ends at p.
__device__ void euler_terms(const double *X, double *Y, const int32_t *par, const int32_t *end, int m) {
  for (int p = threadIdx.x; p < m; p += blockDim.x) {
    double e = 0.0;
    for (int a = p - 1; a >= 0 && end[a] == p; a = par[a]) e += X[a];
    Y[p] = X[p] - e;
  }
  __syncthreads();
}

__device__ void rc_wide_net(const DevDesign &D, const BigNet &B, const int32_t *big_end, const float *big_pc,
                            double *scratch, double *s_w) {
  const int x = B.x, m = B.m;
  const int k0 = D.rc_ptr[x];
  const int32_t *par = D.rc_parent + k0;
  const float *R = D.rc_res + k0;
  const float *Cw = D.rc_cap + k0;
  const int32_t *end = big_end + B.aux;
  const float *pc = big_pc + B.aux;
  double *A = scratch + B.scr, *P = A + (m + 1), *X = P + (m + 1), *Y = X + (m + 1);
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int k = tid; k < m; k += nt) A[k] = (double)Cw[k] + (double)pc[k];  // C^
  __syncthreads();
  block_scan(A, P, m, true, s_w);                                          // P: prefix of C^
  const double total = P[m];
  for (int k = tid; k < m; k += nt) X[k] = k ? (double)R[k] * (P[end[k]] - P[k]) : 0.0;  // R load
  __syncthreads();
  euler_terms(X, Y, par, end, m);
  block_scan(Y, Y, m, false, s_w);                                         // Y: d
  for (int k = tid; k < m; k += nt) X[k] = A[k] * Y[k];                    // C^ d
  __syncthreads();
  block_scan(X, P, m, true, s_w);                                          // P: prefix of C^ d
  for (int k = tid; k < m; k += nt) X[k] = k ? (double)R[k] * (P[end[k]] - P[k]) : 0.0;  // R ld
  __syncthreads();
  euler_terms(X, A, par, end, m);
  block_scan(A, A, m, false, s_w);                                         // A: m2
  if (tid == 0) D.L_net[x] = (float)total;
  for (int s = D.sink_ptr[x] + tid; s < D.sink_ptr[x + 1]; s += nt) {
    const int k = D.sink_node[s];
    const double d = Y[k];
    D.dq[s] = make_float2((float)d, (float)fmax(0.0, 2.0 * A[k] - d * d));
  }
}

// One launch for the whole RC pass: blocks [0, n_big) each take a wide net
// (dispatched first, so they overlap the small-net blocks), the rest take a
// chunk of <= 256 small nets (<= kRcChunkNodes nodes): coalesced staging of
// parent/R/C into LDS, one net per thread, coalesced sink output.  Block 0 also
// clears the sweep counters for the launches that follow.
__global__ __launch_bounds__(kRcBlock) void k_rc(DevDesign D, const int2 *chunks, int n_chunks,
                                                 const BigNet *big, int n_big, const int32_t *big_end,
                                                 const float *big_pc, double *scratch, uint32_t *counters,
                                                 int n_counters) {
  __shared__ uint8_t s_par[kRcChunkNodes];
  __shared__ float s_R[kRcChunkNodes], s_C[kRcChunkNodes], s_A[kRcChunkNodes], s_B[kRcChunkNodes];
  __shared__ int s_base[kRcBlock + 1];
  __shared__ double s_w[kRcBlock / kWave + 1];
  const int tid = threadIdx.x;
  if (blockIdx.x == 0)
    for (int i = tid; i < n_counters; i += kRcBlock) counters[i] = 0u;
  if ((int)blockIdx.x < n_big) {
    rc_wide_net(D, big[blockIdx.x], big_end, big_pc, scratch, s_w);
    return;
  }
  const int ci = blockIdx.x - n_big;
  if (ci >= n_chunks) return;
  const int2 ch = chunks[ci];
  const int x0 = ch.x, x1 = ch.y;
  const int k0 = D.rc_ptr[x0], nk = D.rc_ptr[x1] - k0;
  for (int i = tid; i < nk; i += kRcBlock) {
    s_par[i] = (uint8_t)D.rc_parent[k0 + i];
    s_R[i] = D.rc_res[k0 + i];
    s_C[i] = D.rc_cap[k0 + i];
  }
  for (int i = tid; i <= x1 - x0; i += kRcBlock) s_base[i] = D.rc_ptr[x0 + i] - k0;
  __syncthreads();
  const int x = x0 + tid;
  if (x < x1) {
    const int b = s_base[tid], m = s_base[tid + 1] - b;
    for (int s = D.sink_ptr[x]; s < D.sink_ptr[x + 1]; ++s) s_C[b + D.sink_node[s]] += D.sink_pincap[s];
    D.L_net[x] = rc_tree_lds(s_par, s_R, s_C, s_A, s_B, b, m);
  }
  __syncthreads();
  const int s0 = D.sink_ptr[x0], s1 = D.sink_ptr[x1];
  for (int s = s0 + tid; s < s1; s += kRcBlock) {
    const int k = s_base[D.sink_drv[s] - x0] + D.sink_node[s];
    const float d = s_B[k];
    D.dq[s] = make_float2(d, fmaxf(0.0f, 2.0f * s_A[k] - d * d));
  }
}

// ------------------------------------------------------------ reduction

// WNS = min(0, min slack), TNS = sum of negative slacks, per early/late, in
// FP64 with a fixed partition and tree so results are bitwise reproducible;
// also writes the radix-sort keys of the endpoint order.
__global__ __launch_bounds__(256) void k_reduce(DevDesign D, double *partials, double *out,
                                               uint32_t *keys, int32_t *vals) {
  __shared__ double sh[4][256];
  const int n = D.n_ep;
  const int per = (n + kReduceBlocks - 1) / kReduceBlocks;
  const int b0 = blockIdx.x * per, b1 = min(n, b0 + per);
  double w0 = 0.0, w1 = 0.0, t0 = 0.0, t1 = 0.0;
  for (int e = b0 + (int)threadIdx.x; e < b1; e += 256) {
    const float2 s = D.ep_slack[e];
    w0 = fmin(w0, (double)s.x);
    w1 = fmin(w1, (double)s.y);
    if (s.x < 0.0f) t0 += (double)s.x;
    if (s.y < 0.0f) t1 += (double)s.y;
    if (keys) {
      keys[e] = f2ukey(s.x);
      keys[n + e] = f2ukey(s.y);
      vals[e] = e;
    }
  }
  const int tid = threadIdx.x;
  sh[0][tid] = w0; sh[1][tid] = w1; sh[2][tid] = t0; sh[3][tid] = t1;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      sh[0][tid] = fmin(sh[0][tid], sh[0][tid + o]);
      sh[1][tid] = fmin(sh[1][tid], sh[1][tid + o]);
      sh[2][tid] = sh[2][tid] + sh[2][tid + o];
      sh[3][tid] = sh[3][tid] + sh[3][tid + o];
    }
    __syncthreads();
  }
  if (tid == 0) {
    for (int k = 0; k < 4; ++k) partials[blockIdx.x * 4 + k] = sh[k][0];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint32_t prev =
        __hip_atomic_fetch_add(D.counters + kCtrReduce, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == (uint32_t)(kReduceBlocks - 1)) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      double W0 = 0.0, W1 = 0.0, T0 = 0.0, T1 = 0.0;
      for (int b = 0; b < kReduceBlocks; ++b) {
        W0 = fmin(W0, partials[b * 4 + 0]);
        W1 = fmin(W1, partials[b * 4 + 1]);
        T0 += partials[b * 4 + 2];
        T1 += partials[b * 4 + 3];
      }
      out[0] = W0; out[1] = W1; out[2] = T0; out[3] = T1;
      D.counters[kCtrReduce] = 0u;
    }
  }
}

// ------------------------------------------------------- levelization

__global__ void k_level_init(int32_t *pending, int32_t *cell_level, const int32_t *cell_nin, int n) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) {
    pending[c] = cell_nin[c];
    cell_level[c] = -1;
  }
}

// Frontier = the driver pins whose level is final (level lvl of cells, 0 = PIs).
// A cell whose last pending input is reached here has cell level lvl + 1,
// because frontiers are processed in increasing level.
__global__ void k_level_step(const int32_t *frontier, int n_front, int lvl,
                             const int32_t *net_of_drv_pin, const int32_t *net_sink_ptr,
                             const int32_t *net_sink_pin, const int32_t *cell_of_in_pin,
                             const int32_t *cell_out_pin, int32_t *pending, int32_t *cell_level,
                             int32_t *next, uint32_t *next_count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_front) return;
  const int n = net_of_drv_pin[frontier[i]];
  for (int s = net_sink_ptr[n]; s < net_sink_ptr[n + 1]; ++s) {
    const int c = cell_of_in_pin[net_sink_pin[s]];
    if (c < 0) continue;
    if (atomicSub(&pending[c], 1) == 1) {
      cell_level[c] = lvl + 1;
      next[atomicAdd(next_count, 1u)] = cell_out_pin[c];
    }
  }
}

// Pin level: PI 0, cell output 2 * cell level, sink = driver level + 1.
__global__ void k_pin_levels(const int32_t *pin_kind, const int32_t *cell_of_pin,
                             const int32_t *cell_level, const int32_t *drv_of_sink_pin,
                             int32_t *pin_level, int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int k = pin_kind[p];
  int lv;
  if (k == 0) {
    lv = 0;
  } else if (k == 2) {
    lv = 2 * cell_level[cell_of_pin[p]];
  } else {
    const int drv = drv_of_sink_pin[p];
    lv = (pin_kind[drv] == 0 ? 0 : 2 * cell_level[cell_of_pin[drv]]) + 1;
  }
  pin_level[p] = lv;
}

__global__ void k_iota(int32_t *a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = i;
}

__global__ void k_reset(uint32_t *c, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = 0u;
}

// --------------------------------------------------------------- reports

__global__ void k_report_pins(DevDesign D, const int32_t *pin_loc, int n_pins, float4 *at, float4 *slew,
                              float4 *rat, uint32_t *crit, float4 *slack) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pins) return;
  const int loc = pin_loc[p];
  if (loc >= 0) {
    if (at || slew) {
      const PinState st = D.drv_state[loc];
      if (at) at[p] = st.at;
      if (slew) slew[p] = st.slew;
    }
    if (rat) rat[p] = D.drv_rat[loc];
    if (crit) crit[p] = D.drv_crit[loc];
    if (slack) slack[p] = D.drv_slack[loc];
  } else {
    const int s = -1 - loc;
    if (at || slew) {
      const PinState st = D.sink_state[s];
      if (at) at[p] = st.at;
      if (slew) slew[p] = st.slew;
    }
    if (rat) rat[p] = D.sink_rat[s];
    if (crit) crit[p] = 0xffffffffu;
    if (slack) slack[p] = D.sink_slack[s];
  }
}

__global__ void k_report_rc(DevDesign D, const int32_t *net_slot, int n_nets, const int32_t *sink_slot,
                            int n_sinks, float *net_load, float *sink_delay, float *sink_spread) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (net_load && i < n_nets) net_load[i] = D.L_net[net_slot[i]];
  if (i < n_sinks) {
    const float2 w = D.dq[sink_slot[i]];
    if (sink_delay) sink_delay[i] = w.x;
    if (sink_spread) sink_spread[i] = w.y;
  }
}

__global__ void k_permute_caps(const float *src, const int32_t *node_src, float *dst, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = src[node_src[k]];
}

inline int blocks_for(int64_t n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

// ------------------------------------------------------------ wrappers

size_t sweep_lds_bytes(const DevDesign &D) {
  const size_t per_wave = sizeof(PinState) * kWave;  // >= 4 ints per lane for the backward
  return lib_lds_bytes(D.n_types, D.tstride) + per_wave * (kSweepBlock / kWave);
}

int sweep_blocks_per_cu(size_t lds_bytes) {
  int nf = 0, nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nf, k_forward, kSweepBlock, lds_bytes) != hipSuccess)
    return 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_backward, kSweepBlock, lds_bytes) != hipSuccess)
    return 1;
  const int n = nf < nb ? nf : nb;
  return n < 1 ? 1 : n;
}

hipError_t launch_rc(const DevDesign &D, const int2 *chunks, int n_chunks, const BigNet *big, int n_big,
                     const int32_t *big_end, const float *big_pc, double *scratch, hipStream_t s) {
  const int n_ctr = kCtrLevels + 2 * (D.n_cell_levels + 1);
  int grid = n_big + n_chunks;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_rc, dim3(grid), dim3(kRcBlock), 0, s, D, chunks, n_chunks, big, n_big, big_end, big_pc,
                     scratch, D.counters, n_ctr);
  return hipGetLastError();
}

hipError_t launch_forward(const DevDesign &D, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_forward, dim3(grid), dim3(kSweepBlock), sweep_lds_bytes(D), s, D, 0, 0, 1);
  return hipGetLastError();
}

hipError_t launch_forward_level(const DevDesign &D, int c0, int c1, hipStream_t s) {
  if (c1 <= c0) return hipSuccess;
  const int per = kSweepBlock / kWave;
  hipLaunchKernelGGL(k_forward, dim3(blocks_for(c1 - c0, per)), dim3(kSweepBlock), sweep_lds_bytes(D), s,
                     D, c0, c1, 0);
  return hipGetLastError();
}

hipError_t launch_backward(const DevDesign &D, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_backward, dim3(grid), dim3(kSweepBlock), sweep_lds_bytes(D), s, D, 0, 0, 1);
  return hipGetLastError();
}

hipError_t launch_backward_level(const DevDesign &D, int c0, int c1, hipStream_t s) {
  if (c1 <= c0) return hipSuccess;
  const int per = kSweepBlock / kWave;
  hipLaunchKernelGGL(k_backward, dim3(blocks_for(c1 - c0, per)), dim3(kSweepBlock), sweep_lds_bytes(D), s,
                     D, c0, c1, 0);
  return hipGetLastError();
}

hipError_t launch_reset_counters(uint32_t *counters, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_reset, dim3(blocks_for(n, 256)), dim3(256), 0, s, counters, n);
  return hipGetLastError();
}

hipError_t launch_reduce(const DevDesign &D, double *partials, double *out, uint32_t *keys, int32_t *vals,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(kReduceBlocks), dim3(256), 0, s, D, partials, out, keys, vals);
  return hipGetLastError();
}

size_t sort_temp_bytes(int n) {
  size_t bytes = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                     (const int32_t *)nullptr, (int32_t *)nullptr, n);
  return bytes;
}

hipError_t sort_endpoints(void *temp, size_t temp_bytes, const uint32_t *keys_in, uint32_t *keys_out,
                          const int32_t *vals_in, int32_t *vals_out, int n, hipStream_t s) {
  return hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys_in, keys_out, vals_in, vals_out, n, 0, 32,
                                            s);
}

size_t level_sort_temp_bytes(int n) {
  size_t bytes = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const int32_t *)nullptr, (int32_t *)nullptr,
                                     (const int32_t *)nullptr, (int32_t *)nullptr, n);
  return bytes;
}

hipError_t sort_levels(void *temp, size_t temp_bytes, const int32_t *keys_in, int32_t *keys_out,
                       const int32_t *vals_in, int32_t *vals_out, int n, int key_bits, hipStream_t s) {
  return hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys_in, keys_out, vals_in, vals_out, n, 0,
                                            key_bits, s);
}

hipError_t launch_level_init(int32_t *pending, int32_t *cell_level, const int32_t *cell_nin, int n_cells,
                             hipStream_t s) {
  if (n_cells <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_level_init, dim3(blocks_for(n_cells, 256)), dim3(256), 0, s, pending, cell_level,
                     cell_nin, n_cells);
  return hipGetLastError();
}

hipError_t launch_level_step(const int32_t *frontier, int n_front, int lvl, const int32_t *net_of_drv_pin,
                             const int32_t *net_sink_ptr, const int32_t *net_sink_pin,
                             const int32_t *cell_of_in_pin, const int32_t *cell_out_pin, int32_t *pending,
                             int32_t *cell_level, int32_t *next, uint32_t *next_count, hipStream_t s) {
  if (n_front <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_level_step, dim3(blocks_for(n_front, 256)), dim3(256), 0, s, frontier, n_front, lvl,
                     net_of_drv_pin, net_sink_ptr, net_sink_pin, cell_of_in_pin, cell_out_pin, pending,
                     cell_level, next, next_count);
  return hipGetLastError();
}

hipError_t launch_pin_levels(const int32_t *pin_kind, const int32_t *cell_of_pin, const int32_t *cell_level,
                             const int32_t *drv_of_sink_pin, int32_t *pin_level, int n_pins, hipStream_t s) {
  hipLaunchKernelGGL(k_pin_levels, dim3(blocks_for(n_pins, 256)), dim3(256), 0, s, pin_kind, cell_of_pin,
                     cell_level, drv_of_sink_pin, pin_level, n_pins);
  return hipGetLastError();
}

hipError_t launch_iota(int32_t *a, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota, dim3(blocks_for(n, 256)), dim3(256), 0, s, a, n);
  return hipGetLastError();
}

hipError_t launch_report_pins(const DevDesign &D, const int32_t *pin_loc, int n_pins, float4 *at,
                              float4 *slew, float4 *rat, uint32_t *crit, float4 *slack, hipStream_t s) {
  hipLaunchKernelGGL(k_report_pins, dim3(blocks_for(n_pins, 256)), dim3(256), 0, s, D, pin_loc, n_pins, at,
                     slew, rat, crit, slack);
  return hipGetLastError();
}

hipError_t launch_report_rc(const DevDesign &D, const int32_t *net_slot, int n_nets, const int32_t *sink_slot,
                            int n_sinks, float *net_load, float *sink_delay, float *sink_spread,
                            hipStream_t s) {
  const int n = n_nets > n_sinks ? n_nets : n_sinks;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_report_rc, dim3(blocks_for(n, 256)), dim3(256), 0, s, D, net_slot, n_nets, sink_slot,
                     n_sinks, net_load, sink_delay, sink_spread);
  return hipGetLastError();
}

hipError_t launch_permute_caps(const float *src, const int32_t *node_src, float *dst, int64_t n,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_permute_caps, dim3(blocks_for(n, 256)), dim3(256), 0, s, src, node_src, dst, n);
  return hipGetLastError();
}

}  // namespace sta
