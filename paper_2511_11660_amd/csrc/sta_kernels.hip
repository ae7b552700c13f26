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

// Block barrier that orders LDS accesses only.  __syncthreads also waits for
// the block's global stores to complete (a workgroup-scope fence on every
// address space); where no thread of the block reads back another's global
// stores, that wait only lengthens the level's critical path.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The hardware deals consecutive block ids to the 8 XCDs in turn.  For a grid
// of 8 * ceil(n / 8) blocks this returns the item of the calling block such
// that each XCD takes one contiguous run of items, so the cache lines a run
// writes are filled in one L2 instead of being written back in parts by
// several (items >= n: the block has none).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_major(int n) {
  const int per = (n + kXcds - 1) / kXcds;
  return (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
}
__host__ __device__ inline int xcd_grid(int n) { return kXcds * ((n + kXcds - 1) / kXcds); }

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
// The axis is strictly increasing, so i is the number of interior points
// ax[1..n-2] that are <= X: all of them are read at once (points past n-1 lie
// inside the type's packed block and are masked), then ax[i] and the
// reciprocal width, two dependent LDS round trips in all.
__device__ __forceinline__ AxisPos axis_find(const float *ax, const float *rd, int n, float X) {
  float a[kMaxAxis - 2];
#pragma unroll
  for (int m = 1; m < kMaxAxis - 1; ++m) a[m - 1] = ax[m];
  int i = 0;
#pragma unroll
  for (int m = 1; m < kMaxAxis - 1; ++m) i += (m <= n - 2 && a[m - 1] <= X) ? 1 : 0;
  return {i, (X - ax[i]) * rd[i]};
}

__device__ __forceinline__ float bilerp(const float *T, int ny, AxisPos px, AxisPos py) {
  const float *r0 = T + px.i * ny + py.i;
  const float *r1 = r0 + ny;
  float a = r0[0] + px.t * (r1[0] - r0[0]);
  float b = r0[1] + px.t * (r1[1] - r0[1]);
  return a + py.t * (b - a);
}

// Bilinear value and its partials in X and Y on the chosen segment.
__device__ __forceinline__ float bilerp_d(const float *T, int ny, AxisPos px, AxisPos py, float rdx, float rdy,
                                          float &dX, float &dY) {
  const float *r0 = T + px.i * ny + py.i;
  const float *r1 = r0 + ny;
  const float e0 = r1[0] - r0[0], e1 = r1[1] - r0[1];
  const float a = r0[0] + px.t * e0;
  const float b = r0[1] + px.t * e1;
  dX = (e0 + py.t * (e1 - e0)) * rdx;
  dY = (b - a) * rdy;
  return a + py.t * (b - a);
}

__device__ __forceinline__ float4 slack4(float4 at, float4 rat) {
  return make_float4(at.x - rat.x, at.y - rat.y, rat.z - at.z, rat.w - at.w);
}

__device__ __forceinline__ float2 ep_slack2(float4 at, float4 rat) {
  return make_float2(fminf(at.x - rat.x, at.y - rat.y), fminf(rat.z - at.z, rat.w - at.w));
}

// Bitwise equality (an incremental update stops where a recomputed value is
// bitwise unchanged; -0 and +0 count as different).
__device__ __forceinline__ bool same_bits(const PinState &a, const PinState &b) {
  return __float_as_uint(a.at.x) == __float_as_uint(b.at.x) && __float_as_uint(a.at.y) == __float_as_uint(b.at.y) &&
         __float_as_uint(a.at.z) == __float_as_uint(b.at.z) && __float_as_uint(a.at.w) == __float_as_uint(b.at.w) &&
         __float_as_uint(a.slew.x) == __float_as_uint(b.slew.x) &&
         __float_as_uint(a.slew.y) == __float_as_uint(b.slew.y) &&
         __float_as_uint(a.slew.z) == __float_as_uint(b.slew.z) && __float_as_uint(a.slew.w) == __float_as_uint(b.slew.w);
}

__device__ __forceinline__ bool same_bits4(float4 a, float4 b) {
  return __float_as_uint(a.x) == __float_as_uint(b.x) && __float_as_uint(a.y) == __float_as_uint(b.y) &&
         __float_as_uint(a.z) == __float_as_uint(b.z) && __float_as_uint(a.w) == __float_as_uint(b.w);
}

// Accesses to values that one wave writes and another wave of the same
// persistent sweep reads.  kCoh selects agent-scope relaxed atomic loads and
// stores (coherent across the XCDs' separate L2 caches on their own, emitted
// with the device-scope cache bit), so the sweep's completion counters need no
// L2 write-back or invalidate: a producer waits for its own coherent stores to
// complete before bumping a counter, and a consumer issues its coherent loads
// only after it has read the counter.  Without kCoh (one launch per level) the
// kernel boundary orders everything and plain vector accesses are used.
template <bool kCoh>
__device__ __forceinline__ float4 ld4(const float4 *p) {
  if constexpr (kCoh) {
    const uint64_t *q = reinterpret_cast<const uint64_t *>(p);
    const uint64_t a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t b = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_float4(__uint_as_float((uint32_t)a), __uint_as_float((uint32_t)(a >> 32)),
                       __uint_as_float((uint32_t)b), __uint_as_float((uint32_t)(b >> 32)));
  } else {
    return *p;
  }
}

template <bool kCoh>
__device__ __forceinline__ void st4(float4 *p, float4 v) {
  if constexpr (kCoh) {
    uint64_t *q = reinterpret_cast<uint64_t *>(p);
    __hip_atomic_store(q, (uint64_t)__float_as_uint(v.x) | ((uint64_t)__float_as_uint(v.y) << 32),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(q + 1, (uint64_t)__float_as_uint(v.z) | ((uint64_t)__float_as_uint(v.w) << 32),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    *p = v;
  }
}

template <bool kCoh>
__device__ __forceinline__ PinState ld_state(const PinState *p) {
  PinState s;
  s.at = ld4<kCoh>(&p->at);
  s.slew = ld4<kCoh>(&p->slew);
  return s;
}

template <bool kCoh>
__device__ __forceinline__ void st_state(PinState *p, const PinState &v) {
  st4<kCoh>(&p->at, v.at);
  st4<kCoh>(&p->slew, v.slew);
}

// LDS image of the library: packed tables then the sense codes.
struct LdsLib {
  const float *tab;
  const int *sense;
  int shift;  // packed-table float index held at tab[0] (0: the whole library is staged)
};

// The LDS copy of type t's packed block.
__device__ __forceinline__ const float *lib_type(const LdsLib &lib, const DevDesign &D, int t) {
  return lib.tab + (t * D.tstride - lib.shift);
}

// Library staging into LDS (packed tables padded to a multiple of 4 floats,
// then the sense codes), split in two so a level kernel can keep the loads in
// flight under its dependent gathers: lib_issue requests up to kLibRegs float4
// per thread into registers at kernel entry, all together; lib_store writes
// them with unpredicated stores (a lane past the end rewrites the last element
// with its own copy of it: a predicated store would let the compiler sink each
// load into its branch, one round trip per element) and stages any remainder
// of a library larger than kLibRegs x blockDim float4 element by element.
constexpr int kLibRegs = 8;
struct LibRegs {
  float4 v[kLibRegs];
};

__device__ __forceinline__ LibRegs lib_issue(const DevDesign &D) {
  LibRegs r;
  const int n4 = (D.n_types * D.tstride + 3) >> 2;
  const float4 *src = reinterpret_cast<const float4 *>(D.tables);
#pragma unroll
  for (int u = 0; u < kLibRegs; ++u)  // clamped, unpredicated
    r.v[u] = src[min(u * (int)blockDim.x + (int)threadIdx.x, n4 - 1)];
  __builtin_amdgcn_sched_barrier(0);  // all requested here, none moved past later waits
  return r;
}

__device__ __forceinline__ LdsLib lib_store(const DevDesign &D, unsigned char *smem, LibRegs r) {
  float *tab = reinterpret_cast<float *>(smem);
  const int n4 = (D.n_types * D.tstride + 3) >> 2;
  float4 *dst = reinterpret_cast<float4 *>(tab);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int u = 0; u < kLibRegs; ++u) dst[min(u * (int)blockDim.x + (int)threadIdx.x, n4 - 1)] = r.v[u];
  const float4 *src = reinterpret_cast<const float4 *>(D.tables);
  for (int i = kLibRegs * (int)blockDim.x + (int)threadIdx.x; i < n4; i += blockDim.x) dst[i] = src[i];
  int *sense = reinterpret_cast<int *>(tab + 4 * n4);
  for (int i = threadIdx.x; i < D.n_types; i += blockDim.x) sense[i] = D.sense[i];
  return {tab, sense, 0};
}

// Both halves back to back (kernels with nothing to overlap the staging with).
__device__ __forceinline__ LdsLib load_lib(const DevDesign &D, unsigned char *smem) {
  float *tab = reinterpret_cast<float *>(smem);
  const int n4 = (D.n_types * D.tstride + 3) >> 2, t = threadIdx.x, B = blockDim.x;
  const float4 *src = reinterpret_cast<const float4 *>(D.tables);
  float4 *dst = reinterpret_cast<float4 *>(tab);
  for (int b = 0; b < n4; b += 4 * B) {  // four loads in flight, then four stores
    const int i0 = min(b + t, n4 - 1), i1 = min(b + B + t, n4 - 1);
    const int i2 = min(b + 2 * B + t, n4 - 1), i3 = min(b + 3 * B + t, n4 - 1);
    const float4 v0 = src[i0], v1 = src[i1], v2 = src[i2], v3 = src[i3];
    __builtin_amdgcn_sched_barrier(0);
    dst[i0] = v0;
    dst[i1] = v1;
    dst[i2] = v2;
    dst[i3] = v3;
  }
  int *sense = reinterpret_cast<int *>(tab + 4 * n4);
  for (int i = t; i < D.n_types; i += B) sense[i] = D.sense[i];
  return {tab, sense, 0};
}

// Staging of only the types [t_lo, t_hi] a block's cells use (within a level
// the cells are ordered by type, so a block of two chunks usually needs one or
// two types): one float4 per thread, requested at once, when the types' tables
// fit the block; any remainder element by element.  The LDS image keeps the
// whole-library layout (type t at t * tstride), so lookups are unchanged.
struct LibSpan {
  int f0, f1;  // float4 range [f0, f1) of the packed tables
};

__device__ __forceinline__ LibSpan lib_span(const DevDesign &D, int t_lo, int t_hi) {
  // float4 granules covering floats [t_lo * tstride, (t_hi + 1) * tstride)
  // (a type's block need not start on a granule: the edge granules copy a
  // neighbour's floats to their own places, which is harmless)
  return t_hi >= t_lo ? LibSpan{(t_lo * D.tstride) >> 2, ((t_hi + 1) * D.tstride + 3) >> 2} : LibSpan{0, 0};
}

__device__ __forceinline__ float4 lib_issue_span(const DevDesign &D, LibSpan sp) {
  const float4 *src = reinterpret_cast<const float4 *>(D.tables);
  const float4 v = src[min(sp.f0 + (int)threadIdx.x, max(sp.f1 - 1, 0))];  // clamped, unpredicated
  __builtin_amdgcn_sched_barrier(0);
  return v;
}

// The span's granules go to LDS from its start (lib_f4 granules reserved, the
// most any block of the launch needs), then the sense codes of every type.
__device__ __forceinline__ LdsLib lib_store_span(const DevDesign &D, unsigned char *smem, LibSpan sp, float4 v,
                                                 int lib_f4) {
  float *tab = reinterpret_cast<float *>(smem);
  __builtin_amdgcn_sched_barrier(0);
  if (sp.f1 > sp.f0) {
    float4 *dst = reinterpret_cast<float4 *>(tab);  // dst[i - f0]: granule i of the packed tables
    dst[min((int)threadIdx.x, sp.f1 - sp.f0 - 1)] = v;
    const float4 *src = reinterpret_cast<const float4 *>(D.tables);
    for (int i = (int)blockDim.x + (int)threadIdx.x; i < sp.f1 - sp.f0; i += blockDim.x) dst[i] = src[sp.f0 + i];
  }
  int *sense = reinterpret_cast<int *>(tab + 4 * lib_f4);
  for (int i = threadIdx.x; i < D.n_types; i += blockDim.x) sense[i] = D.sense[i];
  return {tab, sense, 4 * sp.f0};
}

// LDS bytes of a span image of lib_f4 granules and the sense codes.
__host__ __device__ inline size_t span_lds_bytes(int lib_f4, int n_types) {
  return ((size_t)lib_f4 * 16 + (size_t)n_types * 4 + 31) & ~(size_t)31;
}

__host__ __device__ inline size_t lib_lds_bytes(int n_types, int tstride) {
  size_t b = (((size_t)n_types * tstride + 3) & ~(size_t)3) * 4 + (size_t)n_types * 4;
  return (b + 31) & ~(size_t)31;
}

// ------------------------------------------------------------ forward

// Arrival/slew merge of one cell output over its fanin arcs: AT_in + delay
// (late max, early min), slew merged the same way independent of the AT
// winner; the critical code is 2*fanin + input transition of the AT winner,
// ties kept by the earlier candidate.  In smooth mode (gamma > 0) the late
// merges keep a running log-sum-exp: lse[ro] = sum exp((z - max) / gamma)
// against the running max at[2 + ro].
struct Merge {
  float at[4], sl[4], lse[2];
  int cr[4];
};

struct CellCtx {
  int sense;
  const float *tb;
  AxisPos py;
};

__device__ __forceinline__ CellCtx cell_ctx(const DevDesign &D, const LdsLib &lib, int t, float L) {
  const TabLayout lay{D.nx, D.ny};
  const float *tb = lib_type(lib, D, t);
  return {lib.sense[t], tb, axis_find(tb + lay.ya(), tb + lay.rdy(), D.ny, L)};
}

__device__ __forceinline__ void merge_init(Merge &m) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    m.at[v] = v < 2 ? kInf : -kInf;
    m.sl[v] = v < 2 ? kInf : -kInf;
    m.cr[v] = -1;
  }
  m.lse[0] = m.lse[1] = 0.0f;
}

__device__ __forceinline__ void merge_one(const DevDesign &D, const CellCtx &cc, const PinState &in, int pos,
                                          Merge &m) {
  const TabLayout lay{D.nx, D.ny};
  const float g = D.gamma;
  const float ia[4] = {in.at.x, in.at.y, in.at.z, in.at.w};
  const float is[4] = {in.slew.x, in.slew.y, in.slew.z, in.slew.w};
  const int k2 = pos * 2;
#pragma unroll
  for (int el = 0; el < 2; ++el) {
#pragma unroll
    for (int ri = 0; ri < 2; ++ri) {
      const int vi = el * 2 + ri;
      const AxisPos px = axis_find(cc.tb + lay.xa(), cc.tb + lay.rdx(), D.nx, is[vi]);
#pragma unroll
      for (int ro = 0; ro < 2; ++ro) {
        if (!arc_maps(cc.sense, ri, ro)) continue;
        const int vo = el * 2 + ro;
        const float dl = bilerp(cc.tb + lay.tab(ro), D.ny, px, cc.py);
        const float os = bilerp(cc.tb + lay.tab(2 + ro), D.ny, px, cc.py);
        const float cand = ia[vi] + dl;
        if (el ? cand > m.at[vo] : cand < m.at[vo]) {
          if (el && g > 0.0f) m.lse[ro] = m.lse[ro] * expf((m.at[vo] - cand) / g) + 1.0f;
          m.at[vo] = cand;
          m.cr[vo] = k2 + ri;
        } else if (el && g > 0.0f) {
          m.lse[ro] += expf((cand - m.at[vo]) / g);
        }
        m.sl[vo] = el ? fmaxf(m.sl[vo], os) : fminf(m.sl[vo], os);
      }
    }
  }
}

__device__ __forceinline__ void merge_finish(const DevDesign &D, Merge &m, PinState &out, uint32_t &crit) {
  const float g = D.gamma;
  if (g > 0.0f) {
    m.at[2] += g * logf(m.lse[0]);
    m.at[3] += g * logf(m.lse[1]);
  }
  out.at = make_float4(m.at[0], m.at[1], m.at[2], m.at[3]);
  out.slew = make_float4(m.sl[0], m.sl[1], m.sl[2], m.sl[3]);
  crit = (uint32_t)(m.cr[0] & 0xff) | ((uint32_t)(m.cr[1] & 0xff) << 8) |
         ((uint32_t)(m.cr[2] & 0xff) << 16) | ((uint32_t)(m.cr[3] & 0xff) << 24);
}

// Cells of a library with types of more than 4 inputs: fanins through the CSR.
template <bool kCoh>
__device__ void cell_forward_csr(const DevDesign &D, const LdsLib &lib, int x, PinState &out, uint32_t &crit) {
  const int f0 = D.fanin_ptr[x], f1 = D.fanin_ptr[x + 1];
  const CellCtx cc = cell_ctx(D, lib, D.cell_type[x], D.L_net[x]);
  Merge m;
  merge_init(m);
  for (int f = f0; f < f1; ++f) merge_one(D, cc, ld_state<kCoh>(D.sink_state + D.fanin_sink[f]), f - f0, m);
  merge_finish(D, m, out, crit);
}

// One chunk: the 64 drivers, then every sink of their nets
// (AT_s = AT_drv + d, slew_s = sqrt(slew_drv^2 + q)).  Split in two:
// fwd_prefetch requests everything that does not depend on the sweep itself
// (the chunk record, the sink metadata of the first two sink rounds, each
// lane's cell type, load and inline fanin ids, or its PI constraint), so a
// persistent wave can issue it before it waits for the previous level;
// fwd_finish gathers the input sink states and does the arithmetic.
struct FwdPre {
  int x0, x1, s0, s1;
  int dA, dB;
  float2 wA, wB;
  int t;
  float L;
  int4 f4;
  float4 pat, psl;
};

__device__ __forceinline__ FwdPre fwd_prefetch(const DevDesign &D, int c) {
  FwdPre p;
  const int lane = lane_id();
  const int4 cr = D.chunk_rec[c];
  p.x0 = __builtin_amdgcn_readfirstlane(cr.x);
  p.x1 = __builtin_amdgcn_readfirstlane(cr.y);
  p.s0 = __builtin_amdgcn_readfirstlane(cr.z);
  p.s1 = __builtin_amdgcn_readfirstlane(cr.w);
  const int smax = max(p.s1 - 1, 0);
  const int sA = min(p.s0 + lane, smax), sB = min(p.s0 + lane + kWave, smax);
  p.dA = D.sink_drv[sA];
  p.dB = D.sink_drv[sB];
  p.wA = D.dq[sA];
  p.wB = D.dq[sB];
  const int x = p.x0 + lane;
  const int xc = x < p.x1 ? x : p.x0;
  p.t = 0;
  p.L = 0.0f;
  p.f4 = make_int4(-1, -1, -1, -1);
  p.pat = p.psl = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (p.x0 < D.n_pi) {  // level 0: primary inputs only
    p.pat = D.pi_at[xc];
    p.psl = D.pi_slew[xc];
  } else if (D.fanin4) {
    p.t = D.cell_type[xc];
    p.L = D.L_net[xc];
    p.f4 = D.fanin4[xc];
  }
  return p;
}

template <bool kCoh>
__device__ void fwd_finish(const DevDesign &D, const LdsLib &lib, PinState *wst, const FwdPre &p) {
  const int lane = lane_id();
  const int x0 = p.x0, x1 = p.x1, s1 = p.s1;
  const int sA = p.s0 + lane, sB = sA + kWave;
  const int x = x0 + lane;
  const bool live = x < x1;
  PinState st;
  uint32_t crit = 0xffffffffu;
  if (x0 < D.n_pi) {
    st.at = p.pat;
    st.slew = p.psl;
  } else if (D.fanin4) {
    const int fs[4] = {p.f4.x, p.f4.y, p.f4.z, p.f4.w};
    PinState in[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) in[k] = ld_state<kCoh>(D.sink_state + max(fs[k], 0));
    const CellCtx cc = cell_ctx(D, lib, p.t, p.L);
    Merge m;
    merge_init(m);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (fs[k] >= 0) merge_one(D, cc, in[k], k, m);
    merge_finish(D, m, st, crit);
  } else {
    cell_forward_csr<kCoh>(D, lib, live ? x : x0, st, crit);
  }
  if (live) {
    st_state<kCoh>(D.drv_state + x, st);  // sink pieces of this driver read it in the next phase
    D.drv_crit[x] = crit;
    wst[lane] = st;
  }
  wave_sync();
  auto emit = [&](int s, int drv, float2 w) {
    const PinState ds = wst[drv - x0];
    PinState o;
    o.at = make_float4(ds.at.x + w.x, ds.at.y + w.x, ds.at.z + w.x, ds.at.w + w.x);
    o.slew = make_float4(sqrtf(ds.slew.x * ds.slew.x + w.y), sqrtf(ds.slew.y * ds.slew.y + w.y),
                         sqrtf(ds.slew.z * ds.slew.z + w.y), sqrtf(ds.slew.w * ds.slew.w + w.y));
    st_state<kCoh>(D.sink_state + s, o);
  };
  if (sA < s1) emit(sA, p.dA, p.wA);
  if (sB < s1) emit(sB, p.dB, p.wB);
  for (int s = sB + kWave; s < s1; s += kWave) emit(s, D.sink_drv[s], D.dq[s]);
  wave_sync();
}

template <bool kCoh>
__device__ __forceinline__ void fwd_chunk(const DevDesign &D, const LdsLib &lib, PinState *wst, int c) {
  fwd_finish<kCoh>(D, lib, wst, fwd_prefetch(D, c));
}

// Sinks beyond a high-fanout driver's first piece ("pieces"): every lane
// derives sink states from the one driver state.
template <bool kCoh>
__device__ void fwd_piece(const DevDesign &D, int j) {
  const int4 pr = D.piece_rec[j];
  const int x = __builtin_amdgcn_readfirstlane(pr.x);
  const int sa = __builtin_amdgcn_readfirstlane(pr.y), sb = __builtin_amdgcn_readfirstlane(pr.z);
  const PinState ds = ld_state<kCoh>(D.drv_state + x);
  for (int s = sa + lane_id(); s < sb; s += kWave) {
    const float2 w = D.dq[s];
    PinState o;
    o.at = make_float4(ds.at.x + w.x, ds.at.y + w.x, ds.at.z + w.x, ds.at.w + w.x);
    o.slew = make_float4(sqrtf(ds.slew.x * ds.slew.x + w.y), sqrtf(ds.slew.y * ds.slew.y + w.y),
                         sqrtf(ds.slew.z * ds.slew.z + w.y), sqrtf(ds.slew.w * ds.slew.w + w.y));
    st_state<kCoh>(D.sink_state + s, o);
  }
}

// One launch per phase (chunks of one level, or the pieces of one level).
// Per-level forward: one block per chunk, thread 4 d + v computing output
// view v = (early/late, rise/fall) of driver d of the chunk, so each thread
// merges only the candidates of one view (in the same fanin / input-transition
// order as the per-cell merge, so the results are identical); then the block
// writes the chunk's sinks.  Every sweep-independent load is requested before
// the library is staged.
__device__ __forceinline__ void merge_view(const DevDesign &D, const CellCtx &cc, int el, int ro, const float ia[2],
                                           const float is[2], int pos, float &at, float &sl, int &cr, float &lse) {
  const TabLayout lay{D.nx, D.ny};
  const float g = D.gamma;
#pragma unroll
  for (int ri = 0; ri < 2; ++ri) {
    if (!arc_maps(cc.sense, ri, ro)) continue;
    const AxisPos px = axis_find(cc.tb + lay.xa(), cc.tb + lay.rdx(), D.nx, is[ri]);
    const float dl = bilerp(cc.tb + lay.tab(ro), D.ny, px, cc.py);
    const float os = bilerp(cc.tb + lay.tab(2 + ro), D.ny, px, cc.py);
    const float cand = ia[ri] + dl;
    if (el ? cand > at : cand < at) {
      if (el && g > 0.0f) lse = lse * expf((at - cand) / g) + 1.0f;
      at = cand;
      cr = pos * 2 + ri;
    } else if (el && g > 0.0f) {
      lse += expf((cand - at) / g);
    }
    sl = el ? fmaxf(sl, os) : fminf(sl, os);
  }
}

// merge_view without divergent branches, for the inline-fanin path where all
// four lanes of a driver run every fanin slot together (an empty slot is
// masked by valid).  The two lanes of one early/late half share their x-axis
// searches: lane (el, ro) searches the input slew of transition ri = ro and
// takes the other transition's search from its neighbour.  Candidates,
// comparisons and the log-sum-exp updates are merge_view's, in its order, so
// the results are the same bits.
__device__ __forceinline__ void merge_view_pair(const DevDesign &D, const CellCtx &cc, int el, int ro,
                                                const float ia[2], const float is[2], bool valid, int pos,
                                                float &at, float &sl, int &cr, float &lse) {
  const TabLayout lay{D.nx, D.ny};
  const float g = D.gamma;
  const AxisPos mine = axis_find(cc.tb + lay.xa(), cc.tb + lay.rdx(), D.nx, is[ro]);
  AxisPos other;
  other.i = __shfl_xor(mine.i, 1);
  other.t = __shfl_xor(mine.t, 1);
#pragma unroll
  for (int ri = 0; ri < 2; ++ri) {
    const AxisPos px = ri == ro ? mine : other;
    const bool m = valid && arc_maps(cc.sense, ri, ro);
    const float dl = bilerp(cc.tb + lay.tab(ro), D.ny, px, cc.py);
    const float os = bilerp(cc.tb + lay.tab(2 + ro), D.ny, px, cc.py);
    const float cand = ia[ri] + dl;
    const bool better = m && (el ? cand > at : cand < at);
    if (g > 0.0f) {
      const float up = lse * expf((at - cand) / g) + 1.0f;
      const float add = lse + expf((cand - at) / g);
      if (el && m) lse = better ? up : add;
    }
    at = better ? cand : at;
    cr = better ? pos * 2 + ri : cr;
    if (m) sl = el ? fmaxf(sl, os) : fminf(sl, os);
  }
}

// The inline-fanin merge of one view over kSlots fanin slots, staged so that
// every LDS access of a stage is independent of the others: the cell's x axis
// once, the segment of each slot's input slew (ALU), each segment's axis
// point and reciprocal width, the searches shared across the lane pair, all
// bilinear corners, then the merges in (slot, input transition) order.  Each
// value is computed by the expressions of axis_find, bilerp and
// merge_view_pair, so the results are the same bits.
template <int kSlots>
__device__ __forceinline__ void merge_slots(const DevDesign &D, const CellCtx &cc, int el, int ro, const float2 *iat,
                                            const float2 *isl, const int *fs, float &at, float &sl, int &cr,
                                            float &lse) {
  const TabLayout lay{D.nx, D.ny};
  const float *xa = cc.tb + lay.xa(), *rdx = cc.tb + lay.rdx();
  float a[kMaxAxis - 2];
#pragma unroll
  for (int m = 1; m < kMaxAxis - 1; ++m) a[m - 1] = xa[m];
  float X[kSlots];
  int seg[kSlots];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    X[k] = ro ? isl[k].y : isl[k].x;
    int i = 0;
#pragma unroll
    for (int m = 1; m < kMaxAxis - 1; ++m) i += (m <= D.nx - 2 && a[m - 1] <= X[k]) ? 1 : 0;
    seg[k] = i;
  }
  float ax[kSlots], rd[kSlots];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    ax[k] = xa[seg[k]];
    rd[k] = rdx[seg[k]];
  }
  AxisPos mine[kSlots], other[kSlots];  // (static indices only: no private-memory arrays)
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    mine[k] = AxisPos{seg[k], (X[k] - ax[k]) * rd[k]};
    other[k].i = __shfl_xor(mine[k].i, 1);
    other[k].t = __shfl_xor(mine[k].t, 1);
  }
  float dl[kSlots][2], os[kSlots][2];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
#pragma unroll
    for (int ri = 0; ri < 2; ++ri) {
      AxisPos px;
      px.i = ri == ro ? mine[k].i : other[k].i;
      px.t = ri == ro ? mine[k].t : other[k].t;
      dl[k][ri] = bilerp(cc.tb + lay.tab(ro), D.ny, px, cc.py);
      os[k][ri] = bilerp(cc.tb + lay.tab(2 + ro), D.ny, px, cc.py);
    }
  }
  const float g = D.gamma;
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    const float ia[2] = {iat[k].x, iat[k].y};
#pragma unroll
    for (int ri = 0; ri < 2; ++ri) {
      const bool m = fs[k] >= 0 && arc_maps(cc.sense, ri, ro);
      const float cand = ia[ri] + dl[k][ri];
      const bool better = m && (el ? cand > at : cand < at);
      if (g > 0.0f) {
        const float up = lse * expf((at - cand) / g) + 1.0f;
        const float add = lse + expf((cand - at) / g);
        lse = (el && m) ? (better ? up : add) : lse;
      }
      at = better ? cand : at;
      cr = better ? k * 2 + ri : cr;
      sl = m ? (el ? fmaxf(sl, os[k][ri]) : fminf(sl, os[k][ri])) : sl;
    }
  }
}

// With kInc (incremental continuation, IncArgs valid) an unflagged chunk
// returns at once; a flagged one compares its results bitwise with the stored
// ones, rewrites the sinks only of drivers that changed or whose net was
// recomputed, and flags the consumers of changed sinks and itself for the
// backward sweep.
// kSlots: inline fanin slots to merge (the library's most inputs, <= 4), so
// the slot loop is straight-line code whose table loads can all be issued
// together; a cell with fewer inputs masks its empty slots.
// kCpb: chunks per block (256 threads each; the full update uses kLevelCpb).
// Chunks of one block share one staging of their types' tables; a block's
// chunk past the phase's n chunks only reaches the barriers (reads clamped to
// the last chunk, nothing written).  The incremental kernels keep one.
template <bool kInc, int kSlots, int kCpb>
__global__ __launch_bounds__(kSweepBlock * kCpb) void k_forward(DevDesign D, int c0, int xb, int xr, int n,
                                                                 int lib_f4, IncArgs I) {
  extern __shared__ __align__(32) unsigned char smem[];
  static_assert(kSweepBlock == 4 * kChunk, "one thread per driver view");
  static_assert(kCpb == 1 || !kInc, "incremental chunks return early: one chunk per block");
  const int half = (int)threadIdx.x / kSweepBlock, tid = (int)threadIdx.x % kSweepBlock;
  const int cb_raw = (int)blockIdx.x * kCpb + half;
  const bool active = cb_raw < n;
  const int cb = active ? cb_raw : n - 1;
  const int c = c0 + cb;
  // (incremental: the chunk's flag is requested with the first loads and
  // tested before the input gathers and the library staging)
  uint32_t flagged = 1u;
  if constexpr (kInc) flagged = I.flag[c];
  const int dv = tid >> 2, v = tid & 3, el = v >> 1, ro = v & 1;
  // regular chunks are the level's runs of kChunk slots from xb (no record
  // load on the path to the fanin gathers); a high-fanout driver's own chunk
  // comes after them and is read from its record
  // Load order matters: the wait for a load also waits for every load issued
  // before it, so the cell's own loads (the fanin ids first) come first, then
  // the library, then the sink range (only needed for the stores).
  const bool regular = cb * kChunk < xr - xb;
  int x0, x1, s0v = 0, s1v = 0;
  if (regular) {
    x0 = xb + cb * kChunk;
    x1 = min(x0 + kChunk, xr);
  } else {
    const int4 cr4 = D.chunk_rec[c];
    x0 = __builtin_amdgcn_readfirstlane(cr4.x);
    x1 = __builtin_amdgcn_readfirstlane(cr4.y);
    s0v = cr4.z;
    s1v = cr4.w;
  }
  if (!active) x1 = x0;  // no drivers (and no sinks, below)
  const int x = x0 + dv;
  const bool live = x < x1;
  const int xc = live ? x : x0;
  const bool pis = x0 < D.n_pi;  // level 0: primary inputs only
  // every load unconditional (all indices valid for PI and cell slots alike):
  // a load under a branch makes the compiler wait for it at the branch's end
  const bool inl = kSlots > 0 && !pis;
  const int4 f4 = kSlots > 0 ? D.fanin4[xc] : make_int4(-1, -1, -1, -1);
  const int t = D.cell_type[xc];
  const float L = D.L_net[xc];
  const int xpi = min(xc, max(D.n_pi - 1, 0));
  const float pa = reinterpret_cast<const float *>(D.pi_at + xpi)[v];
  const float ps = reinterpret_cast<const float *>(D.pi_slew + xpi)[v];
  // the types of the block's chunks (a chunk past the phase repeats the last)
  int t_lo = INT32_MAX, t_hi = -1;
#pragma unroll
  for (int h = 0; h < kCpb; ++h) {
    const int2 tr = D.chunk_trange[c0 + min((int)blockIdx.x * kCpb + h, n - 1)];
    if (tr.y >= tr.x) {
      t_lo = min(t_lo, tr.x);
      t_hi = max(t_hi, tr.y);
    }
  }
  const LibSpan span = lib_span(D, t_lo, t_hi);
  const float4 lib_r = lib_issue_span(D, span);
  if (regular) {
    s0v = D.sink_ptr[x0];
    s1v = D.sink_ptr[x1];
  }
  if constexpr (kInc) {
    if (__builtin_amdgcn_readfirstlane(flagged) == 0u) return;
  }
  // input states of this view's early/late half: AT and slew of (el, rise/fall)
  const int fs[4] = {f4.x, f4.y, f4.z, f4.w};
  float2 iat[4], isl[4];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    const float *st = reinterpret_cast<const float *>(D.sink_state + max(fs[k], 0));
    iat[k] = *reinterpret_cast<const float2 *>(st + 2 * el);
    isl[k] = *reinterpret_cast<const float2 *>(st + 4 + 2 * el);
  }
  const int s0 = __builtin_amdgcn_readfirstlane(s0v);
  const int s1 = active ? __builtin_amdgcn_readfirstlane(s1v) : s0;
  const int sA = min(s0 + tid, max(s1 - 1, 0));
  const int dA = D.sink_drv[sA];
  const float2 wA = D.dq[sA];
  float old_at = 0.0f, old_sl = 0.0f;
  bool rcd = false;
  PinState oldA{};
  int ccA = -1;
  if constexpr (kInc) {
    old_at = reinterpret_cast<const float *>(D.drv_state + xc)[v];
    old_sl = reinterpret_cast<const float *>(D.drv_state + xc)[4 + v];
    rcd = I.rcd[xc] != 0;
    oldA = D.sink_state[sA];
    ccA = I.sink_cc[sA];
  }
  const LdsLib lib = lib_store_span(D, smem, span, lib_r, lib_f4);
  PinState *wst = reinterpret_cast<PinState *>(smem + span_lds_bytes(lib_f4, D.n_types)) + half * kChunk;
  int *s_redo = reinterpret_cast<int *>(wst + kChunk);  // [kChunk], incremental only
  lds_barrier();
  float at_v, sl_v;
  int cr_v = -1;
  if (pis) {
    at_v = pa;
    sl_v = ps;
  } else {
    const CellCtx cc = cell_ctx(D, lib, t, L);
    at_v = el ? -kInf : kInf;
    sl_v = el ? -kInf : kInf;
    float lse = 0.0f;
    if constexpr (kSlots > 0) {
      merge_slots<kSlots>(D, cc, el, ro, iat, isl, fs, at_v, sl_v, cr_v, lse);
    } else {
      const int f0 = D.fanin_ptr[xc], f1 = D.fanin_ptr[xc + 1];
      for (int f = f0; f < f1; ++f) {
        const float *st = reinterpret_cast<const float *>(D.sink_state + D.fanin_sink[f]);
        const float ia[2] = {st[2 * el], st[2 * el + 1]}, is[2] = {st[4 + 2 * el], st[5 + 2 * el]};
        merge_view(D, cc, el, ro, ia, is, f - f0, at_v, sl_v, cr_v, lse);
      }
    }
    if (el && D.gamma > 0.0f) at_v += D.gamma * logf(lse);
  }
  // the four views of a driver sit in adjacent lanes: assemble the crit word
  uint32_t cw = (uint32_t)(cr_v & 0xff) << (8 * v);
  cw |= __shfl_xor(cw, 1);
  cw |= __shfl_xor(cw, 2);
  bool moved = true;
  if constexpr (kInc) {
    int ch = (__float_as_uint(at_v) != __float_as_uint(old_at) || __float_as_uint(sl_v) != __float_as_uint(old_sl));
    ch |= __shfl_xor(ch, 1);
    ch |= __shfl_xor(ch, 2);
    moved = ch != 0;
  }
  if (live) {
    if (moved) {
      float *o = reinterpret_cast<float *>(D.drv_state + x);
      o[v] = at_v;
      o[4 + v] = sl_v;
    }
    if (v == 0) D.drv_crit[x] = pis ? 0xffffffffu : cw;
    float *w = reinterpret_cast<float *>(wst + dv);
    w[v] = at_v;
    w[4 + v] = sl_v;
  }
  if constexpr (kInc) {
    const int redo = live && (moved || rcd);
    if (v == 0) s_redo[dv] = redo;
    if (__syncthreads_or(redo) == 0) return;
    if (tid == 0) I.flag[I.n_chunks + c] = 1u;
  } else {
    lds_barrier();
  }
  // (incremental: old is the sink's stored state, cc its consumer's chunk)
  auto emit = [&](int s, int drv, float2 w, const PinState &old, int cc) {
    if constexpr (kInc) {
      if (s_redo[drv - x0] == 0) return;
    }
    const PinState ds = wst[drv - x0];
    PinState o;
    o.at = make_float4(ds.at.x + w.x, ds.at.y + w.x, ds.at.z + w.x, ds.at.w + w.x);
    o.slew = make_float4(sqrtf(ds.slew.x * ds.slew.x + w.y), sqrtf(ds.slew.y * ds.slew.y + w.y),
                         sqrtf(ds.slew.z * ds.slew.z + w.y), sqrtf(ds.slew.w * ds.slew.w + w.y));
    if constexpr (kInc) {
      if (same_bits(o, old)) return;
      D.sink_state[s] = o;
      if (cc >= 0) I.flag[cc] = 1u;
    } else {
      D.sink_state[s] = o;
    }
  };
  if (s0 + tid < s1) emit(s0 + tid, dA, wA, oldA, ccA);
  for (int s = s0 + tid + kSweepBlock; s < s1; s += kSweepBlock) {
    if constexpr (kInc)
      emit(s, D.sink_drv[s], D.dq[s], D.sink_state[s], I.sink_cc[s]);
    else
      emit(s, D.sink_drv[s], D.dq[s], oldA, ccA);
  }
}

__device__ void inc_fwd_piece(const DevDesign &D, const IncArgs &I, int j);

template <bool kInc>
__global__ __launch_bounds__(kSweepBlock) void k_forward_pieces(DevDesign D, int j0, int j1, IncArgs I) {
  const int j = j0 + blockIdx.x * (kSweepBlock / kWave) + threadIdx.x / kWave;
  if (j >= j1) return;
  if constexpr (kInc) {
    if (I.flag[I.n_chunks + D.piece_rec[j].w] != 0u) inc_fwd_piece(D, I, j);
  } else {
    fwd_piece<false>(D, j);
  }
}

// ------------------------------------------------------------ backward

// RAT of one sink: its endpoint constraint, or its consumer cell's output RAT
// minus the recomputed arc delay (min for late, max for early over the output
// transitions the input reaches).
template <bool kCoh>
__device__ __forceinline__ float4 sink_rat(const DevDesign &D, const LdsLib &lib, const PinState &ss, int cons) {
  if (cons < 0) return D.ep_rat[-1 - cons];
  const TabLayout lay{D.nx, D.ny};
  // consumer's output RAT, load and type: one 32-byte record
  const float4 Ro4 = ld4<kCoh>(&D.cons_rec[cons].rat);
  const float2 Lt = *reinterpret_cast<const float2 *>(&D.cons_rec[cons].L);
  const int t = __float_as_int(Lt.y);
  const int sense = lib.sense[t];
  const float Ro[4] = {Ro4.x, Ro4.y, Ro4.z, Ro4.w};
  const float is[4] = {ss.slew.x, ss.slew.y, ss.slew.z, ss.slew.w};
  const float *tb = lib_type(lib, D, t);
  const AxisPos py = axis_find(tb + lay.ya(), tb + lay.rdy(), D.ny, Lt.x);
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
  return make_float4(r[0], r[1], r[2], r[3]);
}

// One chunk: every sink of the 64 drivers gets its RAT (sink_rat) and slack;
// the drivers merge RAT_s - d over their sinks through LDS integer atomics on
// order-preserving keys, starting from the neutral element; a dangling
// endpoint driver's own constraint joins the merge last (min/max are
// order-independent, so the result is the same and bit-reproducible).
// bwd_prefetch requests what the sweep does not produce (chunk record, first
// sink round's state, consumer id and delay, the drivers' endpoint index and
// arrival); bwd_finish does the consumer gathers and the arithmetic.
struct BwdPre {
  int x0, x1, s0, s1;
  PinState ssA, ssB;  // the first two sink rounds
  int consA, drvA, consB, drvB, e;
  float dA, dB;
  float4 A;
  int2 pcs;  // sink pieces of a high-fanout driver (first, count)
};

__device__ __forceinline__ BwdPre bwd_prefetch(const DevDesign &D, int c) {
  BwdPre p;
  const int lane = lane_id();
  const int4 cr = D.chunk_rec[c];
  p.x0 = __builtin_amdgcn_readfirstlane(cr.x);
  p.x1 = __builtin_amdgcn_readfirstlane(cr.y);
  p.s0 = __builtin_amdgcn_readfirstlane(cr.z);
  p.s1 = __builtin_amdgcn_readfirstlane(cr.w);
  const int smax = max(p.s1 - 1, 0);
  const int sAc = min(p.s0 + lane, smax), sBc = min(p.s0 + lane + kWave, smax);
  p.ssA = D.sink_state[sAc];
  p.consA = D.sink_cons[sAc];
  p.dA = D.dq[sAc].x;
  p.drvA = D.sink_drv[sAc];
  p.ssB = D.sink_state[sBc];
  p.consB = D.sink_cons[sBc];
  p.dB = D.dq[sBc].x;
  p.drvB = D.sink_drv[sBc];
  const int x = p.x0 + lane;
  const int xc = x < p.x1 ? x : p.x0;
  p.e = D.drv_ep[xc];
  p.A = D.drv_state[xc].at;
  const int2 pcs = D.chunk_pieces[c];
  p.pcs = make_int2(__builtin_amdgcn_readfirstlane(pcs.x), __builtin_amdgcn_readfirstlane(pcs.y));
  return p;
}

template <bool kCoh>
__device__ void bwd_finish(const DevDesign &D, const LdsLib &lib, int *wacc, const BwdPre &p) {
  const int lane = lane_id();
  const int x0 = p.x0, x1 = p.x1, s1 = p.s1;
  const int sA = p.s0 + lane;
  const int x = x0 + lane;
  const bool live = x < x1;
  wacc[lane * 4 + 0] = f2key(-kInf);
  wacc[lane * 4 + 1] = f2key(-kInf);
  wacc[lane * 4 + 2] = f2key(kInf);
  wacc[lane * 4 + 3] = f2key(kInf);
  wave_sync();
  auto sink = [&](int s, const PinState &ss, int cons, float d, int drv) {
    const float4 R = sink_rat<kCoh>(D, lib, ss, cons);
    D.sink_rat[s] = R;
    D.sink_slack[s] = slack4(ss.at, R);
    int *acc = wacc + (drv - x0) * 4;
    atomicMax(acc + 0, f2key(R.x - d));
    atomicMax(acc + 1, f2key(R.y - d));
    atomicMin(acc + 2, f2key(R.z - d));
    atomicMin(acc + 3, f2key(R.w - d));
  };
  if (sA < s1) sink(sA, p.ssA, p.consA, p.dA, p.drvA);
  if (sA + kWave < s1) sink(sA + kWave, p.ssB, p.consB, p.dB, p.drvB);
  for (int s = sA + 2 * kWave; s < s1; s += kWave) sink(s, D.sink_state[s], D.sink_cons[s], D.dq[s].x, D.sink_drv[s]);
  wave_sync();
  if (live) {
    float4 R = make_float4(key2f(wacc[lane * 4 + 0]), key2f(wacc[lane * 4 + 1]),
                           key2f(wacc[lane * 4 + 2]), key2f(wacc[lane * 4 + 3]));
    if (p.e >= 0) {
      const float4 E = D.ep_rat[p.e];
      R = make_float4(fmaxf(R.x, E.x), fmaxf(R.y, E.y), fminf(R.z, E.z), fminf(R.w, E.w));
    }
    for (int k = 0; k < p.pcs.y; ++k) {  // a high-fanout driver (alone in its chunk): its pieces' merges
      const float4 E = ld4<kCoh>(D.piece_rat + p.pcs.x + k);
      R = make_float4(fmaxf(R.x, E.x), fmaxf(R.y, E.y), fminf(R.z, E.z), fminf(R.w, E.w));
    }
    st4<kCoh>(&D.cons_rec[x].rat, R);
    D.drv_slack[x] = slack4(p.A, R);
  }
  wave_sync();
}

template <bool kCoh>
__device__ __forceinline__ void bwd_chunk(const DevDesign &D, const LdsLib &lib, int *wacc, int c) {
  bwd_finish<kCoh>(D, lib, wacc, bwd_prefetch(D, c));
}

// Sink RATs of one piece of a high-fanout driver's sinks; the piece's merge
// of RAT_s - d (max early, min late) is reduced across the wave and left in
// piece_rat for the driver's own chunk, which runs in the next phase.
template <bool kCoh>
__device__ void bwd_piece(const DevDesign &D, const LdsLib &lib, int j) {
  const int4 pr = D.piece_rec[j];
  const int sa = __builtin_amdgcn_readfirstlane(pr.y), sb = __builtin_amdgcn_readfirstlane(pr.z);
  float4 acc = make_float4(-kInf, -kInf, kInf, kInf);
  for (int s = sa + lane_id(); s < sb; s += kWave) {
    const PinState ss = D.sink_state[s];
    const int cons = D.sink_cons[s];
    const float d = D.dq[s].x;
    const float4 R = sink_rat<kCoh>(D, lib, ss, cons);
    D.sink_rat[s] = R;
    D.sink_slack[s] = slack4(ss.at, R);
    acc = make_float4(fmaxf(acc.x, R.x - d), fmaxf(acc.y, R.y - d), fminf(acc.z, R.z - d), fminf(acc.w, R.w - d));
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    acc.x = fmaxf(acc.x, __shfl_xor(acc.x, off));
    acc.y = fmaxf(acc.y, __shfl_xor(acc.y, off));
    acc.z = fminf(acc.z, __shfl_xor(acc.z, off));
    acc.w = fminf(acc.w, __shfl_xor(acc.w, off));
  }
  if (lane_id() == 0) st4<kCoh>(D.piece_rat + j, acc);
}

// Per-level backward: one block per chunk.  Threads 2 j + el take sink j of
// the chunk's range (in rounds of 128 sinks) for its early or late half (two
// views each), merging RAT_s - d into LDS keys; then thread 4 d + v finishes
// view v of driver d (endpoint constraint, pieces, slacks).  Sweep-independent
// loads are requested before the library is staged.
// With kInc an unflagged chunk returns at once; a flagged one compares each
// driver's RAT bitwise with the stored one and, where it changed or the
// driver's net was recomputed, flags the chunks of the cell's input sinks.
// kCpb: chunks per block, as for k_forward.
template <bool kInc, int kCpb>
__global__ __launch_bounds__(kSweepBlock * kCpb) void k_backward(DevDesign D, int c0, int c1, IncArgs I) {
  extern __shared__ __align__(32) unsigned char smem[];
  static_assert(kCpb == 1 || !kInc, "incremental chunks return early: one chunk per block");
  const int half = (int)threadIdx.x / kSweepBlock, tid = (int)threadIdx.x % kSweepBlock;
  const int c_raw = c0 + (int)blockIdx.x * kCpb + half;
  const bool active = c_raw < c1;
  const int c = active ? c_raw : c1 - 1;
  uint32_t flagged = 1u;  // (incremental: tested once the first loads are in flight)
  if constexpr (kInc) flagged = I.flag[I.n_chunks + c];
  const int el = tid & 1, dv = tid >> 2, v = tid & 3;
  const int4 cr4 = D.chunk_rec[c];
  const int x0 = __builtin_amdgcn_readfirstlane(cr4.x);
  const int x1 = active ? __builtin_amdgcn_readfirstlane(cr4.y) : x0;  // past the phase: no drivers,
  const int s0 = __builtin_amdgcn_readfirstlane(cr4.z);
  const int s1 = active ? __builtin_amdgcn_readfirstlane(cr4.w) : s0;  // no sinks
  const int smax = max(s1 - 1, 0);
  const int sA = s0 + (tid >> 1), sAc = min(sA, smax);
  auto ld_half = [&](int s, float2 &at, float2 &sl) {
    const float *st = reinterpret_cast<const float *>(D.sink_state + s);
    at = *reinterpret_cast<const float2 *>(st + 2 * el);
    sl = *reinterpret_cast<const float2 *>(st + 4 + 2 * el);
  };
  float2 atA, slA;
  ld_half(sAc, atA, slA);
  const int consA = D.sink_cons[sAc];
  const float dA = D.dq[sAc].x;
  const int drvA = D.sink_drv[sAc];
  const int x = x0 + dv;
  const bool live = x < x1;
  const int xc = live ? x : x0;
  const int e = D.drv_ep[xc];
  const float Av = reinterpret_cast<const float *>(D.drv_state + xc)[v];
  const int2 pcs = D.chunk_pieces[c];
  float old_r = 0.0f;
  bool rcd = false;
  int4 fcc = make_int4(-1, -1, -1, -1);
  if constexpr (kInc) {
    old_r = reinterpret_cast<const float *>(&D.cons_rec[xc].rat)[v];
    rcd = I.rcd[xc] != 0;
    if (I.fanin_cc) fcc = I.fanin_cc[xc];
    if (__builtin_amdgcn_readfirstlane(flagged) == 0u) return;
  }
  // Load order matters (a wait covers every earlier load): the sink data
  // above, then the library, then the first sink's consumer record, which
  // thus travels while the library is stored and the block synchronizes.
  // A consumer's (RAT of this half, (load, type)); an endpoint's RAT pair.
  struct ConsIn {
    float2 ro, lt;
  };
  auto ld_cons = [&](int cons) {  // unpredicated loads (an endpoint reads record 0's (load, type) unused)
    ConsIn ci;
    const float *rp = cons < 0 ? reinterpret_cast<const float *>(D.ep_rat + (-1 - cons))
                               : reinterpret_cast<const float *>(&D.cons_rec[cons].rat);
    ci.ro = *reinterpret_cast<const float2 *>(rp + 2 * el);
    ci.lt = *reinterpret_cast<const float2 *>(&D.cons_rec[max(cons, 0)].L);
    return ci;
  };
  const LibRegs lib_r = lib_issue(D);
  const ConsIn ciA = ld_cons(consA);
  const LdsLib lib = lib_store(D, smem, lib_r);
  int *wacc = reinterpret_cast<int *>(smem + lib_lds_bytes(D.n_types, D.tstride)) + half * kSweepBlock;
  wacc[tid] = f2key((v >> 1) ? kInf : -kInf);
  lds_barrier();
  const TabLayout lay{D.nx, D.ny};
  auto sink = [&](int s, float2 at, float2 sl, int cons, float d, int drv, const ConsIn &ci) {
    float r[2];
    if (cons < 0) {
      r[0] = ci.ro.x;
      r[1] = ci.ro.y;
    } else {
      const float2 Ro = ci.ro;
      const float2 Lt = ci.lt;
      const int t = __float_as_int(Lt.y);
      const int sense = lib.sense[t];
      const float *tb = lib_type(lib, D, t);
      const float ro_[2] = {Ro.x, Ro.y}, is[2] = {sl.x, sl.y};
      // staged as in merge_slots: both axes, then the three segments' points
      // and widths, then all corners; every (ri, ro) pair evaluated and the
      // unmapped ones masked (min / max are exact, so the order is free)
      const float *xa = tb + lay.xa(), *ya = tb + lay.ya();
      float ax6[kMaxAxis - 2], ay6[kMaxAxis - 2];
#pragma unroll
      for (int m = 1; m < kMaxAxis - 1; ++m) {
        ax6[m - 1] = xa[m];
        ay6[m - 1] = ya[m];
      }
      int iy = 0, ix[2] = {0, 0};
#pragma unroll
      for (int m = 1; m < kMaxAxis - 1; ++m) {
        iy += (m <= D.ny - 2 && ay6[m - 1] <= Lt.x) ? 1 : 0;
        ix[0] += (m <= D.nx - 2 && ax6[m - 1] <= is[0]) ? 1 : 0;
        ix[1] += (m <= D.nx - 2 && ax6[m - 1] <= is[1]) ? 1 : 0;
      }
      const float y0 = ya[iy], ry = tb[lay.rdy() + iy];
      const float x0[2] = {xa[ix[0]], xa[ix[1]]}, rx[2] = {tb[lay.rdx() + ix[0]], tb[lay.rdx() + ix[1]]};
      const AxisPos py{iy, (Lt.x - y0) * ry};
#pragma unroll
      for (int ri = 0; ri < 2; ++ri) {
        const AxisPos px{ix[ri], (is[ri] - x0[ri]) * rx[ri]};
        float best = el ? kInf : -kInf;
#pragma unroll
        for (int ro = 0; ro < 2; ++ro) {
          const float cand = ro_[ro] - bilerp(tb + lay.tab(ro), D.ny, px, py);
          const float nb = el ? fminf(best, cand) : fmaxf(best, cand);
          best = arc_maps(sense, ri, ro) ? nb : best;
        }
        r[ri] = best;
      }
    }
    float *rat = reinterpret_cast<float *>(D.sink_rat + s);
    float *slk = reinterpret_cast<float *>(D.sink_slack + s);
    rat[2 * el] = r[0];
    rat[2 * el + 1] = r[1];
    const float sk0 = el ? r[0] - at.x : at.x - r[0], sk1 = el ? r[1] - at.y : at.y - r[1];
    slk[2 * el] = sk0;
    slk[2 * el + 1] = sk1;
    int *acc = wacc + (drv - x0) * 4 + 2 * el;
    if (el) {
      atomicMin(acc + 0, f2key(r[0] - d));
      atomicMin(acc + 1, f2key(r[1] - d));
    } else {
      atomicMax(acc + 0, f2key(r[0] - d));
      atomicMax(acc + 1, f2key(r[1] - d));
    }
  };
  if (sA < s1) sink(sA, atA, slA, consA, dA, drvA, ciA);
  for (int sj = sA + kSweepBlock / 2; sj < s1; sj += kSweepBlock / 2) {
    float2 at, sl;
    ld_half(sj, at, sl);
    const int cons = D.sink_cons[sj];
    sink(sj, at, sl, cons, D.dq[sj].x, D.sink_drv[sj], ld_cons(cons));
  }
  lds_barrier();
  float R = key2f(wacc[tid]);
  const bool late = (v >> 1) != 0;
  if (live && e >= 0) {
    const float E = reinterpret_cast<const float *>(D.ep_rat + e)[v];
    R = late ? fminf(R, E) : fmaxf(R, E);
  }
  for (int k = 0; k < pcs.y; ++k) {  // a high-fanout driver (alone in its chunk): its pieces' merges
    const float E = reinterpret_cast<const float *>(D.piece_rat + pcs.x + k)[v];
    R = late ? fminf(R, E) : fmaxf(R, E);
  }
  const float sk = late ? R - Av : Av - R;
  if (live) {
    reinterpret_cast<float *>(&D.cons_rec[x].rat)[v] = R;
    reinterpret_cast<float *>(D.drv_slack + x)[v] = sk;
  }
  if constexpr (kInc) {
    int ch = __float_as_uint(R) != __float_as_uint(old_r);
    ch |= __shfl_xor(ch, 1);
    ch |= __shfl_xor(ch, 2);
    if (live && v == 0 && (ch || rcd) && x >= D.n_pi) {
      if (I.fanin_cc) {
        const int fc[4] = {fcc.x, fcc.y, fcc.z, fcc.w};
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (fc[k] >= 0) I.flag[I.n_chunks + fc[k]] = 1u;
      } else {
        for (int f = D.fanin_ptr[x]; f < D.fanin_ptr[x + 1]; ++f)
          I.flag[I.n_chunks + I.chunk_of[D.sink_drv[D.fanin_sink[f]]]] = 1u;
      }
    }
  }
}

template <bool kInc>
__global__ __launch_bounds__(kSweepBlock) void k_backward_pieces(DevDesign D, int j0, int j1, IncArgs I) {
  extern __shared__ __align__(32) unsigned char smem[];
  const LdsLib lib = load_lib(D, smem);
  lds_barrier();
  const int j = j0 + blockIdx.x * (kSweepBlock / kWave) + threadIdx.x / kWave;
  if (j >= j1) return;
  if constexpr (kInc) {
    if (I.flag[I.n_chunks + D.piece_rec[j].w] == 0u) return;
  }
  bwd_piece<false>(D, lib, j);
}

// ------------------------------------------ backward with RATs pushed to inputs
//
// Per-level backward of the per-level and graph schedules.  The RAT of a sink
// is its endpoint constraint, or its consumer cell's output RAT minus the arc
// delay, merged over the output transitions the input transition reaches; here
// the consumer computes it, when its own level runs.  The kernel of a level,
// one 256-thread block per chunk (two chunks per block, as the forward):
//  (a) threads 2 j + el take sink j of the chunk for the early or late half:
//      its RAT (written by its consumer at a higher level, or its endpoint
//      constraint), its slack, and RAT_s - d merged into its driver through
//      LDS keys; then thread 4 d + v finishes view v of driver d (endpoint
//      constraint, the pieces of a high-fanout driver, slack);
//  (b) thread 4 d + v = (early/late, output transition ro) recomputes driver
//      d's cell arc delays into ro from the inputs' stored slews (tables of the
//      chunk's own types only: cells are ordered by type within a level) and,
//      with its neighbour lane of the other ro, writes the RAT of every input
//      sink.
// Each input sink has one consumer, and min / max are exact, so every value
// is the same bits as the sink-centric sweep's (sink_rat), which the
// persistent and incremental schedules keep.  The arc-delay loads do not
// depend on (a), so they are in flight while (a) runs.
template <int kSlots>
__device__ __forceinline__ void slot_delays(const DevDesign &D, const CellCtx &cc, int ro, const float2 *isl,
                                            float (*dl)[2]) {
  const TabLayout lay{D.nx, D.ny};
  const float *xa = cc.tb + lay.xa(), *rdx = cc.tb + lay.rdx();
  float a[kMaxAxis - 2];
#pragma unroll
  for (int m = 1; m < kMaxAxis - 1; ++m) a[m - 1] = xa[m];
  float X[kSlots];
  int seg[kSlots];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    X[k] = ro ? isl[k].y : isl[k].x;
    int i = 0;
#pragma unroll
    for (int m = 1; m < kMaxAxis - 1; ++m) i += (m <= D.nx - 2 && a[m - 1] <= X[k]) ? 1 : 0;
    seg[k] = i;
  }
  float ax[kSlots], rd[kSlots];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    ax[k] = xa[seg[k]];
    rd[k] = rdx[seg[k]];
  }
  AxisPos mine[kSlots], other[kSlots];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    mine[k] = AxisPos{seg[k], (X[k] - ax[k]) * rd[k]};
    other[k].i = __shfl_xor(mine[k].i, 1);
    other[k].t = __shfl_xor(mine[k].t, 1);
  }
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
#pragma unroll
    for (int ri = 0; ri < 2; ++ri) {
      AxisPos px;
      px.i = ri == ro ? mine[k].i : other[k].i;
      px.t = ri == ro ? mine[k].t : other[k].t;
      dl[k][ri] = bilerp(cc.tb + lay.tab(ro), D.ny, px, cc.py);
    }
  }
}

// RAT of input transition ri = ro of one input, in the lane (el, ro): this
// lane's candidate R_out(el, ro) - delay(ri -> ro) and the neighbour lane's
// R_out(el, 1 - ro) - delay(ri -> 1 - ro), each where the arc maps.
__device__ __forceinline__ float push_rat(int sense, int el, int ro, float Rv, float d_same, float d_cross,
                                          bool valid) {
  const float neutral = el ? kInf : -kInf;
  const float own = valid && arc_maps(sense, ro, ro) ? Rv - d_same : neutral;
  // what this lane offers its neighbour: its candidate for ri = 1 - ro
  const float give = valid && arc_maps(sense, 1 - ro, ro) ? Rv - d_cross : neutral;
  const float nb = __shfl_xor(give, 1);
  return el ? fminf(own, nb) : fmaxf(own, nb);
}

template <int kSlots, int kCpb>
__global__ __launch_bounds__(kSweepBlock * kCpb) void k_backward_push(DevDesign D, int c0, int xb, int xr, int n,
                                                                       int lib_f4) {
  extern __shared__ __align__(32) unsigned char smem[];
  static_assert(kSweepBlock == 4 * kChunk, "one thread per driver view");
  const int half = (int)threadIdx.x / kSweepBlock, tid = (int)threadIdx.x % kSweepBlock;
  const int cb_raw = (int)blockIdx.x * kCpb + half;
  const bool active = cb_raw < n;
  const int cb = active ? cb_raw : n - 1;
  const int c = c0 + cb;
  const int dv = tid >> 2, v = tid & 3, el = v >> 1, ro = v & 1;
  const int sel = tid & 1;  // early/late half of this thread's sinks in (a)
  const bool regular = cb * kChunk < xr - xb;
  int x0, x1, s0v = 0, s1v = 0;
  if (regular) {
    x0 = xb + cb * kChunk;
    x1 = min(x0 + kChunk, xr);
  } else {
    const int4 cr4 = D.chunk_rec[c];
    x0 = __builtin_amdgcn_readfirstlane(cr4.x);
    x1 = __builtin_amdgcn_readfirstlane(cr4.y);
    s0v = cr4.z;
    s1v = cr4.w;
  }
  if (!active) x1 = x0;
  const int x = x0 + dv;
  const bool live = x < x1;
  const int xc = live ? x : x0;
  const bool pis = x0 < D.n_pi;
  // (b)'s cell loads first (the fanin ids head the longest chain), every load
  // unconditional
  const int4 f4 = kSlots > 0 ? D.fanin4[xc] : make_int4(-1, -1, -1, -1);
  const int t = max(D.cell_type[xc], 0);
  const float L = D.L_net[xc];
  const int e = D.drv_ep[xc];
  const float Av = reinterpret_cast<const float *>(D.drv_state + xc)[v];
  int t_lo = INT32_MAX, t_hi = -1;
#pragma unroll
  for (int h = 0; h < kCpb; ++h) {
    const int2 tr = D.chunk_trange[c0 + min((int)blockIdx.x * kCpb + h, n - 1)];
    if (tr.y >= tr.x) {
      t_lo = min(t_lo, tr.x);
      t_hi = max(t_hi, tr.y);
    }
  }
  const LibSpan span = lib_span(D, t_lo, t_hi);
  const float4 lib_r = lib_issue_span(D, span);
  if (regular) {
    s0v = D.sink_ptr[x0];
    s1v = D.sink_ptr[x1];
  }
  const int fs[4] = {f4.x, f4.y, f4.z, f4.w};
  float2 isl[4];
#pragma unroll
  for (int k = 0; k < kSlots; ++k)
    isl[k] = *reinterpret_cast<const float2 *>(reinterpret_cast<const float *>(D.sink_state + max(fs[k], 0)) + 4 +
                                               2 * el);
  const int2 pcs = D.chunk_pieces[c];
  const int s0 = __builtin_amdgcn_readfirstlane(s0v);
  const int s1 = active ? __builtin_amdgcn_readfirstlane(s1v) : s0;
  const int smax = max(s1 - 1, 0);
  const int sA = s0 + (tid >> 1), sAc = min(sA, smax);
  struct SinkIn {
    float2 rat, at;
    int cons, drv;
    float d;
  };
  auto ld_sink = [&](int s) {  // unpredicated (an endpoint sink reads its stale sink_rat unused)
    SinkIn q;
    q.cons = D.sink_cons[s];
    q.drv = D.sink_drv[s];
    q.d = D.dq[s].x;
    q.rat = *reinterpret_cast<const float2 *>(reinterpret_cast<const float *>(D.sink_rat + s) + 2 * sel);
    q.at = *reinterpret_cast<const float2 *>(reinterpret_cast<const float *>(D.sink_state + s) + 2 * sel);
    return q;
  };
  const SinkIn qA = ld_sink(sAc);
  const LdsLib lib = lib_store_span(D, smem, span, lib_r, lib_f4);
  int *wacc = reinterpret_cast<int *>(smem + span_lds_bytes(lib_f4, D.n_types)) + half * kSweepBlock;
  wacc[tid] = f2key((v >> 1) ? kInf : -kInf);
  lds_barrier();
  // (a) the chunk's sinks
  auto sink = [&](int s, const SinkIn &q) {
    float2 r = q.rat;
    if (q.cons < 0) {
      r = *reinterpret_cast<const float2 *>(reinterpret_cast<const float *>(D.ep_rat + (-1 - q.cons)) + 2 * sel);
      *reinterpret_cast<float2 *>(reinterpret_cast<float *>(D.sink_rat + s) + 2 * sel) = r;
    }
    const float sk0 = sel ? r.x - q.at.x : q.at.x - r.x, sk1 = sel ? r.y - q.at.y : q.at.y - r.y;
    *reinterpret_cast<float2 *>(reinterpret_cast<float *>(D.sink_slack + s) + 2 * sel) = make_float2(sk0, sk1);
    int *acc = wacc + (q.drv - x0) * 4 + 2 * sel;
    if (sel) {
      atomicMin(acc + 0, f2key(r.x - q.d));
      atomicMin(acc + 1, f2key(r.y - q.d));
    } else {
      atomicMax(acc + 0, f2key(r.x - q.d));
      atomicMax(acc + 1, f2key(r.y - q.d));
    }
  };
  if (sA < s1) sink(sA, qA);
  for (int sj = sA + kSweepBlock / 2; sj < s1; sj += kSweepBlock / 2) sink(sj, ld_sink(sj));
  lds_barrier();
  float R = key2f(wacc[tid]);
  const bool late = el != 0;
  if (live && e >= 0) {
    const float E = reinterpret_cast<const float *>(D.ep_rat + e)[v];
    R = late ? fminf(R, E) : fmaxf(R, E);
  }
  for (int k = 0; k < pcs.y; ++k) {  // a high-fanout driver (alone in its chunk): its pieces' merges
    const float E = reinterpret_cast<const float *>(D.piece_rat + pcs.x + k)[v];
    R = late ? fminf(R, E) : fmaxf(R, E);
  }
  // the driver's whole consumer record (RAT, NLDM load, type, padding) in
  // 8-byte parts, thread v part v, so no part of it is left for another pass
  const float r1 = __shfl_xor(R, 1), r2 = __shfl_xor(R, 2), r3 = __shfl_xor(R, 3);
  const float2 part = v == 0 ? make_float2(R, r1)
                      : v == 1 ? make_float2(r3, r2)
                      : v == 2 ? make_float2(L, __int_as_float(D.cell_type[xc]))
                               : make_float2(0.0f, 0.0f);
  if (live) {
    reinterpret_cast<float2 *>(&D.cons_rec[x])[v] = part;
    reinterpret_cast<float *>(D.drv_slack + x)[v] = late ? R - Av : Av - R;
  }
  if (pis) return;  // (wave-uniform: a chunk is PIs only or cells only)
  // (b) the RATs of the cells' input sinks
  const CellCtx cc = cell_ctx(D, lib, t, L);
  if constexpr (kSlots > 0) {
    float dl[kSlots > 0 ? kSlots : 1][2];
    slot_delays<kSlots>(D, cc, ro, isl, dl);
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
      const float r = push_rat(cc.sense, el, ro, R, dl[k][ro], dl[k][1 - ro], fs[k] >= 0);
      if (live && fs[k] >= 0) reinterpret_cast<float *>(D.sink_rat + fs[k])[2 * el + ro] = r;
    }
  } else {
    const TabLayout lay{D.nx, D.ny};
    const int f0 = D.fanin_ptr[xc], f1 = D.fanin_ptr[xc + 1];
    for (int f = f0; f < f1; ++f) {  // the lane pair of (el, *) runs the same fanins together
      const int sk = D.fanin_sink[f];
      const float *st = reinterpret_cast<const float *>(D.sink_state + sk);
      float dd[2];
#pragma unroll
      for (int ri = 0; ri < 2; ++ri) {
        const AxisPos px = axis_find(cc.tb + lay.xa(), cc.tb + lay.rdx(), D.nx, st[4 + 2 * el + ri]);
        dd[ri] = bilerp(cc.tb + lay.tab(ro), D.ny, px, cc.py);
      }
      const float r = push_rat(cc.sense, el, ro, R, dd[ro], dd[1 - ro], true);
      if (live) reinterpret_cast<float *>(D.sink_rat + sk)[2 * el + ro] = r;
    }
  }
}

// A piece of a high-fanout driver's sinks (rounds of one wave): the sinks'
// RATs as written by their consumers (or their endpoint constraints) and
// slacks, and the piece's merge of RAT_s - d for the driver's chunk.
__global__ __launch_bounds__(kSweepBlock) void k_backward_push_pieces(DevDesign D, int j0, int j1) {
  const int j = j0 + blockIdx.x * (kSweepBlock / kWave) + threadIdx.x / kWave;
  if (j >= j1) return;
  const int4 pr = D.piece_rec[j];
  const int sa = __builtin_amdgcn_readfirstlane(pr.y), sb = __builtin_amdgcn_readfirstlane(pr.z);
  float4 acc = make_float4(-kInf, -kInf, kInf, kInf);
  for (int s = sa + lane_id(); s < sb; s += kWave) {
    const int cons = D.sink_cons[s];
    const float d = D.dq[s].x;
    const float4 at = D.sink_state[s].at;
    float4 R = D.sink_rat[s];
    if (cons < 0) {
      R = D.ep_rat[-1 - cons];
      D.sink_rat[s] = R;
    }
    D.sink_slack[s] = slack4(at, R);
    acc = make_float4(fmaxf(acc.x, R.x - d), fmaxf(acc.y, R.y - d), fminf(acc.z, R.z - d), fminf(acc.w, R.w - d));
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    acc.x = fmaxf(acc.x, __shfl_xor(acc.x, off));
    acc.y = fmaxf(acc.y, __shfl_xor(acc.y, off));
    acc.z = fminf(acc.z, __shfl_xor(acc.z, off));
    acc.w = fminf(acc.w, __shfl_xor(acc.w, off));
  }
  if (lane_id() == 0) D.piece_rat[j] = acc;
}

// ------------------------------------------------ dataflow sweeps
//
// The flow schedule: one cooperative launch per sweep, every block resident,
// and no level barrier.  The sweep's items (the forward: per level its chunks,
// then its sink pieces; the backward: per level descending, its pieces, then
// its chunks) are dealt to the blocks round robin in that order; a block runs
// its items in order, and an item waits only for the items that produce its
// inputs, each of which publishes a completion flag (the update's epoch) once
// its stores are complete.  Every item waits only for earlier items and each
// block runs its items in order, so by induction over the item order every
// item completes.  The library is staged into LDS once per block.
//
// Values produced and consumed inside one sweep (input sink states and driver
// states forward, sink RATs and piece merges backward) and the flags are
// written and read with agent-scope relaxed atomics, which are coherent across
// the XCDs without an L2 write-back or invalidate; a producer waits for its
// stores to complete (vmcnt 0) and for its whole block before one thread
// stores the flag, and a consumer issues those loads only after its poll loop
// has seen every flag it needs.  A poll gives up after kFlowSpin rounds and
// raises err[0] (results are then wrong, but the kernel ends).
constexpr uint32_t kFlowSpin = 1u << 20;

__device__ __forceinline__ uint32_t ld_flag(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-wide wait until every thread's item ids (id < 0: none) show epoch.
// Once any wait of the sweep has given up (err raised), every wait passes, so
// the kernel drains quickly.  The exit is decided block-wide (every thread
// leaves the loop together).
__device__ __forceinline__ void flow_wait4(const uint32_t *flag, int4 ids, uint32_t epoch, uint32_t *err) {
  const int q[4] = {ids.x, ids.y, ids.z, ids.w};
  bool ready = false;
  for (uint32_t spin = 0;; ++spin) {
    bool all = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) all = all && (q[k] < 0 || ld_flag(flag + q[k]) == epoch);
    const bool mine = all || ld_flag(err) != 0u;
    ready = __syncthreads_and(mine);
    if (ready || spin >= kFlowSpin) break;
    __builtin_amdgcn_s_sleep(1);
  }
  if (!ready && threadIdx.x == 0) atomicOr(err, 1u);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);  // the coherent data loads stay after the poll
}

// Publishes item `id` once every store of the block has completed.
__device__ __forceinline__ void flow_publish(uint32_t *flag, int id, uint32_t epoch) {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag + id, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ float2 ld_coh2(const float *p) {
  const uint64_t u = __hip_atomic_load(reinterpret_cast<const uint64_t *>(p), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return make_float2(__uint_as_float((uint32_t)u), __uint_as_float((uint32_t)(u >> 32)));
}

__device__ __forceinline__ void st_coh1(float *p, float v) {
  __hip_atomic_store(reinterpret_cast<uint32_t *>(p), __float_as_uint(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// One forward chunk: the per-level kernel's arithmetic (thread 4 d + v on
// view v of driver d, the same merge order) on one 256-thread block.
template <int kSlots>
__device__ void flow_fwd_chunk(const DevDesign &D, const LdsLib &lib, PinState *wst, const FlowArgs &F, int c) {
  const int tid = threadIdx.x;
  const int dv = tid >> 2, v = tid & 3, el = v >> 1, ro = v & 1;
  const int4 cr4 = D.chunk_rec[c];
  const int x0 = __builtin_amdgcn_readfirstlane(cr4.x), x1 = __builtin_amdgcn_readfirstlane(cr4.y);
  const int s0 = __builtin_amdgcn_readfirstlane(cr4.z), s1 = __builtin_amdgcn_readfirstlane(cr4.w);
  const int x = x0 + dv;
  const bool live = x < x1;
  const int xc = live ? x : x0;
  const bool pis = x0 < D.n_pi;
  const int4 f4 = D.fanin4[xc];
  const int t = D.cell_type[xc];
  const float L = D.L_net[xc];
  const int xpi = min(xc, max(D.n_pi - 1, 0));
  const float pa = reinterpret_cast<const float *>(D.pi_at + xpi)[v];
  const float ps = reinterpret_cast<const float *>(D.pi_slew + xpi)[v];
  const int4 fi = pis ? make_int4(-1, -1, -1, -1) : F.fin_item[xc];
  const int sA = min(s0 + tid, max(s1 - 1, 0));
  const int dA = D.sink_drv[sA];
  const float2 wA = D.dq[sA];
  flow_wait4(F.flag, fi, F.epoch, F.err);
  const int fs[4] = {f4.x, f4.y, f4.z, f4.w};
  float2 iat[4], isl[4];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    const float *st = reinterpret_cast<const float *>(D.sink_state + max(fs[k], 0));
    iat[k] = ld_coh2(st + 2 * el);
    isl[k] = ld_coh2(st + 4 + 2 * el);
  }
  float at_v, sl_v;
  int cr_v = -1;
  if (pis) {
    at_v = pa;
    sl_v = ps;
  } else {
    const CellCtx cc = cell_ctx(D, lib, t, L);
    at_v = el ? -kInf : kInf;
    sl_v = el ? -kInf : kInf;
    float lse = 0.0f;
    merge_slots<kSlots>(D, cc, el, ro, iat, isl, fs, at_v, sl_v, cr_v, lse);
    if (el && D.gamma > 0.0f) at_v += D.gamma * logf(lse);
  }
  uint32_t cw = (uint32_t)(cr_v & 0xff) << (8 * v);
  cw |= __shfl_xor(cw, 1);
  cw |= __shfl_xor(cw, 2);
  if (live) {
    float *o = reinterpret_cast<float *>(D.drv_state + x);
    st_coh1(o + v, at_v);  // the driver's pieces read it in this sweep
    st_coh1(o + 4 + v, sl_v);
    if (v == 0) D.drv_crit[x] = pis ? 0xffffffffu : cw;
    float *w = reinterpret_cast<float *>(wst + dv);
    w[v] = at_v;
    w[4 + v] = sl_v;
  }
  lds_barrier();
  auto emit = [&](int s, int drv, float2 w) {
    const PinState ds = wst[drv - x0];
    PinState o;
    o.at = make_float4(ds.at.x + w.x, ds.at.y + w.x, ds.at.z + w.x, ds.at.w + w.x);
    o.slew = make_float4(sqrtf(ds.slew.x * ds.slew.x + w.y), sqrtf(ds.slew.y * ds.slew.y + w.y),
                         sqrtf(ds.slew.z * ds.slew.z + w.y), sqrtf(ds.slew.w * ds.slew.w + w.y));
    st_state<true>(D.sink_state + s, o);
  };
  if (s0 + tid < s1) emit(s0 + tid, dA, wA);
  for (int s = s0 + tid + kSweepBlock; s < s1; s += kSweepBlock) emit(s, D.sink_drv[s], D.dq[s]);
}

// One forward piece: sinks of a high-fanout driver from its published state.
__device__ void flow_fwd_piece(const DevDesign &D, const FlowArgs &F, int j) {
  const int4 pr = D.piece_rec[j];
  const int x = __builtin_amdgcn_readfirstlane(pr.x);
  const int sa = __builtin_amdgcn_readfirstlane(pr.y), sb = __builtin_amdgcn_readfirstlane(pr.z);
  const int owner = __builtin_amdgcn_readfirstlane(pr.w);
  flow_wait4(F.flag, make_int4(owner, -1, -1, -1), F.epoch, F.err);
  const PinState ds = ld_state<true>(D.drv_state + x);
  for (int s = sa + (int)threadIdx.x; s < sb; s += kSweepBlock) {
    const float2 w = D.dq[s];
    PinState o;
    o.at = make_float4(ds.at.x + w.x, ds.at.y + w.x, ds.at.z + w.x, ds.at.w + w.x);
    o.slew = make_float4(sqrtf(ds.slew.x * ds.slew.x + w.y), sqrtf(ds.slew.y * ds.slew.y + w.y),
                         sqrtf(ds.slew.z * ds.slew.z + w.y), sqrtf(ds.slew.w * ds.slew.w + w.y));
    st_state<true>(D.sink_state + s, o);
  }
}

template <int kSlots>
__global__ __launch_bounds__(kSweepBlock) void k_flow_fwd(DevDesign D, FlowArgs F) {
  extern __shared__ __align__(32) unsigned char smem[];
  const LdsLib lib = load_lib(D, smem);
  PinState *wst = reinterpret_cast<PinState *>(smem + lib_lds_bytes(D.n_types, D.tstride));
  __syncthreads();
  for (int i = blockIdx.x; i < F.n_items; i += gridDim.x) {
    const int2 it = F.items[i];
    const int kind = __builtin_amdgcn_readfirstlane(it.x), id = __builtin_amdgcn_readfirstlane(it.y);
    if (kind == kItemChunk) {
      flow_fwd_chunk<kSlots>(D, lib, wst, F, id);
      flow_publish(F.flag, id, F.epoch);
    } else {
      flow_fwd_piece(D, F, id);
      flow_publish(F.flag, D.n_chunks + id, F.epoch);
    }
  }
}

// One backward chunk: the per-level push kernel's arithmetic on one block,
// after the consumers of its sinks (and its pieces) have published.
template <int kSlots>
__device__ void flow_bwd_chunk(const DevDesign &D, const LdsLib &lib, int *wacc, const FlowArgs &F, int c) {
  const int tid = threadIdx.x;
  const int dv = tid >> 2, v = tid & 3, el = v >> 1, ro = v & 1;
  const int sel = tid & 1;
  const int4 cr4 = D.chunk_rec[c];
  const int x0 = __builtin_amdgcn_readfirstlane(cr4.x), x1 = __builtin_amdgcn_readfirstlane(cr4.y);
  const int s0 = __builtin_amdgcn_readfirstlane(cr4.z), s1 = __builtin_amdgcn_readfirstlane(cr4.w);
  const int x = x0 + dv;
  const bool live = x < x1;
  const int xc = live ? x : x0;
  const bool pis = x0 < D.n_pi;
  const int4 f4 = D.fanin4[xc];
  const int t = max(D.cell_type[xc], 0);
  const float L = D.L_net[xc];
  const int e = D.drv_ep[xc];
  const float Av = reinterpret_cast<const float *>(D.drv_state + xc)[v];
  const int2 pcs = D.chunk_pieces[c];
  const int fs[4] = {f4.x, f4.y, f4.z, f4.w};
  float2 isl[4];
#pragma unroll
  for (int k = 0; k < kSlots; ++k)
    isl[k] = *reinterpret_cast<const float2 *>(reinterpret_cast<const float *>(D.sink_state + max(fs[k], 0)) + 4 +
                                               2 * el);
  wacc[tid] = f2key((v >> 1) ? kInf : -kInf);
  // (a) the chunk's sinks, rounds of 128: wait for their consumers, then merge
  for (int base = s0; base < s1; base += kSweepBlock / 2) {
    const int s = base + (tid >> 1);
    const int sc = min(s, s1 - 1);
    const int cons = D.sink_cons[sc];
    const int drv = D.sink_drv[sc];
    const float d = D.dq[sc].x;
    const float2 at = *reinterpret_cast<const float2 *>(reinterpret_cast<const float *>(D.sink_state + sc) + 2 * sel);
    const int item = s < s1 ? F.sink_item[sc] : -1;
    // the pieces of a high-fanout driver join the first round's wait
    const int pw = base == s0 && tid < pcs.y ? D.n_chunks + pcs.x + tid : -1;
    flow_wait4(F.flag, make_int4(item, pw, -1, -1), F.epoch, F.err);
    if (s < s1) {
      float2 r;
      if (cons < 0) {
        r = *reinterpret_cast<const float2 *>(reinterpret_cast<const float *>(D.ep_rat + (-1 - cons)) + 2 * sel);
        *reinterpret_cast<float2 *>(reinterpret_cast<float *>(D.sink_rat + s) + 2 * sel) = r;
      } else {
        r = ld_coh2(reinterpret_cast<const float *>(D.sink_rat + s) + 2 * sel);
      }
      const float sk0 = sel ? r.x - at.x : at.x - r.x, sk1 = sel ? r.y - at.y : at.y - r.y;
      *reinterpret_cast<float2 *>(reinterpret_cast<float *>(D.sink_slack + s) + 2 * sel) = make_float2(sk0, sk1);
      int *acc = wacc + (drv - x0) * 4 + 2 * sel;
      if (sel) {
        atomicMin(acc + 0, f2key(r.x - d));
        atomicMin(acc + 1, f2key(r.y - d));
      } else {
        atomicMax(acc + 0, f2key(r.x - d));
        atomicMax(acc + 1, f2key(r.y - d));
      }
    }
  }
  lds_barrier();
  float R = key2f(wacc[tid]);
  const bool late = el != 0;
  if (live && e >= 0) {
    const float E = reinterpret_cast<const float *>(D.ep_rat + e)[v];
    R = late ? fminf(R, E) : fmaxf(R, E);
  }
  for (int k = 0; k < pcs.y; ++k) {
    const float2 E = ld_coh2(reinterpret_cast<const float *>(D.piece_rat + pcs.x + k) + 2 * el);
    const float Ev = ro ? E.y : E.x;
    R = late ? fminf(R, Ev) : fmaxf(R, Ev);
  }
  if (live) {
    reinterpret_cast<float *>(&D.cons_rec[x].rat)[v] = R;
    reinterpret_cast<float *>(D.drv_slack + x)[v] = late ? R - Av : Av - R;
  }
  if (!pis) {
    const CellCtx cc = cell_ctx(D, lib, t, L);
    float dl[kSlots][2];
    slot_delays<kSlots>(D, cc, ro, isl, dl);
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
      const float r = push_rat(cc.sense, el, ro, R, dl[k][ro], dl[k][1 - ro], fs[k] >= 0);
      if (live && fs[k] >= 0) st_coh1(reinterpret_cast<float *>(D.sink_rat + fs[k]) + 2 * el + ro, r);
    }
  }
  lds_barrier();  // wacc is reused by the block's next item
}

// One backward piece: RATs of a high-fanout driver's sinks once their
// consumers have published, and the piece's merge for the driver's chunk.
__device__ void flow_bwd_piece(const DevDesign &D, const FlowArgs &F, float4 *s_acc, int j) {
  const int4 pr = D.piece_rec[j];
  const int sa = __builtin_amdgcn_readfirstlane(pr.y), sb = __builtin_amdgcn_readfirstlane(pr.z);
  float4 acc = make_float4(-kInf, -kInf, kInf, kInf);
  for (int base = sa; base < sb; base += kSweepBlock) {
    const int s = base + (int)threadIdx.x;
    const int sc = min(s, sb - 1);
    flow_wait4(F.flag, make_int4(s < sb ? F.sink_item[sc] : -1, -1, -1, -1), F.epoch, F.err);
    if (s < sb) {
      const int cons = D.sink_cons[s];
      const float d = D.dq[s].x;
      const float4 at = D.sink_state[s].at;
      float4 R;
      if (cons < 0) {
        R = D.ep_rat[-1 - cons];
        D.sink_rat[s] = R;
      } else {
        const float2 a = ld_coh2(reinterpret_cast<const float *>(D.sink_rat + s));
        const float2 b = ld_coh2(reinterpret_cast<const float *>(D.sink_rat + s) + 2);
        R = make_float4(a.x, a.y, b.x, b.y);
      }
      D.sink_slack[s] = slack4(at, R);
      acc = make_float4(fmaxf(acc.x, R.x - d), fmaxf(acc.y, R.y - d), fminf(acc.z, R.z - d), fminf(acc.w, R.w - d));
    }
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    acc.x = fmaxf(acc.x, __shfl_xor(acc.x, off));
    acc.y = fmaxf(acc.y, __shfl_xor(acc.y, off));
    acc.z = fminf(acc.z, __shfl_xor(acc.z, off));
    acc.w = fminf(acc.w, __shfl_xor(acc.w, off));
  }
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) s_acc[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float4 a = s_acc[0];
    for (int k = 1; k < kSweepBlock / kWave; ++k)
      a = make_float4(fmaxf(a.x, s_acc[k].x), fmaxf(a.y, s_acc[k].y), fminf(a.z, s_acc[k].z), fminf(a.w, s_acc[k].w));
    st4<true>(D.piece_rat + j, a);
  }
  __syncthreads();
}

template <int kSlots>
__global__ __launch_bounds__(kSweepBlock) void k_flow_bwd(DevDesign D, FlowArgs F) {
  extern __shared__ __align__(32) unsigned char smem[];
  const LdsLib lib = load_lib(D, smem);
  int *wacc = reinterpret_cast<int *>(smem + lib_lds_bytes(D.n_types, D.tstride));
  float4 *s_acc = reinterpret_cast<float4 *>(wacc + kSweepBlock);
  __syncthreads();
  for (int i = blockIdx.x; i < F.n_items; i += gridDim.x) {
    const int2 it = F.items[i];
    const int kind = __builtin_amdgcn_readfirstlane(it.x), id = __builtin_amdgcn_readfirstlane(it.y);
    if (kind == kItemChunk) {
      flow_bwd_chunk<kSlots>(D, lib, wacc, F, id);
      flow_publish(F.flag, id, F.epoch);
    } else {
      flow_bwd_piece(D, F, s_acc, id);
      flow_publish(F.flag, D.n_chunks + id, F.epoch);
    }
  }
}

// ------------------------------------------------ persistent sweeps
//
// A sweep is a list of phases in order (`Phase`: the chunks of one level, or
// the sink pieces of one level's high-fanout drivers); every input of a phase
// comes from earlier phases, so a phase may start once the previous one is
// complete (which, by induction, implies all earlier ones).  Each phase has
// kDoneGroups completion counters whose sum counts its finished items.
//
// All loop control is wave-uniform: counter atomics are issued by every lane
// (lane 0 adds the count, the others 0, which the compiler folds into one
// wave-level atomic) and polled or ticketed values are broadcast with
// readfirstlane, so every loop exit is a scalar branch.  (With
// `if (lane == 0) atomic` at both ends of a loop, jump threading once merged
// the two regions into a lane-0-only path and the other lanes re-entered the
// loop without a ticket.)

constexpr int kSweepFwd = 0, kSweepBwd = 1;

__device__ __forceinline__ const int4 *sweep_phases(const DevDesign &D, int kind, int &n, int &ctr_base) {
  if (kind == kSweepBwd) {
    n = D.n_ph_bwd;
    ctr_base = D.n_ph_fwd;
    return D.phases + D.n_ph_fwd;
  }
  n = D.n_ph_fwd;
  ctr_base = 0;
  return D.phases;
}

__device__ __forceinline__ uint32_t *done_ctr(const DevDesign &D, int k) {
  return D.counters + kCtrPhases + (size_t)k * kDoneGroups;
}

__device__ __forceinline__ uint32_t *ticket_ctr(const DevDesign &D, int k) {
  return D.counters + kCtrPhases + (size_t)(D.n_ph_fwd + D.n_ph_bwd) * kDoneGroups + k;
}

// Polls until the phase's group counters sum to target.  Every lane loads one
// of the group words (lane & 7) and the sum is formed across 8 lanes.
__device__ __forceinline__ void wait_done(uint32_t *ctr, uint32_t target) {
  for (;;) {
    uint32_t v = __hip_atomic_load(ctr + (lane_id() & (kDoneGroups - 1)), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    if (__builtin_amdgcn_readfirstlane(v) >= target) break;
    __builtin_amdgcn_s_sleep(1);
  }
  // acquire at agent scope: the producers' stores (released with their count)
  // are visible to every load after this point, coherent or not
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ __forceinline__ int take_ticket(uint32_t *ctr) {
  const uint32_t old = atomicAdd(ctr, lane_id() == 0 ? 1u : 0u);
  return (int)__builtin_amdgcn_readfirstlane(old);
}

// A release at agent scope: every store of this wave before it is visible to
// a consumer that acquires the count (wait_done) after seeing it.
__device__ __forceinline__ void signal_add(uint32_t *ctr, uint32_t n) {
  __hip_atomic_fetch_add(ctr, lane_id() == 0 ? n : 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// The wide-net barrier's arrival: its data moves only through agent-scope
// atomic loads and stores, which are coherent across the device by
// themselves, so the count needs only those stores completed (vmcnt 0)
// before it moves, not the cache write-back of a release.
__device__ __forceinline__ void arrive_add(uint32_t *ctr, uint32_t n) {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __hip_atomic_fetch_add(ctr, lane_id() == 0 ? n : 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int kKind>
struct SweepPre {
  using type = int;
};
template <>
struct SweepPre<kSweepFwd> {
  using type = FwdPre;
};
template <>
struct SweepPre<kSweepBwd> {
  using type = BwdPre;
};

// What a chunk needs that the sweep does not produce, requested early.
template <int kKind>
__device__ __forceinline__ typename SweepPre<kKind>::type sweep_pre(const DevDesign &D, int c);
template <>
__device__ __forceinline__ FwdPre sweep_pre<kSweepFwd>(const DevDesign &D, int c) { return fwd_prefetch(D, c); }
template <>
__device__ __forceinline__ BwdPre sweep_pre<kSweepBwd>(const DevDesign &D, int c) { return bwd_prefetch(D, c); }

// (Dispatch is by template constant rather than lambdas: a lambda capturing
// the by-value kernel argument D by reference forces D into scratch memory.)
template <int kKind>
__device__ __forceinline__ void sweep_chunk(const DevDesign &D, const LdsLib &lib, unsigned char *wsm, int wave,
                                            float g_tns, float g_wns, const typename SweepPre<kKind>::type &p) {
  if constexpr (kKind == kSweepFwd) {
    fwd_finish<true>(D, lib, reinterpret_cast<PinState *>(wsm) + wave * kWave, p);
  } else {
    bwd_finish<true>(D, lib, reinterpret_cast<int *>(wsm) + wave * kWave * 4, p);
  }
}

template <int kKind>
__device__ __forceinline__ void sweep_piece(const DevDesign &D, const LdsLib &lib, int j) {
  if constexpr (kKind == kSweepFwd) fwd_piece<true>(D, j);
  if constexpr (kKind == kSweepBwd) bwd_piece<true>(D, lib, j);
}

// Cooperative schedule (every block resident, guaranteed by the cooperative
// launch): of each phase, wave w of W takes items first + w, first + w + W, ...
// A block with items in a phase first waits until the previous phase is
// complete (its first chunk's sweep-independent loads already in flight),
// runs them, waits for its waves' stores, and adds their number to its group
// counter; blocks without items in a phase skip it.  No per-item atomics.
template <int kKind>
__device__ __forceinline__ void sweep_coop(const DevDesign &D, const LdsLib &lib, unsigned char *wsm, float g_tns,
                                           float g_wns) {
  constexpr int kWaves = kSweepBlock / kWave;
  int n_ph = 0, base = 0;
  const int4 *ph = sweep_phases(D, kKind, n_ph, base);
  const int W = (int)gridDim.x * kWaves;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int b0 = blockIdx.x * kWaves;
  const int g = blockIdx.x & (kDoneGroups - 1);
  int prev_n = -1;
  for (int k = 0; k < n_ph; ++k) {
    const int4 P = ph[k];
    const int kind = __builtin_amdgcn_readfirstlane(P.x), first = __builtin_amdgcn_readfirstlane(P.y);
    const int n = __builtin_amdgcn_readfirstlane(P.z);
    int mine = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w)
      if (b0 + w < n) mine += (n - (b0 + w) + W - 1) / W;
    if (mine > 0) {
      const int cf = first + b0 + wave;
      const bool chunks = kind == kItemChunk;
      auto p = sweep_pre<kKind>(D, chunks && cf < first + n ? cf : 0);
      if (prev_n >= 0 && wave == 0) wait_done(done_ctr(D, base + k - 1), (uint32_t)prev_n);
      __syncthreads();
      for (int c = cf; c < first + n; c += W) {
        if (chunks) {
          if (c != cf) p = sweep_pre<kKind>(D, c);
          sweep_chunk<kKind>(D, lib, wsm, wave, g_tns, g_wns, p);
        } else {
          sweep_piece<kKind>(D, lib, c);
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (wave == 0) signal_add(done_ctr(D, base + k) + g, (uint32_t)mine);
    }
    prev_n = n;
  }
}

// Ticket schedule (any grid size): waves take the items of each phase from the
// phase's ticket counter in order and move to the next phase when it is
// exhausted; an item waits for the previous phase to complete.  Only running
// waves hold tickets, so the items of every earlier phase are in the hands of
// running waves and finish.
template <int kKind>
__device__ __forceinline__ void sweep_tickets(const DevDesign &D, const LdsLib &lib, unsigned char *wsm, float g_tns,
                                              float g_wns) {
  int n_ph = 0, base = 0;
  const int4 *ph = sweep_phases(D, kKind, n_ph, base);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  int prev_n = -1;
  for (int k = 0; k < n_ph; ++k) {
    const int4 P = ph[k];
    const int kind = __builtin_amdgcn_readfirstlane(P.x), first = __builtin_amdgcn_readfirstlane(P.y);
    const int n = __builtin_amdgcn_readfirstlane(P.z);
    for (;;) {
      const int t = take_ticket(ticket_ctr(D, base + k));
      if (t >= n) break;
      if (prev_n >= 0) wait_done(done_ctr(D, base + k - 1), (uint32_t)prev_n);
      if (kind == kItemChunk) {
        sweep_chunk<kKind>(D, lib, wsm, wave, g_tns, g_wns, sweep_pre<kKind>(D, first + t));
      } else {
        sweep_piece<kKind>(D, lib, first + t);
      }
      signal_add(done_ctr(D, base + k), 1u);
    }
    prev_n = n;
  }
}

template <int kKind, bool kCoop>
__global__ __launch_bounds__(kSweepBlock) void k_sweep(DevDesign D, float g_tns, float g_wns) {
  extern __shared__ __align__(32) unsigned char smem[];
  const LdsLib lib = load_lib(D, smem);
  __syncthreads();
  unsigned char *wsm = smem + lib_lds_bytes(D.n_types, D.tstride);
  if constexpr (kCoop)
    sweep_coop<kKind>(D, lib, wsm, g_tns, g_wns);
  else
    sweep_tickets<kKind>(D, lib, wsm, g_tns, g_wns);
}

// ------------------------------------------------- incremental update
//
// After the caps of a few nets change, only their fan-out cone needs new
// arrivals and only the fan-in cone of what changed needs new RATs.  A chunk
// is flagged for the forward sweep when a net of its drivers was recomputed
// (seeded) or when a sink feeding one of its drivers changed value; for the
// backward sweep when its forward pass changed a driver state (or its net was
// recomputed), or when a consumer of one of its sinks changed its RAT or load.
// "Changed" is a bitwise comparison with the stored value, so a flagged chunk
// whose result is unchanged stops the cone there.  A flagged chunk is
// recomputed with the same arithmetic as a full update, so the result is
// bitwise the full update's.  Flags always point to a strictly later phase (a
// consumer is at a higher level, a fan-in driver at a lower one).
//
// Two schedules share the flags.  While the cone is small, one cooperative
// launch per sweep walks per-phase queues of the flagged items (queue lengths
// are final once the previous phases are complete, so every block reads the
// same length after waiting for the last non-empty phase).  At the first
// phase whose queue exceeds a threshold the whole grid stops, records the
// phase, and the host continues with one launch per remaining phase whose
// blocks return at once for unflagged chunks.  The backward queues are built
// from the backward flags after the forward sweep.

__device__ __forceinline__ void st_coh_i32(int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_coh_i32(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Queue chunk c for the forward sweep (once).
__device__ __forceinline__ void inc_queue_fwd(const DevDesign &D, const IncArgs &I, int c) {
  if (__hip_atomic_exchange(I.flag + c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return;
  const int k = I.chunk_ph[c].x;
  const uint32_t pos = __hip_atomic_fetch_add(I.cnt + k, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  st_coh_i32(I.wl_c + D.phases[k].y + pos, c);
}

// Queue chunk c, and the sink pieces of its driver if it has any, for the
// backward sweep (once); a level's pieces run in the phase before its chunks.
__device__ __forceinline__ void inc_queue_bwd(const DevDesign &D, const IncArgs &I, int c) {
  if (__hip_atomic_exchange(I.flag + I.n_chunks + c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return;
  const int k = D.n_ph_fwd + I.chunk_ph[c].y;
  const uint32_t pos = __hip_atomic_fetch_add(I.cnt + k, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  st_coh_i32(I.wl_c + I.n_chunks + D.phases[k].y + pos, c);
  const int2 pcs = D.chunk_pieces[c];
  if (pcs.y > 0) {
    const uint32_t p0 = __hip_atomic_fetch_add(I.cnt + k - 1, (uint32_t)pcs.y, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
    int32_t *wl = I.wl_p + I.n_pieces + D.phases[k - 1].y + p0;
    for (int i = 0; i < pcs.y; ++i) st_coh_i32(wl + i, pcs.x + i);
  }
}

// Forward of one queued chunk: the drivers as in a full update; a driver whose
// state is unchanged and whose net was not recomputed keeps its sinks; changed
// sinks queue their consumers' chunks.
__device__ void inc_fwd_chunk(const DevDesign &D, const LdsLib &lib, PinState *wst, const IncArgs &I, int c) {
  const FwdPre p = fwd_prefetch(D, c);
  const int lane = lane_id();
  const int x0 = p.x0, x1 = p.x1, s1 = p.s1;
  const int x = x0 + lane;
  const bool live = x < x1;
  const int xc = live ? x : x0;
  const PinState old = D.drv_state[xc];
  const bool rcd = I.rcd[xc] != 0;
  PinState st;
  uint32_t crit = 0xffffffffu;
  if (x0 < D.n_pi) {
    st.at = p.pat;
    st.slew = p.psl;
  } else if (D.fanin4) {
    const int fs[4] = {p.f4.x, p.f4.y, p.f4.z, p.f4.w};
    PinState in[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) in[k] = ld_state<true>(D.sink_state + max(fs[k], 0));
    const CellCtx cc = cell_ctx(D, lib, p.t, p.L);
    Merge m;
    merge_init(m);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (fs[k] >= 0) merge_one(D, cc, in[k], k, m);
    merge_finish(D, m, st, crit);
  } else {
    cell_forward_csr<true>(D, lib, xc, st, crit);
  }
  const bool moved = live && !same_bits(st, old);
  if (live) {
    if (moved) st_state<true>(D.drv_state + x, st);
    D.drv_crit[x] = crit;
    wst[lane] = st;
  }
  const uint64_t redo = __ballot(live && (moved || rcd));
  wave_sync();
  if (redo == 0) return;
  if (lane == 0) {
    I.flag[I.n_chunks + c] = 1u;  // backward queues are built from these flags
    const int2 pcs = D.chunk_pieces[c];
    if (pcs.y > 0) {  // a high-fanout driver: its remaining sinks in the pieces phase that follows
      const int k = I.chunk_ph[c].x + 1;
      const uint32_t p0 = __hip_atomic_fetch_add(I.cnt + k, (uint32_t)pcs.y, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
      int32_t *wl = I.wl_p + D.phases[k].y + p0;
      for (int i = 0; i < pcs.y; ++i) st_coh_i32(wl + i, pcs.x + i);
    }
  }
  for (int s = p.s0 + lane; s < s1; s += kWave) {
    const int drv = D.sink_drv[s];
    if (!((redo >> (drv - x0)) & 1)) continue;
    const PinState ds = wst[drv - x0];
    const float2 w = D.dq[s];
    PinState o;
    o.at = make_float4(ds.at.x + w.x, ds.at.y + w.x, ds.at.z + w.x, ds.at.w + w.x);
    o.slew = make_float4(sqrtf(ds.slew.x * ds.slew.x + w.y), sqrtf(ds.slew.y * ds.slew.y + w.y),
                         sqrtf(ds.slew.z * ds.slew.z + w.y), sqrtf(ds.slew.w * ds.slew.w + w.y));
    if (same_bits(o, D.sink_state[s])) continue;
    st_state<true>(D.sink_state + s, o);
    const int cc = I.sink_cc[s];
    if (cc >= 0) inc_queue_fwd(D, I, cc);
  }
  wave_sync();
}

// Forward of one queued piece (its driver changed or its net was recomputed).
__device__ void inc_fwd_piece(const DevDesign &D, const IncArgs &I, int j) {
  const int4 pr = D.piece_rec[j];
  const int x = __builtin_amdgcn_readfirstlane(pr.x);
  const int sa = __builtin_amdgcn_readfirstlane(pr.y), sb = __builtin_amdgcn_readfirstlane(pr.z);
  const PinState ds = ld_state<true>(D.drv_state + x);
  for (int s = sa + lane_id(); s < sb; s += kWave) {
    const float2 w = D.dq[s];
    PinState o;
    o.at = make_float4(ds.at.x + w.x, ds.at.y + w.x, ds.at.z + w.x, ds.at.w + w.x);
    o.slew = make_float4(sqrtf(ds.slew.x * ds.slew.x + w.y), sqrtf(ds.slew.y * ds.slew.y + w.y),
                         sqrtf(ds.slew.z * ds.slew.z + w.y), sqrtf(ds.slew.w * ds.slew.w + w.y));
    if (same_bits(o, D.sink_state[s])) continue;
    st_state<true>(D.sink_state + s, o);
    const int cc = I.sink_cc[s];
    if (cc >= 0) inc_queue_fwd(D, I, cc);
  }
}

// Backward of one queued chunk, as in a full update; a driver whose RAT
// changed, or whose load changed (its net was recomputed, so the delays of
// its cell's input arcs did), queues the chunks of its fan-in sinks.
__device__ void inc_bwd_chunk(const DevDesign &D, const LdsLib &lib, int *wacc, const IncArgs &I, int c) {
  const BwdPre p = bwd_prefetch(D, c);
  const int lane = lane_id();
  const int x0 = p.x0, x1 = p.x1, s1 = p.s1;
  const int sA = p.s0 + lane;
  const int x = x0 + lane;
  const bool live = x < x1;
  const int xc = live ? x : x0;
  const float4 old = D.cons_rec[xc].rat;
  const bool rcd = I.rcd[xc] != 0;
  wacc[lane * 4 + 0] = f2key(-kInf);
  wacc[lane * 4 + 1] = f2key(-kInf);
  wacc[lane * 4 + 2] = f2key(kInf);
  wacc[lane * 4 + 3] = f2key(kInf);
  wave_sync();
  auto sink = [&](int s, const PinState &ss, int cons, float d, int drv) {
    const float4 R = sink_rat<true>(D, lib, ss, cons);
    D.sink_rat[s] = R;
    D.sink_slack[s] = slack4(ss.at, R);
    int *acc = wacc + (drv - x0) * 4;
    atomicMax(acc + 0, f2key(R.x - d));
    atomicMax(acc + 1, f2key(R.y - d));
    atomicMin(acc + 2, f2key(R.z - d));
    atomicMin(acc + 3, f2key(R.w - d));
  };
  if (sA < s1) sink(sA, p.ssA, p.consA, p.dA, p.drvA);
  if (sA + kWave < s1) sink(sA + kWave, p.ssB, p.consB, p.dB, p.drvB);
  for (int s = sA + 2 * kWave; s < s1; s += kWave) sink(s, D.sink_state[s], D.sink_cons[s], D.dq[s].x, D.sink_drv[s]);
  wave_sync();
  if (live) {
    float4 R = make_float4(key2f(wacc[lane * 4 + 0]), key2f(wacc[lane * 4 + 1]),
                           key2f(wacc[lane * 4 + 2]), key2f(wacc[lane * 4 + 3]));
    if (p.e >= 0) {
      const float4 E = D.ep_rat[p.e];
      R = make_float4(fmaxf(R.x, E.x), fmaxf(R.y, E.y), fminf(R.z, E.z), fminf(R.w, E.w));
    }
    for (int k = 0; k < p.pcs.y; ++k) {
      const float4 E = ld4<true>(D.piece_rat + p.pcs.x + k);
      R = make_float4(fmaxf(R.x, E.x), fmaxf(R.y, E.y), fminf(R.z, E.z), fminf(R.w, E.w));
    }
    const bool moved = !same_bits4(R, old);
    if (moved) st4<true>(&D.cons_rec[x].rat, R);
    D.drv_slack[x] = slack4(p.A, R);
    if ((moved || rcd) && x >= D.n_pi) {
      if (I.fanin_cc) {
        const int4 f4 = I.fanin_cc[x];
        const int fc[4] = {f4.x, f4.y, f4.z, f4.w};
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (fc[k] >= 0) inc_queue_bwd(D, I, fc[k]);
      } else {
        for (int f = D.fanin_ptr[x]; f < D.fanin_ptr[x + 1]; ++f)
          inc_queue_bwd(D, I, I.chunk_of[D.sink_drv[D.fanin_sink[f]]]);
      }
    }
  }
  wave_sync();
}

// One sweep over the queued items: wave w of W takes the items w, w + W, ...
// of each non-empty phase.  Every block reads each phase's queue length after
// the last non-empty phase has completed (all blocks are resident: cooperative
// launch), so all blocks agree on it and every loop ends.
template <int kKind>
__global__ __launch_bounds__(kSweepBlock) void k_inc_sweep(DevDesign D, IncArgs I, int max_items) {
  extern __shared__ __align__(32) unsigned char smem[];
  __shared__ uint32_t s_n[2];
  constexpr int kWaves = kSweepBlock / kWave;
  const LdsLib lib = load_lib(D, smem);
  __syncthreads();
  unsigned char *wsm = smem + lib_lds_bytes(D.n_types, D.tstride);
  int n_ph = 0, base = 0;
  const int4 *ph = sweep_phases(D, kKind, n_ph, base);
  const int W = (int)gridDim.x * kWaves;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int b0 = blockIdx.x * kWaves;
  const int g = blockIdx.x & (kDoneGroups - 1);
  const int off_c = kKind == kSweepBwd ? I.n_chunks : 0, off_p = kKind == kSweepBwd ? I.n_pieces : 0;
  int wait_k = -1;
  uint32_t wait_n = 0;
  for (int k = 0; k < n_ph; ++k) {
    if (wave == 0) {
      if (wait_k >= 0) wait_done(done_ctr(D, base + wait_k), wait_n);
      const uint32_t n = __hip_atomic_load(I.cnt + base + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (lane_id() == 0) s_n[k & 1] = n;
    }
    __syncthreads();
    const int n = (int)__builtin_amdgcn_readfirstlane(s_n[k & 1]);
    wait_k = -1;  // the last non-empty phase has completed
    if (n == 0) continue;
    if (n > max_items) {  // every block sees the same n: all stop here
      if (blockIdx.x == 0 && threadIdx.x == 0) I.stop[kKind == kSweepBwd] = k;
      return;
    }
    const int4 P = ph[k];
    const int kind = __builtin_amdgcn_readfirstlane(P.x), first = __builtin_amdgcn_readfirstlane(P.y);
    int mine = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w)
      if (b0 + w < n) mine += (n - (b0 + w) + W - 1) / W;
    for (int i = b0 + wave; i < n; i += W) {
      if (kind == kItemChunk) {
        const int c = __builtin_amdgcn_readfirstlane(ld_coh_i32(I.wl_c + off_c + first + i));
        if constexpr (kKind == kSweepFwd)
          inc_fwd_chunk(D, lib, reinterpret_cast<PinState *>(wsm) + wave * kWave, I, c);
        else
          inc_bwd_chunk(D, lib, reinterpret_cast<int *>(wsm) + wave * kWave * 4, I, c);
      } else {
        const int j = __builtin_amdgcn_readfirstlane(ld_coh_i32(I.wl_p + off_p + first + i));
        if constexpr (kKind == kSweepFwd)
          inc_fwd_piece(D, I, j);
        else
          bwd_piece<true>(D, lib, j);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (wave == 0 && mine > 0) signal_add(done_ctr(D, base + k) + g, (uint32_t)mine);
    wait_k = k;
    wait_n = (uint32_t)n;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) I.stop[kKind == kSweepBwd] = n_ph;
}

// Queues from flags, one block per phase of the sweep, in ascending id order
// and without atomics: the forward queues from the seeded forward flags (its
// pieces phases start empty: a high-fanout driver's chunk queues its pieces
// when it changes), the backward queues from the backward flags the forward
// sweep left (a flagged chunk's pieces included).
template <int kKind>
__global__ __launch_bounds__(256) void k_inc_queues(DevDesign D, IncArgs I) {
  __shared__ int s_cnt[256 / kWave];
  constexpr bool kBwd = kKind == kSweepBwd;
  const int k = (kBwd ? D.n_ph_fwd : 0) + blockIdx.x;
  const int4 P = D.phases[k];
  const bool pieces = P.x == kItemPiece;
  if (!kBwd && pieces) {
    if (threadIdx.x == 0) I.cnt[k] = 0u;
    return;
  }
  const int fo = kBwd ? I.n_chunks : 0;
  int32_t *wl = pieces ? I.wl_p + (kBwd ? I.n_pieces : 0) + P.y : I.wl_c + fo + P.y;
  const int wave = threadIdx.x / kWave, lane = lane_id();
  int total = 0;
  for (int b = 0; b < P.z; b += 256) {
    const int i = b + (int)threadIdx.x;
    bool f = false;
    if (i < P.z) {
      const int owner = pieces ? D.piece_rec[P.y + i].w : P.y + i;
      f = I.flag[fo + owner] != 0u;
    }
    const uint64_t m = __ballot(f);
    if (lane == 0) s_cnt[wave] = __popcll(m);
    __syncthreads();
    int before = total;
    for (int w = 0; w < wave; ++w) before += s_cnt[w];
    if (f) wl[before + __popcll(m & ((1ull << lane) - 1))] = P.y + i;
    for (int w = 0; w < 256 / kWave; ++w) total += s_cnt[w];
    __syncthreads();
  }
  if (threadIdx.x == 0) I.cnt[k] = (uint32_t)total;
}

// The flag targets of the incremental sweeps: per sink the chunk of its
// consumer (-1 at an endpoint), per driver the chunks holding the drivers of
// its cell's inline input sinks (-1 padded).
__global__ void k_inc_maps(DevDesign D, const int32_t *chunk_of, int32_t *sink_cc, int4 *fanin_cc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < D.n_sinks) {
    const int cons = D.sink_cons[i];
    sink_cc[i] = cons >= 0 ? chunk_of[cons] : -1;
  }
  if (fanin_cc && i < D.n_drv) {
    const int4 f = D.fanin4[i];
    const int fs[4] = {f.x, f.y, f.z, f.w};
    int o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = fs[k] >= 0 ? chunk_of[D.sink_drv[fs[k]]] : -1;
    fanin_cc[i] = make_int4(o[0], o[1], o[2], o[3]);
  }
}

// Seeds an incremental update from the caller's net ids: per net its driver
// ("net recomputed"), the forward flag of the driver's chunk, and the flag of
// the RC chunk or wide net that recomputes it (plain stores of 1; the queues
// are built from the flags afterwards, without atomics).
__global__ void k_inc_seed(DevDesign D, IncArgs I, const int32_t *nets, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int x = I.net_slot[nets[i]];
  I.rcd[x] = 1;
  I.flag[I.chunk_of[x]] = 1u;
  const int r = I.slot_rc[x];
  if (r >= 0)
    I.rc_flag[r] = 1u;
  else
    I.wide_flag[-1 - r] = 1u;
}

// ------------------------------------------------------------------ RC

__device__ __forceinline__ float rc_tree_lds(const uint8_t *par, const float *R, const float *C,
                                             float *A, float *B, int b, int m) {
  for (int k = m - 1; k >= 1; --k) A[b + par[b + k]] += A[b + k];
  const float load = A[b];
  B[b] = 0.0f;
  A[b] = 0.0f;
  for (int k = 1; k < m; ++k) {
    const float c = C[b + k];  // read before B[b + k] is written: B may be C
    const float d = B[b + par[b + k]] + R[b + k] * A[b + k];
    B[b + k] = d;
    A[b + k] = c * d;
  }
  for (int k = m - 1; k >= 1; --k) A[b + par[b + k]] += A[b + k];
  A[b] = 0.0f;
  for (int k = 1; k < m; ++k) A[b + k] = A[b + par[b + k]] + R[b + k] * A[b + k];
  return load;
}

// ---- wide nets: FP64 scans over the DFS preorder ---------------------------
//
// In preorder the subtree of node k is the index range [k, end_k), so
//   load_k = sum of C^ over [k, end_k)           = P[end_k] - P[k]   (P = exclusive scan of C^)
//   ld_k   = sum of C^ d over [k, end_k)         (same with C^ d)
// and a path sum over the ancestors-or-self of k (the a with a <= k < end_a) is
//   sum_{p <= k} (w_p - E_p),   E_p = sum of w_a over the nodes a with end_a = p,
// which gives d (w = R load) and m2 (w = R ld).  The nodes are listed grouped by
// end position (egl, offsets egp), so E is a difference of an FP64 prefix over
// that list.  FP64 keeps the prefix differences exact far below FP32
// resolution.
//
// A net of m nodes is shared by ceil(m / kWideSeg) blocks of 1024 threads, block
// b owning preorder segment [b kWideSeg, (b+1) kWideSeg).  Scans run as a
// segment reduction, a barrier among the net's blocks, a carry summed over the
// earlier segments in block order (deterministic), and the segment scan.
// Values one block writes and another reads (the FP64 scratch arrays) go
// through agent-scope relaxed 64-bit atomics, and a block waits for its stores
// before it arrives at a barrier (the persistent-sweep protocol).  The blocks
// of a net never wait on anything but each other, so every block of a net
// eventually runs; the last block to leave resets the net's counters for the
// next launch (stream-ordered after this one).

struct WideCtx {
  int m, k0, k1, b, nblk;
  uint32_t *arrive, *leave;
  double *tot;
  uint32_t passed;
};

__device__ __forceinline__ double ldc(const double *p) {
  return __longlong_as_double(
      __hip_atomic_load(reinterpret_cast<const long long *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

__device__ __forceinline__ void stc(double *p, double v) {
  __hip_atomic_store(reinterpret_cast<long long *>(p), __double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier among the blocks of one net.
__device__ void wide_sync(WideCtx &c) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  ++c.passed;
  if (c.nblk > 1 && threadIdx.x < kWave) {
    arrive_add(c.arrive, 1u);
    const uint32_t target = c.passed * (uint32_t)c.nblk;
    for (;;) {
      const uint32_t v = __hip_atomic_load(c.arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (__builtin_amdgcn_readfirstlane(v) >= target) break;
      __builtin_amdgcn_s_sleep(1);
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  }
  __syncthreads();
}

// out[k] = load(k) over the block's segment; each thread requests kMapUnroll
// elements (strided by the block) before storing any.
constexpr int kMapUnroll = 4;

template <class Load, class Store>
__device__ __forceinline__ void seg_map(int k0, int k1, Load load, Store store) {
  using V = decltype(load(0));
  const int nt = blockDim.x;
  for (int b = k0 + (int)threadIdx.x; b < k1; b += kMapUnroll * nt) {
    V v[kMapUnroll];
#pragma unroll
    for (int u = 0; u < kMapUnroll; ++u) v[u] = load(min(b + u * nt, k1 - 1));
#pragma unroll
    for (int u = 0; u < kMapUnroll; ++u)
      if (b + u * nt < k1) store(b + u * nt, v[u]);
  }
  __syncthreads();
}

// Sum of in over [k0, k1) in a fixed order (per thread, then a fixed tree).
__device__ double block_sum(const double *in, int k0, int k1, double *s_w) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave, nw = blockDim.x / kWave;
  double acc = 0.0;
  for (int b = k0 + tid; b < k1; b += kMapUnroll * blockDim.x) {
    double v[kMapUnroll];
#pragma unroll
    for (int u = 0; u < kMapUnroll; ++u) v[u] = ldc(in + min(b + u * (int)blockDim.x, k1 - 1));
#pragma unroll
    for (int u = 0; u < kMapUnroll; ++u)
      if (b + u * (int)blockDim.x < k1) acc += v[u];
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) s_w[wid] = acc;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < nw; ++w) t += s_w[w];
  __syncthreads();
  return t;
}

// Scan of in[0, m) into out over the net's blocks: exclusive with out[m] =
// total, or inclusive; in may alias out.  Ends with a barrier, so every block
// may read any of out afterwards.
constexpr int kScanPer = 8;

__device__ void wide_scan(WideCtx &c, const double *in, double *out, bool exclusive, double *s_w) {
  const double part = block_sum(in, c.k0, c.k1, s_w);
  if (c.nblk > 1) {
    if (threadIdx.x == 0) stc(c.tot + c.b, part);
    wide_sync(c);
  }
  double carry = 0.0;
  for (int q = 0; q < c.b; ++q) carry += ldc(c.tot + q);
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int nw = blockDim.x / kWave;
  const int tile = blockDim.x * kScanPer;
  for (int base = c.k0; base < c.k1; base += tile) {
    const int i0 = base + tid * kScanPer;
    double x[kScanPer];
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) x[j] = ldc(in + min(i0 + j, c.k1 - 1));
    double run = 0.0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      if (i0 + j >= c.k1) x[j] = 0.0;
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
      if (i0 + j < c.k1) stc(out + i0 + j, exclusive ? pre : pre + x[j]);
      pre += x[j];
    }
    carry += s_w[nw];
    __syncthreads();
  }
  if (exclusive && c.b == c.nblk - 1 && threadIdx.x == 0) stc(out + c.m, carry);
  wide_sync(c);
}

// X[k] = R[k] (subtree sum of the values whose exclusive prefix is P) for k > 0,
// X[0] = 0, over the block's segment; then a barrier.
__device__ __forceinline__ void wide_edge(WideCtx &c, const float *R, const double *P, const int32_t *end,
                                          double *X) {
  seg_map(c.k0, c.k1, [=](int k) { return k ? (double)R[k] * (ldc(P + end[k]) - ldc(P + k)) : 0.0; },
          [=](int k, double v) { stc(X + k, v); });
  wide_sync(c);
}

// Path sums from edge terms X (complete over the net; X[0] = 0):
// out[p] = sum over the ancestors-or-self a of p of X[a].
__device__ void wide_path_sum(WideCtx &c, const double *X, const int32_t *egp, const int32_t *egl, double *V,
                              double *out, double *s_w) {
  seg_map(c.k0, c.k1, [=](int i) { return ldc(X + egl[i]); }, [=](int i, double v) { stc(V + i, v); });
  wide_scan(c, V, V, true, s_w);
  seg_map(c.k0, c.k1, [=](int p) { return ldc(X + p) - (ldc(V + egp[p + 1]) - ldc(V + egp[p])); },
          [=](int p, double v) { stc(out + p, v); });
  wide_scan(c, out, out, false, s_w);
}

__device__ WideCtx wide_ctx(const BigNet &B, const WideNets &W, int seg, int net) {
  WideCtx c;
  c.m = B.m;
  c.b = seg;
  c.nblk = B.nblk;
  c.k0 = seg * kWideSeg;
  c.k1 = min(B.m, c.k0 + kWideSeg);
  c.arrive = W.sync + 2 * net;
  c.leave = W.sync + 2 * net + 1;
  c.tot = W.tot + B.tot;
  c.passed = 0;
  return c;
}

// The last block of a net to finish resets the net's counters.
__device__ void wide_leave(WideCtx &c) {
  __syncthreads();
  if (c.nblk > 1 && threadIdx.x < kWave) {
    const uint32_t old = atomicAdd(c.leave, lane_id() == 0 ? 1u : 0u);
    if (__builtin_amdgcn_readfirstlane(old) == (uint32_t)(c.nblk - 1) && lane_id() == 0) {
      *c.arrive = 0u;
      *c.leave = 0u;
    }
  }
}

__device__ void rc_wide_net(const DevDesign &D, const BigNet &B, const WideNets &W, WideCtx &c, double *s_w) {
  const int x = B.x, m = B.m;
  const int k0 = D.rc_ptr[x];
  const float *R = D.rc_res + k0;
  const float *Cw = D.rc_cap + k0;
  const int32_t *end = W.end + B.aux;
  const float *pc = W.pc + B.aux;
  const int32_t *egp = W.egp + B.egp, *egl = W.egl + B.aux;
  const int st = m + 1;
  double *A = W.scratch + B.scr, *P = A + st, *X = P + st, *Y = X + st, *V = Y + st;
  seg_map(c.k0, c.k1, [=](int k) { return (double)Cw[k] + (double)pc[k]; }, [=](int k, double v) { stc(A + k, v); });
  wide_scan(c, A, P, true, s_w);                                           // P: prefix of C^
  const double total = ldc(P + m);
  wide_edge(c, R, P, end, X);                                              // R load
  wide_path_sum(c, X, egp, egl, V, Y, s_w);                                // Y: d
  seg_map(c.k0, c.k1, [=](int k) { return ldc(A + k) * ldc(Y + k); }, [=](int k, double v) { stc(X + k, v); });
  wide_scan(c, X, P, true, s_w);                                           // P: prefix of C^ d
  wide_edge(c, R, P, end, X);                                              // R ld
  wide_path_sum(c, X, egp, egl, V, A, s_w);                                // A: m2
  if (c.b == 0 && threadIdx.x == 0) {
    D.L_net[x] = (float)total;
    if (D.rc_cons_l) D.cons_rec[x].L = (float)total;
  }
  // the net's sinks, split evenly over its blocks
  const int s0 = D.sink_ptr[x], ns = D.sink_ptr[x + 1] - s0;
  const int per = (ns + c.nblk - 1) / c.nblk;
  const int j0 = min(ns, c.b * per), j1 = min(ns, j0 + per);
  const int32_t *snode = D.sink_node + s0;
  float2 *dq = D.dq + s0;
  seg_map(j0, j1,
          [=](int j) {
            const int k = snode[j];
            const double d = ldc(Y + k);
            return make_float2((float)d, (float)fmax(0.0, 2.0 * ldc(A + k) - d * d));
          },
          [=](int j, float2 v) { dq[j] = v; });
  wide_leave(c);
}

// Wide nets: blocks of 1024 threads, several per net (launched on a side
// stream so they overlap the small-net kernel).
// only: optional per-wide-net flags; the blocks of an unflagged net return
// together, before touching the net's barrier counters.
__global__ __launch_bounds__(kWideBlock) void k_rc_wide(DevDesign D, WideNets W, const uint32_t *only) {
  __shared__ double s_w[kWideBlock / kWave + 1];
  const int2 nb = W.blk[blockIdx.x];
  if (only && only[nb.x] == 0u) return;
  const BigNet &B = W.big[nb.x];
  WideCtx c = wide_ctx(B, W, nb.y, nb.x);
  rc_wide_net(D, B, W, c, s_w);
}

// ---- reduced-order (Arnoldi) net delay -------------------------------------
//
// The step response of the tree (root driven by a unit step) is projected on
// the Krylov space {d, A d} of A = G^-1 C in the G inner product, where A is
// self-adjoint, so Arnoldi is the Lanczos recurrence.  For vectors in the
// range of A, <A x, A y>_G = x^T C A y, so the whole two-step process needs
// only four sums over the net's non-root nodes,
//   S1 = sum C^ d, S2 = sum C^ d^2, S3 = sum C^ d m2, S4 = sum C^ m2^2,
// with d the Elmore delays and m2 = A d the second moments the RC pass already
// forms (sum C^ m2 = S2 is one of the identities):
//   alpha1 = S2 / S1,  beta1^2 = (S3 S1 - S2^2) / S1^2,
//   alpha2 = (S4 - 2 alpha1 S3 + alpha1^2 S2) / (S1 beta1^2),
// T = [[alpha1, beta1], [beta1, alpha2]] = U diag(tau) U^T, and at a node
//   1 - Y(t) = sum_j a_j exp(-t / tau_j),
//   a_j = u_1j (u_1j d + u_2j (m2 - alpha1 d) / beta1) / tau_j,
// which keeps the node's first two time moments (d and m2).  beta1^2 at or
// below 1e-24 alpha1^2 leaves the one-pole model a = d / alpha1,
// tau = alpha1.  The delay is the first time the response reaches 1/2: 0 when
// it starts at or above it, else 64 bisections of [0, t_hi], t_hi the first
// doubling of the largest tau where 1 - Y < 1/2.  All in FP64.
struct Red2 {
  double tau0, tau1;      // kept poles (1.0 where absent: its weight is 0)
  double u10, u20, u11, u21;  // first and second components of their eigenvectors
  double alpha1, inv_b1;  // inv_b1 = 0 for the one-pole model
  bool p0, p1;            // which poles are kept
};

__device__ Red2 red2_model(double S1, double S2, double S3, double S4) {
  Red2 r{1.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, false, false};
  if (!(S1 > 0.0)) return r;
  const double a1 = S2 / S1;
  const double b1sq = (S3 * S1 - S2 * S2) / (S1 * S1);
  r.alpha1 = a1;
  if (!(b1sq > 1e-24 * a1 * a1)) {
    if (a1 > 0.0) {
      r.p0 = true;
      r.tau0 = a1;
      r.u10 = 1.0;
    }
    return r;
  }
  const double b1 = sqrt(b1sq);
  const double a2 = (S4 - 2.0 * a1 * S3 + a1 * a1 * S2) / (S1 * b1sq);
  const double h = 0.5 * (a1 - a2), rad = sqrt(h * h + b1sq), mean = 0.5 * (a1 + a2);
  r.inv_b1 = 1.0 / b1;
  // eigenvector of [[a1, b1], [b1, a2]] for lam: (b1, lam - a1) or (lam - a2, b1), the longer
  auto vec = [&](double lam, double &v1, double &v2) {
    v1 = b1;
    v2 = lam - a1;
    const double w1 = lam - a2, w2 = b1;
    if (w1 * w1 + w2 * w2 > v1 * v1 + v2 * v2) {
      v1 = w1;
      v2 = w2;
    }
    const double nv = 1.0 / sqrt(v1 * v1 + v2 * v2);
    v1 *= nv;
    v2 *= nv;
  };
  const double l0 = mean + rad, l1 = mean - rad;
  if (l0 > 0.0) {
    r.p0 = true;
    r.tau0 = l0;
    vec(l0, r.u10, r.u20);
  }
  if (l1 > 0.0) {
    r.p1 = true;
    r.tau1 = l1;
    vec(l1, r.u11, r.u21);
  }
  return r;
}

__device__ double red2_half_time(const Red2 &r, double d, double m2) {
  if (!r.p0 && !r.p1) return 0.0;
  const double e = (m2 - r.alpha1 * d) * r.inv_b1;  // 0 for the one-pole model
  const double a0 = r.p0 ? r.u10 * (r.u10 * d + r.u20 * e) / r.tau0 : 0.0;
  const double a1 = r.p1 ? r.u11 * (r.u11 * d + r.u21 * e) / r.tau1 : 0.0;
  // a missing pole has a = 0; its rate is set to 0 so its term stays finite
  const double k0 = r.p0 ? 1.0 / r.tau0 : 0.0, k1 = r.p1 ? 1.0 / r.tau1 : 0.0;
  if (a0 + a1 - 0.5 <= 0.0) return 0.0;
  const double tmax = fmax(r.p0 ? r.tau0 : 0.0, r.p1 ? r.tau1 : 0.0);
  // The impulse response a0 k0 e^{-k0 t} + a1 k1 e^{-k1 t} changes sign at
  // most once, so f(t) = a0 e^{-k0 t} + a1 e^{-k1 t} - 1/2 has exactly one
  // root in (0, inf).  Each solve below is Newton kept inside a bracket
  // [lo, hi] with f(lo) > 0 >= f(hi) (the first doubling of tau_max), with a
  // bisection whenever a step leaves it.
  // 1) FP32 with the hardware exponential, from the Elmore delay times ln 2
  //    (the one-pole answer), to about 1e-6.
  const float a0f = (float)a0, a1f = (float)a1, k0f = (float)k0, k1f = (float)k1;
  auto ff = [&](float t) { return a0f * __expf(-t * k0f) + a1f * __expf(-t * k1f) - 0.5f; };
  float lof = 0.0f, hif = (float)tmax;
  for (int i = 0; i < 300 && ff(hif) > 0.0f; ++i) hif *= 2.0f;
  float tf = 0.6931472f * (float)d;
  if (!(tf > lof && tf < hif)) tf = 0.5f * hif;
  for (int i = 0; i < 60; ++i) {
    const float e0 = __expf(-tf * k0f), e1 = __expf(-tf * k1f);
    const float ft = a0f * e0 + a1f * e1 - 0.5f;
    const float dft = -(a0f * k0f * e0 + a1f * k1f * e1);
    if (ft > 0.0f)
      lof = tf;
    else
      hif = tf;
    float tn = tf - ft / dft;
    if (!(tn > lof && tn < hif)) tn = 0.5f * (lof + hif);
    const bool done = fabsf(tn - tf) <= 1e-6f * tf || hif - lof <= 1e-7f * hif;
    tf = tn;
    if (done) break;
  }
  // 2) One FP64 Newton step from there.  A step under 1e-5 of t means the
  //    FP32 root was that close, and the step (quadratic convergence) leaves
  //    an error near 1e-10 of t.
  {
    const double t = (double)tf;
    const double e0 = exp(-t * k0), e1 = exp(-t * k1);
    const double ft = a0 * e0 + a1 * e1 - 0.5;
    const double dft = -(a0 * k0 * e0 + a1 * k1 * e1);
    const double tn = t - ft / dft;
    if (t > 0.0 && fabs(tn - t) <= 1e-5 * t) return tn;
  }
  // 3) Otherwise (FP32 too coarse for this model) the whole solve in FP64,
  //    until a step moves t by under 1e-13 of itself.
  auto f = [&](double t) { return a0 * exp(-t * k0) + a1 * exp(-t * k1) - 0.5; };
  double hi = tmax;
  for (int i = 0; i < 1100 && f(hi) > 0.0; ++i) hi *= 2.0;
  double lo = 0.0, t = 0.5 * hi;
  for (int i = 0; i < 200; ++i) {
    const double e0 = exp(-t * k0), e1 = exp(-t * k1);
    const double ft = a0 * e0 + a1 * e1 - 0.5;
    const double dft = -(a0 * k0 * e0 + a1 * k1 * e1);
    if (ft > 0.0)
      lo = t;
    else
      hi = t;
    double tn = t - ft / dft;
    if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);  // also catches dft = 0 (NaN or inf)
    const bool done = fabs(tn - t) <= 1e-13 * t || hi - lo <= 1e-15 * hi;
    t = tn;
    if (done) break;
  }
  return t;
}

// Stages nodes [k0, k0 + nk) of one RC chunk into LDS: parent, R and
// C^ = C + lumped pin caps.  Each thread requests all of its (clamped,
// unpredicated) loads before its first LDS store.
template <int kNodes = kRcChunkNodes, int kThreads = kRcBlock>
__device__ __forceinline__ void stage_rc_nodes(const DevDesign &D, int k0, int nk, uint8_t *par, float *R,
                                               float *C, float *A) {
  constexpr int kPer = kNodes / kThreads;
  const int tid = threadIdx.x;
  const int last = k0 + max(nk - 1, 0);
  uint8_t p[kPer];
  float r[kPer], c[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int i = min(k0 + u * kThreads + tid, last);
    p[u] = D.rc_par8[i];
    r[u] = D.rc_res[i];
    c[u] = D.rc_cap[i];  // wire + pin caps (C^)
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int i = u * kThreads + tid;
    if (i < nk) {
      par[i] = p[u];
      R[i] = r[u];
      C[i] = c[u];
      A[i] = c[u];
    }
  }
}

constexpr int kSinkRound = 8;  // sink node ids a lane requests together in the RC kernels

// Reduced-order sink delays of one RC chunk, after every thread has run its
// net's tree passes (d in s_B, m2 in s_A, C^ in s_C): each thread builds its
// net's two-pole model into LDS, then the block's sinks are shared out evenly
// (sink f of the chunk's concatenated sink lists goes to thread f mod the
// block size), so a net with many sinks no longer holds up its wavefront.
__device__ __forceinline__ void rc_reduced_sinks(const DevDesign &D, bool live, int2 sr, const float *s_C,
                                                 const float *s_A, const float *s_B, const int *s_base) {
  __shared__ double s_mod[8][kRcBlock];
  __shared__ uint8_t s_pole[kRcBlock];
  __shared__ int s_sx[kRcBlock], s_pf[kRcBlock + 1], s_wsum[kRcBlock / kWave];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  int cnt = 0;
  if (live) {
    const int b = s_base[tid], m = s_base[tid + 1] - b;
    double S1 = 0.0, S2 = 0.0, S3 = 0.0, S4 = 0.0;
    for (int k = 1; k < m; ++k) {
      const double c = s_C[b + k], d = s_B[b + k], m2 = s_A[b + k];
      S1 += c * d;
      S2 += c * d * d;
      S3 += c * d * m2;
      S4 += c * m2 * m2;
    }
    const Red2 r = red2_model(S1, S2, S3, S4);
    s_mod[0][tid] = r.tau0;
    s_mod[1][tid] = r.tau1;
    s_mod[2][tid] = r.u10;
    s_mod[3][tid] = r.u20;
    s_mod[4][tid] = r.u11;
    s_mod[5][tid] = r.u21;
    s_mod[6][tid] = r.alpha1;
    s_mod[7][tid] = r.inv_b1;
    s_pole[tid] = (uint8_t)((r.p0 ? 1 : 0) | (r.p1 ? 2 : 0));
    cnt = sr.y - sr.x;
  }
  s_sx[tid] = sr.x;
  // exclusive prefix of the sink counts: a scan per wavefront, then the
  // wavefront totals
  int v = cnt;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(v, o, kWave);
    v += lane >= o ? y : 0;
  }
  if (lane == kWave - 1) s_wsum[wave] = v;
  lds_barrier();
  int off = 0;
  for (int w = 0; w < wave; ++w) off += s_wsum[w];
  s_pf[tid + 1] = off + v;
  if (tid == 0) s_pf[0] = 0;
  lds_barrier();
  const int total = s_pf[kRcBlock];
  for (int f = tid; f < total; f += kRcBlock) {
    int lo = 0, hi = kRcBlock;  // s_pf[lo] <= f < s_pf[hi]: lo owns sink f (its count is > 0)
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_pf[mid] <= f)
        lo = mid;
      else
        hi = mid;
    }
    const int sk = s_sx[lo] + (f - s_pf[lo]);
    const int k = s_base[lo] + D.sink_node[sk];
    Red2 r;
    r.tau0 = s_mod[0][lo];
    r.tau1 = s_mod[1][lo];
    r.u10 = s_mod[2][lo];
    r.u20 = s_mod[3][lo];
    r.u11 = s_mod[4][lo];
    r.u21 = s_mod[5][lo];
    r.alpha1 = s_mod[6][lo];
    r.inv_b1 = s_mod[7][lo];
    r.p0 = (s_pole[lo] & 1) != 0;
    r.p1 = (s_pole[lo] & 2) != 0;
    const float d = s_B[k];
    D.dq[sk] = make_float2((float)red2_half_time(r, d, s_A[k]), fmaxf(0.0f, 2.0f * s_A[k] - d * d));
  }
}

// Small nets: one block per chunk of <= 256 nets (<= kRcChunkNodes nodes,
// consecutive in RC order): coalesced staging of parent/R/C into LDS, one net
// per thread, each thread writing its net's load and sink moments (kRed: the
// sink delays of the reduced-order model instead of Elmore's).  Block 0 also
// clears the sweep counters for the launches that follow.
// The Elmore form keeps its LDS at 27,136 bytes, six blocks per CU (the
// register limit; 35,844 bytes held it to four, 12% slower): the delays
// overwrite C^ in place and the nets' node offsets are 16-bit, the last net
// ending at the chunk's end.
// only: optional per-chunk flags (incremental update: unflagged chunks return).
template <bool kRed>
__global__ __launch_bounds__(kRcBlock) void k_rc(DevDesign D, const int2 *chunks, int n_chunks,
                                                 uint32_t *counters, int n_counters, const uint32_t *only) {
  const int tid = threadIdx.x;
  if (blockIdx.x == 0)
    for (int i = tid; i < n_counters; i += kRcBlock) counters[i] = 0u;
  const int ci = xcd_major(n_chunks);
  if (ci >= n_chunks || (only && only[ci] == 0u)) return;
  const int2 ch = chunks[ci];
  const int j0 = ch.x, j1 = ch.y;
  const int k0 = D.rc_start[j0], nk = D.rc_start[j1] - k0;
  const int j = j0 + tid;
  const int jc = j < j1 ? j : j0;
  const int x = D.rc_order[jc];
  const int2 sr = D.rc_sinks[jc];
  if constexpr (kRed) {  // reduced-order delays replace the Elmore ones
    __shared__ uint8_t s_par[kRcChunkNodes];
    __shared__ float s_R[kRcChunkNodes], s_C[kRcChunkNodes], s_A[kRcChunkNodes], s_B[kRcChunkNodes];
    __shared__ int s_base[kRcBlock + 1];
    stage_rc_nodes(D, k0, nk, s_par, s_R, s_C, s_A);
    for (int i = tid; i <= j1 - j0; i += kRcBlock) s_base[i] = D.rc_start[j0 + i] - k0;
    lds_barrier();
    if (j < j1) {
      const float L = rc_tree_lds(s_par, s_R, s_C, s_A, s_B, s_base[tid], s_base[tid + 1] - s_base[tid]);
      D.L_net[x] = L;
      if (D.rc_cons_l) D.cons_rec[x].L = L;
    }
    rc_reduced_sinks(D, j < j1, j < j1 ? sr : make_int2(0, 0), s_C, s_A, s_B, s_base);
  } else {
    __shared__ uint8_t s_par[kRcChunkNodes];
    __shared__ float s_R[kRcChunkNodes], s_C[kRcChunkNodes], s_A[kRcChunkNodes];
    __shared__ uint16_t s_base[kRcBlock];
    static_assert(kRcChunkNodes <= 65536, "16-bit node offsets");
    stage_rc_nodes(D, k0, nk, s_par, s_R, s_C, s_A);
    for (int i = tid; i < j1 - j0; i += kRcBlock) s_base[i] = (uint16_t)(D.rc_start[j0 + i] - k0);
    // the first sinks' node ids, in flight across the tree passes
    constexpr int kPre = 4;
    int sn[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) sn[u] = D.sink_node[min(sr.x + u, max(sr.y - 1, 0))];
    lds_barrier();
    if (j < j1) {
      const int b = s_base[tid], m = (j + 1 < j1 ? (int)s_base[tid + 1] : nk) - b;
      const int s0 = sr.x, s1 = sr.y;
      const float L = rc_tree_lds(s_par, s_R, s_C, s_A, s_C, b, m);  // d in s_C, m2 in s_A
      D.L_net[x] = L;
      if (D.rc_cons_l) D.cons_rec[x].L = L;
#pragma unroll
      for (int u = 0; u < kPre; ++u) {
        if (s0 + u < s1) {
          const int k = b + sn[u];
          const float d = s_C[k];
          D.dq[s0 + u] = make_float2(d, fmaxf(0.0f, 2.0f * s_A[k] - d * d));
        }
      }
      // the rest in rounds of kSinkRound: every node id of a round requested
      // before any is used (clamped, unpredicated loads and stores: a lane past
      // the net's last sink repeats that sink's write), one round trip a round
      for (int s = s0 + kPre; s < s1; s += kSinkRound) {
        int kk[kSinkRound];
#pragma unroll
        for (int u = 0; u < kSinkRound; ++u) kk[u] = D.sink_node[min(s + u, s1 - 1)];
#pragma unroll
        for (int u = 0; u < kSinkRound; ++u) {
          const int k = b + kk[u];
          const float d = s_C[k];
          D.dq[min(s + u, s1 - 1)] = make_float2(d, fmaxf(0.0f, 2.0f * s_A[k] - d * d));
        }
      }
    }
  }
}

// Reduced-order delays of the wide nets from the FP64 d (Y) and m2 (A) the
// wide kernel left in its scratch: one block per net, the four sums by a
// fixed block reduction, then the net's sinks.
__global__ __launch_bounds__(256) void k_rc_wide_reduced(DevDesign D, WideNets W, const uint32_t *only) {
  __shared__ double s_sum[4][256 / kWave];
  const int net = blockIdx.x;
  if (only && only[net] == 0u) return;
  const BigNet &B = W.big[net];
  const int x = B.x, m = B.m, st = m + 1;
  const int k0 = D.rc_ptr[x];
  const double *M2 = W.scratch + B.scr, *Y = M2 + 3 * st;
  const float *Cw = D.rc_cap + k0, *pc = W.pc + B.aux;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 1 + (int)threadIdx.x; k < m; k += 256) {
    const double c = (double)Cw[k] + (double)pc[k], d = Y[k], m2 = M2[k];
    v[0] += c * d;
    v[1] += c * d * d;
    v[2] += c * d * m2;
    v[3] += c * m2 * m2;
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    for (int off = kWave / 2; off > 0; off >>= 1) v[i] += __shfl_down(v[i], off);
    if (lane == 0) s_sum[i][wave] = v[i];
  }
  __syncthreads();
  double S[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    S[i] = 0.0;
    for (int w = 0; w < 256 / kWave; ++w) S[i] += s_sum[i][w];
  }
  const Red2 r = red2_model(S[0], S[1], S[2], S[3]);
  const int s0 = D.sink_ptr[x], ns = D.sink_ptr[x + 1] - s0;
  for (int j = threadIdx.x; j < ns; j += 256) {
    const int k = D.sink_node[s0 + j];
    D.dq[s0 + j].x = (float)red2_half_time(r, Y[k], M2[k]);
  }
}

// ------------------------------------------------------------ reduction

// Endpoint slack (early, late) from the endpoint's arrival and its given
// required time, written for the reports as well.  An endpoint's RAT is its
// constraint alone (a PO sink, or a cell output with no fanout), so this needs
// only the forward sweep and the reduction can run beside the backward sweep.
__device__ __forceinline__ float2 ep_slack_of(const DevDesign &D, int e) {
  const int loc = D.ep_loc[e];
  const float4 at = loc >= 0 ? D.drv_state[loc].at : D.sink_state[-1 - loc].at;
  const float2 s = ep_slack2(at, D.ep_rat[e]);
  D.ep_slack[e] = s;
  return s;
}

// WNS = min(0, min slack), TNS = sum of negative slacks, per early/late, in
// FP64 with a fixed partition and tree so results are bitwise reproducible;
// also writes the radix-sort keys of the endpoint order.
__global__ __launch_bounds__(256) void k_reduce(DevDesign D, double *partials, double *out,
                                               uint64_t *keys, int32_t *vals) {
  __shared__ double sh[4][256];
  const int n = D.n_ep;
  const int per = (n + kReduceBlocks - 1) / kReduceBlocks;
  const int b0 = blockIdx.x * per, b1 = min(n, b0 + per);
  double w0 = 0.0, w1 = 0.0, t0 = 0.0, t1 = 0.0;
  for (int e = b0 + (int)threadIdx.x; e < b1; e += 256) {
    const float2 s = ep_slack_of(D, e);
    w0 = fmin(w0, (double)s.x);
    w1 = fmin(w1, (double)s.y);
    if (s.x < 0.0f) t0 += (double)s.x;
    if (s.y < 0.0f) t1 += (double)s.y;
    if (keys) {  // one sort for both orders: early/late in bit 32
      keys[e] = f2ukey(s.x);
      keys[n + e] = (1ull << 32) | f2ukey(s.y);
      vals[e] = e;
      vals[n + e] = e;
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

// ------------------------------------------------------ batched reduction

// Per-design WNS/TNS of a batch.  Block (b, d) reduces slice b of design d's
// endpoints [ep_off[d], ep_off[d+1]) with the partition, per-thread order and
// tree of k_reduce, and k_reduce_batch_final folds the slices in the same
// order, so each design's figures are bit-identical to timing it alone.
// Sort keys carry the design in their high 32 bits (design-major order);
// values are design-local endpoint indices.
__global__ __launch_bounds__(256) void k_reduce_batch(DevDesign D, const int32_t *ep_off, double *partials,
                                                     uint64_t *keys, int32_t *vals, int dbits) {
  __shared__ double sh[4][256];
  const int dsg = blockIdx.y;
  const int e0 = ep_off[dsg];
  const int n = ep_off[dsg + 1] - e0;
  const int per = (n + kReduceBlocks - 1) / kReduceBlocks;
  const int b0 = blockIdx.x * per, b1 = min(n, b0 + per);
  double w0 = 0.0, w1 = 0.0, t0 = 0.0, t1 = 0.0;
  for (int e = b0 + (int)threadIdx.x; e < b1; e += 256) {
    const float2 s = ep_slack_of(D, e0 + e);
    w0 = fmin(w0, (double)s.x);
    w1 = fmin(w1, (double)s.y);
    if (s.x < 0.0f) t0 += (double)s.x;
    if (s.y < 0.0f) t1 += (double)s.y;
    if (keys) {  // (early/late, design, slack): one sort for both orders of every design
      keys[e0 + e] = ((uint64_t)dsg << 32) | f2ukey(s.x);
      keys[D.n_ep + e0 + e] = (1ull << (32 + dbits)) | ((uint64_t)dsg << 32) | f2ukey(s.y);
      vals[e0 + e] = e;
      vals[D.n_ep + e0 + e] = e;
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
  if (tid == 0)
    for (int k = 0; k < 4; ++k) partials[((size_t)dsg * kReduceBlocks + blockIdx.x) * 4 + k] = sh[k][0];
}

__global__ void k_reduce_batch_final(const double *partials, double *out, int n_designs) {
  const int dsg = blockIdx.x * blockDim.x + threadIdx.x;
  if (dsg >= n_designs) return;
  const double *p = partials + (size_t)dsg * kReduceBlocks * 4;
  double W0 = 0.0, W1 = 0.0, T0 = 0.0, T1 = 0.0;
  for (int b = 0; b < kReduceBlocks; ++b) {
    W0 = fmin(W0, p[b * 4 + 0]);
    W1 = fmin(W1, p[b * 4 + 1]);
    T0 += p[b * 4 + 2];
    T1 += p[b * 4 + 3];
  }
  out[dsg * 4 + 0] = W0; out[dsg * 4 + 1] = W1; out[dsg * 4 + 2] = T0; out[dsg * 4 + 3] = T1;
}

// ------------------------------------------------------ smooth reduction

// Smooth mode: per endpoint the early slack stays hard (min over rise/fall of
// AT - RAT) and the late slack is the smooth minimum s = -LSE_g(AT - RAT over
// rise/fall).  Reduces, in FP64 with a fixed partition and tree:
//   out[0] = early WNS, out[1] = WNS_g = -g log(1 + sum e^{-s/g}),
//   out[2] = early TNS, out[3] = TNS_g = sum -g log(1 + e^{-s/g}),
//   out[4], out[5] = max shift M and denominator e^{-M} + sum e^{-s/g - M}.
// The max-shifted sum is combined as (M, S) pairs so it never overflows.
__global__ __launch_bounds__(256) void k_reduce_smooth(DevDesign D, double *partials, double *out,
                                                      uint64_t *keys, int32_t *vals) {
  __shared__ double sh[5][256];
  const int n = D.n_ep;
  const double g = D.gamma;
  const int per = (n + kReduceBlocks - 1) / kReduceBlocks;
  const int b0 = blockIdx.x * per, b1 = min(n, b0 + per);
  double w0 = 0.0, t0 = 0.0, tg = 0.0, M = 0.0, S = 0.0;
  for (int e = b0 + (int)threadIdx.x; e < b1; e += 256) {
    const int loc = D.ep_loc[e];
    const float4 at = loc >= 0 ? D.drv_state[loc].at : D.sink_state[-1 - loc].at;
    const float4 R = D.ep_rat[e];
    const float se = fminf(at.x - R.x, at.y - R.y);
    const float aR = at.z - R.z, aF = at.w - R.w;
    const float mx = fmaxf(aR, aF);
    const float sl = -(mx + D.gamma * logf(expf((aR - mx) / D.gamma) + expf((aF - mx) / D.gamma)));
    D.ep_slack[e] = make_float2(se, sl);
    w0 = fmin(w0, (double)se);
    if (se < 0.0f) t0 += (double)se;
    const double z = -(double)sl / g;
    tg += -g * (z > 0.0 ? z + log1p(exp(-z)) : log1p(exp(z)));
    if (z > M) {
      S = S * exp(M - z) + 1.0;
      M = z;
    } else {
      S += exp(z - M);
    }
    if (keys) {
      keys[e] = f2ukey(se);
      keys[n + e] = (1ull << 32) | f2ukey(sl);
      vals[e] = e;
      vals[n + e] = e;
    }
  }
  const int tid = threadIdx.x;
  sh[0][tid] = w0; sh[1][tid] = t0; sh[2][tid] = tg; sh[3][tid] = M; sh[4][tid] = S;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      sh[0][tid] = fmin(sh[0][tid], sh[0][tid + o]);
      sh[1][tid] += sh[1][tid + o];
      sh[2][tid] += sh[2][tid + o];
      const double Ma = sh[3][tid], Mb = sh[3][tid + o], Mm = fmax(Ma, Mb);
      sh[4][tid] = sh[4][tid] * exp(Ma - Mm) + sh[4][tid + o] * exp(Mb - Mm);
      sh[3][tid] = Mm;
    }
    __syncthreads();
  }
  if (tid == 0) {
    for (int k = 0; k < 5; ++k) partials[blockIdx.x * 5 + k] = sh[k][0];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint32_t prev =
        __hip_atomic_fetch_add(D.counters + kCtrReduce, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == (uint32_t)(kReduceBlocks - 1)) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      double W0 = 0.0, T0 = 0.0, TG = 0.0, MM = 0.0, SS = 0.0;
      for (int b = 0; b < kReduceBlocks; ++b) {
        W0 = fmin(W0, partials[b * 5 + 0]);
        T0 += partials[b * 5 + 1];
        TG += partials[b * 5 + 2];
        const double Mb = partials[b * 5 + 3], Mm = fmax(MM, Mb);
        SS = SS * exp(MM - Mm) + partials[b * 5 + 4] * exp(Mb - Mm);
        MM = Mm;
      }
      const double den = exp(-MM) + SS;
      out[0] = W0;
      out[1] = -g * (MM + log(den));
      out[2] = T0;
      out[3] = TG;
      out[4] = MM;
      out[5] = den;
      D.counters[kCtrReduce] = 0u;
    }
  }
}

// ------------------------------------------------------------- adjoint

// d J / d(late AT rise, fall) at an endpoint with smooth late slack s, for
// J = g_tns TNS_g + g_wns WNS_g:  dJ/ds = g_tns / (1 + e^{s/g}) + g_wns e^{-s/g - M} / den,
// ds/dAT_rf = -softmax_rf(AT - RAT).
__device__ __forceinline__ float2 endpoint_seed(const DevDesign &D, float g_tns, float g_wns, int e, float4 at) {
  const float g = D.gamma;
  const float4 R = D.ep_rat[e];
  const float s = D.ep_slack[e].y;
  const float gs = g_tns / (1.0f + expf(s / g)) +
                   g_wns * (float)(exp(-(double)s / g - D.norm[0]) / D.norm[1]);
  return make_float2(-gs * expf((at.z - R.z + s) / g), -gs * expf((at.w - R.w + s) / g));
}

// Reverse mode through one cell output's late merges: softmax weights of the
// log-sum-exp arrival merge, the slew merge's subgradient to its winner, and
// the NLDM partials.  Every input sink has this cell as its only consumer, so
// its gradient is written here, once; nothing is accumulated atomically.
// (Libraries of more than four inputs: the inputs from the fanin lists.)
__device__ void cell_adjoint(const DevDesign &D, const LdsLib &lib, int x, int t, float L, int f0,
                             const PinState &me, float gA0, float gA1, float gS0, float gS1) {
  const int sense = lib.sense[t];
  const TabLayout lay{D.nx, D.ny};
  const float *tb = lib_type(lib, D, t);
  const AxisPos py = axis_find(tb + lay.ya(), tb + lay.rdy(), D.ny, L);
  const float rdy = tb[lay.rdy() + py.i];
  const float g = D.gamma;
  const float ato[2] = {me.at.z, me.at.w};
  const float gA[2] = {gA0, gA1}, gS[2] = {gS0, gS1};
  const int f1 = D.fanin_ptr[x + 1];
  // slew winners (same scan order and tie rule as the forward merge)
  float best[2] = {-kInf, -kInf};
  int win[2] = {-1, -1};
  for (int f = f0; f < f1; ++f) {
    const PinState st = D.sink_state[D.fanin_sink[f]];
    const float is[2] = {st.slew.z, st.slew.w};
#pragma unroll
    for (int ri = 0; ri < 2; ++ri) {
      const AxisPos px = axis_find(tb + lay.xa(), tb + lay.rdx(), D.nx, is[ri]);
#pragma unroll
      for (int ro = 0; ro < 2; ++ro) {
        if (!arc_maps(sense, ri, ro)) continue;
        const float cs = bilerp(tb + lay.tab(2 + ro), D.ny, px, py);
        if (cs > best[ro]) {
          best[ro] = cs;
          win[ro] = (f - f0) * 2 + ri;
        }
      }
    }
  }
  float gL = 0.0f;
  for (int f = f0; f < f1; ++f) {
    const int sidx = D.fanin_sink[f];
    const PinState st = D.sink_state[sidx];
    const float ia[2] = {st.at.z, st.at.w};
    const float is[2] = {st.slew.z, st.slew.w};
    float giA[2] = {0.0f, 0.0f}, giS[2] = {0.0f, 0.0f}, ga[2] = {0.0f, 0.0f};
#pragma unroll
    for (int ri = 0; ri < 2; ++ri) {
      const AxisPos px = axis_find(tb + lay.xa(), tb + lay.rdx(), D.nx, is[ri]);
      const float rdx = tb[lay.rdx() + px.i];
#pragma unroll
      for (int ro = 0; ro < 2; ++ro) {
        if (!arc_maps(sense, ri, ro)) continue;
        float dX, dY;
        const float dl = bilerp_d(tb + lay.tab(ro), D.ny, px, py, rdx, rdy, dX, dY);
        const float w = expf((ia[ri] + dl - ato[ro]) / g);
        const float wa = w * gA[ro];
        giA[ri] += wa;
        giS[ri] += wa * dX;
        gL += wa * dY;
        ga[ro] += wa;
        if (win[ro] == (f - f0) * 2 + ri) {
          float sX, sY;
          (void)bilerp_d(tb + lay.tab(2 + ro), D.ny, px, py, rdx, rdy, sX, sY);
          giS[ri] += gS[ro] * sX;
          gL += gS[ro] * sY;
        }
      }
    }
    D.g_sink[sidx] = make_float4(giA[0], giA[1], giS[0], giS[1]);
    D.g_arc[f] = make_float2(ga[0], ga[1]);
  }
  D.g_load[x] = gL;
}

// The same step with four lanes per cell output, lane k holding input slot k
// (inline fanin ids): the slew winner is the first maximum over the slots in
// (slot, transition) order, found by a reduction over the four lanes; each
// lane writes its input's sink and arc gradients, and lane 0 the load
// gradient, the lanes' sums added in slot order.  The four lanes of a cell are
// active together.
__device__ void cell_adjoint_lane(const DevDesign &D, const LdsLib &lib, int x, int t, float L, int f0, int k,
                                  int fk, const PinState &in, float2 ato2, float4 gg) {
  const int sense = lib.sense[t];
  const TabLayout lay{D.nx, D.ny};
  const float *tb = lib_type(lib, D, t);
  const AxisPos py = axis_find(tb + lay.ya(), tb + lay.rdy(), D.ny, L);
  const float rdy = tb[lay.rdy() + py.i];
  const float g = D.gamma;
  const float ato[2] = {ato2.x, ato2.y};
  const float gA[2] = {gg.x, gg.y}, gS[2] = {gg.z, gg.w};
  const bool has = fk >= 0;
  const float ia[2] = {in.at.z, in.at.w};
  const float is[2] = {in.slew.z, in.slew.w};
  AxisPos px[2];
#pragma unroll
  for (int ri = 0; ri < 2; ++ri) px[ri] = axis_find(tb + lay.xa(), tb + lay.rdx(), D.nx, is[ri]);
  // slew winners: this slot's first maximum, then the lanes' in slot order
  float best[2] = {-kInf, -kInf};
  int win[2] = {-1, -1};
#pragma unroll
  for (int ri = 0; ri < 2; ++ri) {
#pragma unroll
    for (int ro = 0; ro < 2; ++ro) {
      if (!has || !arc_maps(sense, ri, ro)) continue;
      const float cs = bilerp(tb + lay.tab(2 + ro), D.ny, px[ri], py);
      if (cs > best[ro]) {
        best[ro] = cs;
        win[ro] = k * 2 + ri;
      }
    }
  }
#pragma unroll
  for (int ro = 0; ro < 2; ++ro) {
#pragma unroll
    for (int o = 1; o < 4; o <<= 1) {
      const float ob = __shfl_xor(best[ro], o, 4);
      const int ow = __shfl_xor(win[ro], o, 4);
      const bool take = ob > best[ro] || (ob == best[ro] && ow >= 0 && (win[ro] < 0 || ow < win[ro]));
      best[ro] = take ? ob : best[ro];
      win[ro] = take ? ow : win[ro];
    }
  }
  float gL = 0.0f;
  if (has) {
    float giA[2] = {0.0f, 0.0f}, giS[2] = {0.0f, 0.0f}, ga[2] = {0.0f, 0.0f};
#pragma unroll
    for (int ri = 0; ri < 2; ++ri) {
      const float rdx = tb[lay.rdx() + px[ri].i];
#pragma unroll
      for (int ro = 0; ro < 2; ++ro) {
        if (!arc_maps(sense, ri, ro)) continue;
        float dX, dY;
        const float dl = bilerp_d(tb + lay.tab(ro), D.ny, px[ri], py, rdx, rdy, dX, dY);
        const float w = expf((ia[ri] + dl - ato[ro]) / g);
        const float wa = w * gA[ro];
        giA[ri] += wa;
        giS[ri] += wa * dX;
        gL += wa * dY;
        ga[ro] += wa;
        if (win[ro] == k * 2 + ri) {
          float sX, sY;
          (void)bilerp_d(tb + lay.tab(2 + ro), D.ny, px[ri], py, rdx, rdy, sX, sY);
          giS[ri] += gS[ro] * sX;
          gL += gS[ro] * sY;
        }
      }
    }
    D.g_sink[fk] = make_float4(giA[0], giA[1], giS[0], giS[1]);
    D.g_arc[f0 + k] = make_float2(ga[0], ga[1]);
  }
  const float l1 = __shfl(gL, 1, 4), l2 = __shfl(gL, 2, 4), l3 = __shfl(gL, 3, 4);
  if (k == 0) D.g_load[x] = ((gL + l1) + l2) + l3;
}

// Per-level reverse sweep: one block per chunk.  The chunk's sinks (all of
// them, also those a high-fanout driver leaves to pieces in the forward
// sweep) are taken 256 at a time, one per thread, with coalesced loads: each
// thread forms its sink's contribution to its driver's gradient and writes
// dJ/dd, dJ/dq; then the thread of each driver adds its sinks' contributions
// in sink order after its own endpoint seed (a fixed order, so the gradients
// are reproducible) and pushes through its cell.  As in the forward level
// kernel, only the chunk's span of cell types is staged (lib_f4 granules
// reserved).  With kSlots > 0 (inline fanin ids) the cell step runs on four
// lanes per driver, thread 4 d + k holding input slot k of driver d, whose id,
// input state and driver values it requests at entry, so their latency hides
// behind the sink rounds; the drivers' summed gradients reach the four lanes
// through LDS.
template <int kSlots>
__global__ __launch_bounds__(kSweepBlock) void k_adjoint(DevDesign D, float g_tns, float g_wns, int c0, int c1,
                                                         int lib_f4) {
  extern __shared__ __align__(32) unsigned char smem[];
  const int c = c0 + blockIdx.x;
  const int tid = threadIdx.x;
  const int4 cr = D.chunk_rec[c];
  const int x0 = __builtin_amdgcn_readfirstlane(cr.x), x1 = __builtin_amdgcn_readfirstlane(cr.y);
  const int x = x0 + tid;
  const bool drv = tid < kChunk && x < x1;
  const int xc = drv ? x : x0;
  // the cell step's loads first (they head the longest chain), every load
  // unconditional: with kSlots > 0 those of driver tid / 4's slot tid % 4
  const int d4 = tid >> 2, k4 = tid & 3;
  const bool live4 = x0 + d4 < x1;
  const int xs = kSlots > 0 ? (live4 ? x0 + d4 : x0) : xc;
  const int4 f4 = kSlots > 0 ? D.fanin4[xs] : make_int4(-1, -1, -1, -1);
  const int t = max(D.cell_type[xs], 0);
  const float L = D.L_net[xs];
  const int f0 = D.fanin_ptr[xs];
  const int2 tr = D.chunk_trange[c];
  const LibSpan span = lib_span(D, tr.x, tr.y);
  const float4 lib_r = lib_issue_span(D, span);
  const int fk = k4 == 0 ? f4.x : k4 == 1 ? f4.y : k4 == 2 ? f4.z : f4.w;
  const PinState ink = D.sink_state[max(fk, 0)];
  const float2 ato4 = kSlots > 0 ? reinterpret_cast<const float2 *>(&D.drv_state[xs].at)[1] : make_float2(0.f, 0.f);
  const int sb = __builtin_amdgcn_readfirstlane(cr.z);
  const int se = __builtin_amdgcn_readfirstlane(D.sink_ptr[x1]);
  const int sAc = min(sb + tid, max(se - 1, 0));
  const PinState ssA = D.sink_state[sAc];
  const int consA = D.sink_cons[sAc], drvA = D.sink_drv[sAc];
  const float4 gA4 = D.g_sink[sAc];
  const PinState me = D.drv_state[xc];
  const int e = D.drv_ep[xc];
  const int sp0 = D.sink_ptr[xc], sp1 = D.sink_ptr[xc + 1];
  const LdsLib lib = lib_store_span(D, smem, span, lib_r, lib_f4);
  float2 *dsl = reinterpret_cast<float2 *>(smem + span_lds_bytes(lib_f4, D.n_types));  // [kChunk]
  float4 *cb = reinterpret_cast<float4 *>(dsl + kChunk);                                // [kSweepBlock]
  if (tid < kChunk) dsl[tid] = make_float2(me.slew.z, me.slew.w);
  lds_barrier();
  float gA0 = 0.0f, gA1 = 0.0f, gS0 = 0.0f, gS1 = 0.0f;
  if (drv && e >= 0) {
    const float2 sd = endpoint_seed(D, g_tns, g_wns, e, me.at);
    gA0 = sd.x;
    gA1 = sd.y;
  }
  for (int r0 = sb; r0 < se; r0 += kSweepBlock) {
    const int s = r0 + tid;
    if (s < se) {
      const bool first = r0 == sb;
      const PinState ss = first ? ssA : D.sink_state[s];
      const int cons = first ? consA : D.sink_cons[s];
      const int dr = first ? drvA : D.sink_drv[s];
      float4 gs;
      if (cons < 0) {
        const float2 sd = endpoint_seed(D, g_tns, g_wns, -1 - cons, ss.at);
        gs = make_float4(sd.x, sd.y, 0.0f, 0.0f);
      } else {
        gs = first ? gA4 : D.g_sink[s];
      }
      const float2 ms = dsl[dr - x0];
      cb[tid] = make_float4(gs.x, gs.y, gs.z * (ms.x / ss.slew.z), gs.w * (ms.y / ss.slew.w));
      D.g_dq[s] = make_float2(gs.x + gs.y, gs.z / (2.0f * ss.slew.z) + gs.w / (2.0f * ss.slew.w));
    }
    lds_barrier();
    if (drv) {
      const int a = max(sp0, r0), b = min(sp1, r0 + kSweepBlock);
      for (int k = a; k < b; ++k) {
        const float4 v = cb[k - r0];
        gA0 += v.x;
        gA1 += v.y;
        gS0 += v.z;
        gS1 += v.w;
      }
    }
    lds_barrier();
  }
  if constexpr (kSlots > 0) {
    if (drv) cb[tid] = make_float4(gA0, gA1, gS0, gS1);  // (cb is free after the last round's barrier)
    lds_barrier();
    if (live4) {  // (uniform over a driver's four lanes)
      const int xd = x0 + d4;
      if (xd >= D.n_pi)
        cell_adjoint_lane(D, lib, xd, t, L, f0, k4, fk, ink, ato4, cb[d4]);
      else if (k4 == 0)
        D.g_load[xd] = 0.0f;
    }
  } else {
    if (drv) {
      if (x >= D.n_pi)
        cell_adjoint(D, lib, x, t, L, f0, me, gA0, gA1, gS0, gS1);
      else
        D.g_load[x] = 0.0f;
    }
  }
}

// ------------------------------------------------------------ RC adjoint
//
// dJ/dC_k for every node k of a net, from dJ/dL (the driver's NLDM load), and
// per sink v dJ/dd_v and dJ/dq_v with q = 2 m2 - d^2.  With R_kj the resistance
// shared by the root->k and root->j paths, dd_v/dC_k = R_vk and
// dm2_v/dC_k = R_vk d_k + sum_j C^_j R_vj R_jk, so with the sink-node seeds
// gd_v = dJ/dd_v - 2 d_v dJ/dq_v and gm_v = 2 dJ/dq_v:
//   dJ/dC_k = dJ/dL + PA_k + d_k H_k + PB_k,
//   PA_k = path sum of R Gd, H_k = path sum of R Gm, PB_k = path sum of R K,
//   Gd, Gm = subtree sums of gd, gm, K = subtree sum of C^ H.
// A segment's resistance enters d_v as R_k S1_k (S1 = downstream cap) and m2_v
// as R_k S2_k (S2 = subtree sum of C^ d) plus through the d_j inside the S2 of
// the segments above it, so
//   dJ/dR_k = S1_k (Gd_k + K_k) + S2_k Gm_k   (0 at the root).
// (dJ/dq is dropped where the clamp q = max(0, .) is active.)

__device__ void rc_adjoint_wide(const DevDesign &D, const BigNet &B, const WideNets &W, WideCtx &c, double *s_w) {
  const int x = B.x, m = B.m;
  const int k0 = D.rc_ptr[x];
  const float *R = D.rc_res + k0;
  const float *Cw = D.rc_cap + k0;
  const int32_t *end = W.end + B.aux;
  const float *pc = W.pc + B.aux;
  const int32_t *nsp = W.nsp + B.nsp;
  const int32_t *nsl = W.nsl;
  const int32_t *egp = W.egp + B.egp, *egl = W.egl + B.aux;
  const float2 *gdq = D.g_dq + D.sink_ptr[x];
  const int st = m + 1;
  double *A = W.scratch + B.scr, *P = A + st, *X = P + st, *Y = X + st, *Z = Y + st;
  double *G1 = Z + st, *G2 = G1 + st, *T = G2 + st, *V = T + st, *S1 = V + st, *DR = S1 + st;
  // forward moments: Y = d, Z = m2; S1 = downstream cap, DR = S2 for now
  seg_map(c.k0, c.k1, [=](int k) { return (double)Cw[k] + (double)pc[k]; }, [=](int k, double v) { stc(A + k, v); });
  wide_scan(c, A, P, true, s_w);
  seg_map(c.k0, c.k1, [=](int k) { return ldc(P + end[k]) - ldc(P + k); }, [=](int k, double v) { stc(S1 + k, v); });
  wide_edge(c, R, P, end, X);
  wide_path_sum(c, X, egp, egl, V, Y, s_w);
  seg_map(c.k0, c.k1, [=](int k) { return ldc(A + k) * ldc(Y + k); }, [=](int k, double v) { stc(X + k, v); });
  wide_scan(c, X, P, true, s_w);
  seg_map(c.k0, c.k1, [=](int k) { return ldc(P + end[k]) - ldc(P + k); }, [=](int k, double v) { stc(DR + k, v); });
  wide_edge(c, R, P, end, X);
  wide_path_sum(c, X, egp, egl, V, Z, s_w);
  // sink-node seeds, sinks of a node in sink order
  for (int k = c.k0 + threadIdx.x; k < c.k1; k += blockDim.x) {
    double gd = 0.0, gm = 0.0;
    const double yk = ldc(Y + k), zk = ldc(Z + k);
    for (int i = nsp[k]; i < nsp[k + 1]; ++i) {
      const float2 g = gdq[nsl[i]];
      const double gq = (2.0 * zk - yk * yk) > 0.0 ? (double)g.y : 0.0;
      gd += (double)g.x - 2.0 * yk * gq;
      gm += 2.0 * gq;
    }
    stc(G1 + k, gd);
    stc(G2 + k, gm);
  }
  __syncthreads();
  wide_scan(c, G1, P, true, s_w);                           // Gd = subtree sums
  seg_map(c.k0, c.k1, [=](int k) { return ldc(P + end[k]) - ldc(P + k); }, [=](int k, double v) { stc(G1 + k, v); });
  wide_scan(c, G2, P, true, s_w);                           // Gm
  // DR = S2 Gm + S1 Gd (K follows below); each k stays with its thread
  seg_map(c.k0, c.k1,
          [=](int k) { return ldc(DR + k) * (ldc(P + end[k]) - ldc(P + k)) + ldc(S1 + k) * ldc(G1 + k); },
          [=](int k, double v) { stc(DR + k, v); });
  wide_edge(c, R, P, end, X);
  wide_path_sum(c, X, egp, egl, V, T, s_w);                 // H = path sum of R Gm
  seg_map(c.k0, c.k1, [=](int k) { return k ? (double)R[k] * ldc(G1 + k) : 0.0; },
          [=](int k, double v) { stc(X + k, v); });
  wide_sync(c);
  wide_path_sum(c, X, egp, egl, V, G1, s_w);                // PA = path sum of R Gd
  seg_map(c.k0, c.k1, [=](int k) { return ldc(A + k) * ldc(T + k); }, [=](int k, double v) { stc(X + k, v); });
  wide_scan(c, X, P, true, s_w);                            // K = subtree sum of C^ H
  float *gres = D.g_res + k0;
  seg_map(c.k0, c.k1, [=](int k) { return k ? (float)(ldc(DR + k) + ldc(S1 + k) * (ldc(P + end[k]) - ldc(P + k))) : 0.0f; },
          [=](int k, float v) { gres[k] = v; });
  wide_edge(c, R, P, end, X);
  wide_path_sum(c, X, egp, egl, V, G2, s_w);                // PB = path sum of R K
  const double gL = (double)D.g_load[x];
  float *gcap = D.g_cap + k0;
  seg_map(c.k0, c.k1, [=](int k) { return (float)(gL + ldc(G1 + k) + ldc(Y + k) * ldc(T + k) + ldc(G2 + k)); },
          [=](int k, float v) { gcap[k] = v; });
  wide_leave(c);
}

// Same block layout as k_rc.  Small nets: one lane per net in LDS, the forward
// recursions recomputed, then the two subtree/path rounds.  Block 0 clears the
// sweep counters (the next update and the next adjoint start from zero).
__global__ __launch_bounds__(kWideBlock) void k_rc_adjoint_wide(DevDesign D, WideNets W) {
  __shared__ double s_w[kWideBlock / kWave + 1];
  const int2 nb = W.blk[blockIdx.x];
  const BigNet &B = W.big[nb.x];
  WideCtx c = wide_ctx(B, W, nb.y, nb.x);
  rc_adjoint_wide(D, B, W, c, s_w);
}

// kRes: also dJ/dR per segment (one more LDS array; only when it is asked for).
// Its own chunks, of at most kRcAdjBlock nets and kRcAdjChunkNodes nodes (the
// same net order as the forward's): eight arrays at 2048 nodes held it to two
// blocks per compute unit.
template <bool kRes>
__global__ __launch_bounds__(kRcAdjBlock) void k_rc_adjoint(DevDesign D, const int2 *chunks, int n_chunks) {
  __shared__ uint8_t s_par[kRcAdjChunkNodes];
  __shared__ float s_R[kRcAdjChunkNodes], s_C[kRcAdjChunkNodes], s_A[kRcAdjChunkNodes], s_B[kRcAdjChunkNodes];
  __shared__ float s_E[kRcAdjChunkNodes], s_F[kRcAdjChunkNodes], s_G[kRes ? kRcAdjChunkNodes : 1];
  __shared__ int s_base[kRcAdjBlock + 1];
  const int tid = threadIdx.x;
  const int ci = xcd_major(n_chunks);
  if (ci >= n_chunks) return;
  const int2 ch = chunks[ci];
  const int j0 = ch.x, j1 = ch.y;
  const int k0 = D.rc_start[j0], nk = D.rc_start[j1] - k0;
  const int j = j0 + tid;
  const int jc = j < j1 ? j : j0;
  const int x = D.rc_order[jc];
  const int2 sr = D.rc_sinks[jc];
  stage_rc_nodes<kRcAdjChunkNodes, kRcAdjBlock>(D, k0, nk, s_par, s_R, s_C, s_A);
  for (int i = tid; i <= j1 - j0; i += kRcAdjBlock) s_base[i] = D.rc_start[j0 + i] - k0;
  __syncthreads();
  if (j < j1) {
    const int b = s_base[tid], m = s_base[tid + 1] - b;
    const uint8_t *par = s_par;
    float *A = s_A, *B = s_B, *C = s_C, *E = s_E, *F = s_F, *G = s_G, *R = s_R;
    (void)rc_tree_lds(par, R, C, A, B, b, m);  // A = m2, B = d
    for (int k = 0; k < m; ++k) E[b + k] = F[b + k] = 0.0f;
    for (int s = sr.x; s < sr.y; s += kSinkRound) {  // (rounds as in k_rc; sinks in order)
      int kk[kSinkRound];
      float2 gg[kSinkRound];
#pragma unroll
      for (int u = 0; u < kSinkRound; ++u) {
        kk[u] = D.sink_node[min(s + u, sr.y - 1)];
        gg[u] = D.g_dq[min(s + u, sr.y - 1)];
      }
#pragma unroll
      for (int u = 0; u < kSinkRound; ++u) {
        const int k = b + kk[u];
        const float gq = (2.0f * A[k] - B[k] * B[k]) > 0.0f ? gg[u].y : 0.0f;
        if (s + u < sr.y) {
          E[k] += gg[u].x - 2.0f * B[k] * gq;
          F[k] += 2.0f * gq;
        }
      }
    }
    for (int k = m - 1; k >= 1; --k) {  // Gd, Gm
      E[b + par[b + k]] += E[b + k];
      F[b + par[b + k]] += F[b + k];
    }
    A[b] = 0.0f;  // H
    for (int k = 1; k < m; ++k) A[b + k] = A[b + par[b + k]] + R[b + k] * F[b + k];
    if constexpr (kRes) {
      for (int k = 0; k < m; ++k) G[b + k] = C[b + k] * B[b + k];  // S2
      for (int k = m - 1; k >= 1; --k) G[b + par[b + k]] += G[b + k];
      for (int k = 0; k < m; ++k) G[b + k] *= F[b + k];  // S2 Gm
    }
    for (int k = 0; k < m; ++k) F[b + k] = C[b + k] * A[b + k];  // K
    for (int k = m - 1; k >= 1; --k) F[b + par[b + k]] += F[b + k];
    for (int k = 0; k < m; ++k) F[b + k] += E[b + k];  // Gd + K
    if constexpr (kRes) {
      for (int k = 0; k < m; ++k) E[b + k] = C[b + k];  // S1
      for (int k = m - 1; k >= 1; --k) E[b + par[b + k]] += E[b + k];
      G[b] = 0.0f;
      for (int k = 1; k < m; ++k) G[b + k] += E[b + k] * F[b + k];  // dJ/dR
    }
    F[b] = 0.0f;  // PA + PB = path sum of R (Gd + K), in place (parents first)
    for (int k = 1; k < m; ++k) F[b + k] = F[b + par[b + k]] + R[b + k] * F[b + k];
    const float gL = D.g_load[x];
    for (int k = 0; k < m; ++k) C[b + k] = gL + F[b + k] + B[b + k] * A[b + k];
  }
  __syncthreads();
  for (int i = tid; i < nk; i += kRcAdjBlock) {
    D.g_cap[k0 + i] = s_C[i];
    if constexpr (kRes) D.g_res[k0 + i] = s_G[i];
  }
}

// Gradients back to caller order: node caps by the node permutation, NLDM
// loads per cell-output pin (0 elsewhere), arc delays per caller arc (early
// views 0).
__global__ void k_scatter_grads(DevDesign D, const int32_t *node_src, int64_t n_nodes, float *grad_cap, float *grad_res,
                                const int32_t *pin_loc, int n_pins, float *grad_load, const int32_t *arc_src,
                                int n_arcs, float4 *grad_arc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (grad_cap && i < n_nodes) grad_cap[node_src[i]] = D.g_cap[i];
  if (grad_res && i < n_nodes) grad_res[node_src[i]] = D.g_res[i];
  if (grad_load && i < n_pins) {
    const int loc = pin_loc[i];
    grad_load[i] = (loc >= D.n_pi) ? D.g_load[loc] : 0.0f;
  }
  if (grad_arc && i < n_arcs) {
    const float2 g = D.g_arc[i];
    grad_arc[arc_src[i]] = make_float4(0.0f, 0.0f, g.x, g.y);
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
    if (rat) rat[p] = D.cons_rec[loc].rat;
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

// Wire caps into the layout; the small nets' nodes (the first n_small) also
// take their lumped receiving pin caps, the sum the RC pass reads.
__global__ void k_permute_caps(const float *src, const int32_t *node_src, float *dst, int64_t n, const float *pc,
                               int64_t n_small) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) {
    const float c = src[node_src[k]];
    dst[k] = k < n_small ? c + pc[k] : c;
  }
}

inline int blocks_for(int64_t n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

// ------------------------------------------------------------ path report
//
// A node is (slot code, transition): code = 2 * slot + rf, driver slots first
// (0..n_drv-1), then sink slots (n_drv + sink).  Backward from a node: a sink's
// only predecessor is its net's driver (deviation 0); a cell output's
// predecessors are the (input, input transition) candidates of its merge, the
// critical one (drv_crit) with deviation 0 and every other with deviation
// AT_out - (AT_in + delay) (late) or (AT_in + delay) - AT_out (early), the delay
// recomputed exactly as the forward merge computes it; a primary input has
// none.  A path = critical completion with a sequence of sidetracks: popping
// the heap item of smallest key yields one complete path (its critical
// completion, slack = key), and pushes one item per sidetrack available along
// that completion (key + deviation).  Every path comes out exactly once, in
// ascending slack.

__device__ __forceinline__ bool item_less(int4 a, int4 b) {
  const float ka = __int_as_float(a.x), kb = __int_as_float(b.x);
  return ka < kb || (ka == kb && a.y < b.y);
}

// An endpoint's pending items, ascending in (key, sequence), in column i * stride
// of q (LDS or global memory).  Only the best lim of them are kept, lim the pops
// still to come: an item pushed later carries at least the key just popped, so
// an item that ranks beyond the remaining pops can never be popped.  Items live
// in positions [h, h + n) with h + lim = m throughout.
struct PathQueue {
  int4 *q;
  int stride, h, n, lim;
  __device__ __forceinline__ int4 at(int i) const { return q[(size_t)i * stride]; }
  __device__ __forceinline__ void set(int i, int4 v) { q[(size_t)i * stride] = v; }
  __device__ void push(int4 it) {
    if (n == lim) {
      if (n == 0 || !item_less(it, at(h + n - 1))) return;
      --n;  // the last falls out
    }
    int p = h + n;
    while (p > h && item_less(it, at(p - 1))) {
      set(p, at(p - 1));
      --p;
    }
    set(p, it);
    ++n;
  }
  __device__ int4 pop() {  // n > 0
    const int4 top = at(h);
    ++h;
    --n;
    --lim;
    n = min(n, lim);
    return top;
  }
};

__device__ __forceinline__ float node_at(const DevDesign &D, int code, int el) {
  const int slot = code >> 1, v = el * 2 + (code & 1);
  const float4 a = slot < D.n_drv ? D.drv_state[slot].at : D.sink_state[slot - D.n_drv].at;
  return v == 0 ? a.x : v == 1 ? a.y : v == 2 ? a.z : a.w;
}

__device__ __forceinline__ float node_slew(const DevDesign &D, int code, int el) {
  const int slot = code >> 1, v = el * 2 + (code & 1);
  const float4 a = slot < D.n_drv ? D.drv_state[slot].slew : D.sink_state[slot - D.n_drv].slew;
  return v == 0 ? a.x : v == 1 ? a.y : v == 2 ? a.z : a.w;
}

// One thread per endpoint (blocks of one wavefront, so the endpoints spread
// over the compute units); its queue in LDS after the library when both fit
// (kLds, so that queue accesses are LDS instructions and never wait for the
// walk's global loads), else in A.items.
template <bool kLds>
__global__ __launch_bounds__(kWave) void k_paths_enum(DevDesign D, PathArgs A) {
  extern __shared__ __align__(32) unsigned char smem[];
  const LdsLib lib = load_lib(D, smem);
  __syncthreads();
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= A.n_eps) return;
  const int el = A.el, m = A.m, lmax = A.lmax;
  PathQueue Q;
  if constexpr (kLds) {
    Q.q = reinterpret_cast<int4 *>(smem + lib_lds_bytes(D.n_types, D.tstride)) + threadIdx.x;
    Q.stride = kWave;
  } else {
    Q.q = A.items + t;
    Q.stride = A.n_eps;
  }
  Q.h = 0;
  Q.n = 0;
  Q.lim = m;
  int32_t *nodes = A.nodes + (size_t)t * m * lmax;
  int32_t *plen = A.plen + (size_t)t * m;
  float *pkey = A.pkey + (size_t)t * m;
  for (int j = 0; j < m; ++j) plen[j] = 0;
  const int e = A.eps[t];
  const int loc = D.ep_loc[e];
  const int slot = loc >= 0 ? loc : D.n_drv + (-1 - loc);
  const float4 R = D.ep_rat[e];
  int seq = 0;
  for (int rf = 0; rf < 2; ++rf) {
    const int v = el * 2 + rf;
    const float rat = v == 0 ? R.x : v == 1 ? R.y : v == 2 ? R.z : R.w;
    if (!(fabsf(rat) < kInf)) continue;
    const int code = slot * 2 + rf;
    const float a = node_at(D, code, el);
    const float key = el ? rat - a : a - rat;
    Q.push(make_int4(__float_as_int(key), seq++, -1, code));
  }
  const TabLayout lay{D.nx, D.ny};
  for (int j = 0; j < m && Q.n > 0; ++j) {
    const int4 it = Q.pop();
    const float key = __int_as_float(it.x);
    if (!(key < A.thr)) break;
    int32_t *path = nodes + (size_t)j * lmax;
    int len = 0;
    if (it.z >= 0) {  // prefix of the parent path up to the sidetrack
      const int parent = it.z >> 24, pos = it.z & 0xffffff;
      const int32_t *pp = nodes + (size_t)parent * lmax;
      // sixteen loads in flight before their stores (the two paths never
      // overlap, which the compiler cannot see), then the tail
      constexpr int kCopy = 16;
      for (; len + kCopy <= pos; len += kCopy) {
        int32_t v[kCopy];
#pragma unroll
        for (int u = 0; u < kCopy; ++u) v[u] = pp[len + u];
#pragma unroll
        for (int u = 0; u < kCopy; ++u) path[len + u] = v[u];
      }
      for (; len < pos; ++len) path[len] = pp[len];
    }
    int code = it.w;
    for (;;) {
      path[len++] = code;
      const int sl = code >> 1, rf = code & 1;
      if (sl >= D.n_drv) {  // sink: its driver, same transition
        code = D.sink_drv[sl - D.n_drv] * 2 + rf;
        continue;
      }
      if (sl < D.n_pi) break;  // startpoint
      const int v = el * 2 + rf;
      if (D.fanin4) {
        // the cell's loads in one round trip (fanin ids inline), then the
        // critical input's driver and every input state in the next; the
        // sidetracks are pushed in the same (input, transition) order
        const uint32_t cw = D.drv_crit[sl];
        const float at_out = node_at(D, code, el);
        const int ty = D.cell_type[sl];
        const float Lc = D.L_net[sl];
        const int4 f4 = D.fanin4[sl];
        const int fin[4] = {f4.x, f4.y, f4.z, f4.w};
        const int crit = (int)((cw >> (8 * v)) & 0xffu);
        const int cs = fin[min(crit >> 1, 3)];
        const int nd = D.sink_drv[max(cs, 0)];  // (unused when the cell has no critical input)
        float4 iat[4], isl[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const PinState &ps = D.sink_state[max(fin[k], 0)];
          iat[k] = ps.at;
          isl[k] = ps.slew;
        }
        const CellCtx cc = cell_ctx(D, lib, ty, Lc);
        bool has_crit = false;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (fin[k] < 0) continue;
#pragma unroll
          for (int ri = 0; ri < 2; ++ri) {
            if (!arc_maps(cc.sense, ri, rf)) continue;
            if (k * 2 + ri == crit) {
              has_crit = true;
              continue;
            }
            const int w = el * 2 + ri;
            const float x = w == 0 ? isl[k].x : w == 1 ? isl[k].y : w == 2 ? isl[k].z : isl[k].w;
            const float ain = w == 0 ? iat[k].x : w == 1 ? iat[k].y : w == 2 ? iat[k].z : iat[k].w;
            const AxisPos px = axis_find(cc.tb + lay.xa(), cc.tb + lay.rdx(), D.nx, x);
            const float dl = bilerp(cc.tb + lay.tab(rf), D.ny, px, cc.py);
            const float cand = ain + dl;
            const float dev = fmaxf(el ? at_out - cand : cand - at_out, 0.0f);
            const float k2 = key + dev;
            if (k2 < A.thr)
              Q.push(make_int4(__float_as_int(k2), seq++, (j << 24) | len, (D.n_drv + fin[k]) * 2 + ri));
          }
        }
        if (!has_crit) break;  // (every cell output has a critical candidate)
        path[len++] = (D.n_drv + cs) * 2 + (crit & 1);  // the critical input sink, then its driver
        code = nd * 2 + (crit & 1);
        continue;
      }
      const int crit = (int)((D.drv_crit[sl] >> (8 * v)) & 0xffu);
      const float at_out = node_at(D, code, el);
      const CellCtx cc = cell_ctx(D, lib, D.cell_type[sl], D.L_net[sl]);
      const int f0 = D.fanin_ptr[sl], nf = D.fanin_ptr[sl + 1] - f0;
      int next = -1;
      for (int k = 0; k < nf; ++k) {
        const int in_slot = D.n_drv + D.fanin_sink[f0 + k];
        for (int ri = 0; ri < 2; ++ri) {
          if (!arc_maps(cc.sense, ri, rf)) continue;
          const int in_code = in_slot * 2 + ri;
          if (k * 2 + ri == crit) {
            next = in_code;
            continue;
          }
          const float x = node_slew(D, in_code, el);
          const AxisPos px = axis_find(cc.tb + lay.xa(), cc.tb + lay.rdx(), D.nx, x);
          const float dl = bilerp(cc.tb + lay.tab(rf), D.ny, px, cc.py);
          const float cand = node_at(D, in_code, el) + dl;
          const float dev = fmaxf(el ? at_out - cand : cand - at_out, 0.0f);
          const float k2 = key + dev;
          if (k2 < A.thr) Q.push(make_int4(__float_as_int(k2), seq++, (j << 24) | len, in_code));
        }
      }
      if (next < 0) break;  // (every cell output has a critical candidate)
      code = next;
    }
    plen[j] = len;
    pkey[j] = key;
  }
}

// Sort keys of every found path (unfilled slots sort last).
__global__ void k_paths_keys(PathArgs A, uint32_t *keys, int32_t *vals) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n_eps * A.m) return;
  keys[i] = A.plen[i] > 0 ? f2ukey(A.pkey[i]) : 0xffffffffu;
  vals[i] = i;
}

__global__ void k_paths_lengths(PathArgs A, const int32_t *sel, int n_sel, int32_t *len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_sel) len[i] = A.plen[sel[i]];
}

// One wavefront per reported path, a lane per pin: pins from startpoint to
// endpoint.
__global__ __launch_bounds__(256) void k_paths_emit(DevDesign D, PathArgs A, const int32_t *sel, int n_sel,
                                                    const int32_t *ptr, int32_t *pin, int8_t *rf, float *slack,
                                                    int32_t *ep) {
  const int i = blockIdx.x * (256 / kWave) + (int)threadIdx.x / kWave, lane = (int)threadIdx.x % kWave;
  if (i >= n_sel) return;
  const int c = sel[i];
  const int t = c / A.m;
  const int len = A.plen[c];
  const int32_t *path = A.nodes + (size_t)c * A.lmax;
  if (lane == 0) {
    if (slack) slack[i] = A.pkey[c];
    if (ep) ep[i] = A.eps[t];
  }
  const int o = ptr[i];
  for (int q = lane; q < len; q += kWave) {
    const int code = path[len - 1 - q];
    const int sl = code >> 1;
    if (pin) pin[o + q] = sl < D.n_drv ? A.drv_pin[sl] : A.sink_pin[sl - D.n_drv];
    if (rf) rf[o + q] = (int8_t)(code & 1);
  }
}

// ------------------------------------------------------------ wrappers

// The level kernels with a type-span image of lib_f4 granules.
static size_t span_sweep_lds_bytes(const DevDesign &D, int lib_f4, int chunks_per_block) {
  return span_lds_bytes(lib_f4, D.n_types) + sizeof(PinState) * kWave * (kSweepBlock / kWave) * chunks_per_block;
}

size_t sweep_lds_bytes(const DevDesign &D, int chunks_per_block) {
  const size_t per_wave = sizeof(PinState) * kWave;  // >= 4 ints per lane for the backward
  return lib_lds_bytes(D.n_types, D.tstride) + per_wave * (kSweepBlock / kWave) * chunks_per_block;
}

// Blocks per CU every sweep kernel of the given schedule can keep resident.
template <bool kCoop>
static int sweep_occupancy(size_t lds_bytes) {
  int n = 1 << 30;
  const void *ks[] = {reinterpret_cast<const void *>(&k_sweep<kSweepFwd, kCoop>),
                      reinterpret_cast<const void *>(&k_sweep<kSweepBwd, kCoop>)};
  for (const void *k : ks) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k, kSweepBlock, lds_bytes) != hipSuccess) return 0;
    n = b < n ? b : n;
  }
  return n;
}

int coop_blocks_per_cu(size_t lds_bytes) { return sweep_occupancy<true>(lds_bytes); }

int sweep_blocks_per_cu(size_t lds_bytes) {
  const int n = sweep_occupancy<false>(lds_bytes);
  return n < 1 ? 1 : n;
}

template <int kKind>
static hipError_t launch_sweep(const DevDesign &D, float g_tns, float g_wns, int grid, bool coop, hipStream_t s) {
  if (coop) {
    DevDesign a = D;
    float gt = g_tns, gw = g_wns;
    void *args[] = {&a, &gt, &gw};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_sweep<kKind, true>), dim3(grid),
                                      dim3(kSweepBlock), args, (unsigned)sweep_lds_bytes(D), s);
  }
  hipLaunchKernelGGL((k_sweep<kKind, false>), dim3(grid), dim3(kSweepBlock), sweep_lds_bytes(D), s, D, g_tns, g_wns);
  return hipGetLastError();
}

hipError_t launch_rc(const DevDesign &D, const int2 *chunks, int n_chunks, hipStream_t s, const uint32_t *only,
                     bool clear_counters) {
  const int n_ctr = clear_counters ? n_counters(D.n_ph_fwd + D.n_ph_bwd) : 0;
  const dim3 grid(xcd_grid(n_chunks > 0 ? n_chunks : 1));
  if (D.delay_model == 1)
    hipLaunchKernelGGL(k_rc<true>, grid, dim3(kRcBlock), 0, s, D, chunks, n_chunks, D.counters, n_ctr, only);
  else
    hipLaunchKernelGGL(k_rc<false>, grid, dim3(kRcBlock), 0, s, D, chunks, n_chunks, D.counters, n_ctr, only);
  return hipGetLastError();
}

hipError_t launch_rc_wide(const DevDesign &D, const WideNets &W, hipStream_t s, const uint32_t *only) {
  if (W.n_big <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rc_wide, dim3(W.n_blk), dim3(kWideBlock), 0, s, D, W, only);
  if (D.delay_model == 1) hipLaunchKernelGGL(k_rc_wide_reduced, dim3(W.n_big), dim3(256), 0, s, D, W, only);
  return hipGetLastError();
}

hipError_t launch_rc_adjoint_wide(const DevDesign &D, const WideNets &W, hipStream_t s) {
  if (W.n_big <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rc_adjoint_wide, dim3(W.n_blk), dim3(kWideBlock), 0, s, D, W);
  return hipGetLastError();
}

hipError_t launch_forward(const DevDesign &D, int grid, bool coop, hipStream_t s) {
  return launch_sweep<kSweepFwd>(D, 0.0f, 0.0f, grid, coop, s);
}

// Chunks per block of the full-update level kernels (the incremental
// continuation keeps one).
constexpr int kFullCpb = kLevelCpb;

template <bool kInc, int kSlots>
static void launch_fwd_chunks(const DevDesign &D, const IncArgs &I, int4 ph, int4 reg, hipStream_t s) {
  constexpr int cpb = kInc ? 1 : kFullCpb;
  hipLaunchKernelGGL((k_forward<kInc, kSlots, cpb>), dim3(blocks_for(ph.z, cpb)), dim3(kSweepBlock * cpb),
                     span_sweep_lds_bytes(D, reg.z, cpb), s, D, ph.y, reg.x, reg.y, ph.z, reg.z, I);
}

template <bool kInc>
static hipError_t forward_phase(const DevDesign &D, const IncArgs &I, int4 ph, int4 reg, hipStream_t s) {
  if (ph.z <= 0) return hipSuccess;
  const int per = kSweepBlock / kWave;
  if (ph.x == kItemPiece)
    hipLaunchKernelGGL(k_forward_pieces<kInc>, dim3(blocks_for(ph.z, per)), dim3(kSweepBlock), 0, s, D, ph.y,
                       ph.y + ph.z, I);
  else if (!D.fanin4)  // a type of more than 4 inputs: fanins through the CSR
    launch_fwd_chunks<kInc, 0>(D, I, ph, reg, s);
  else if (D.max_in <= 1)
    launch_fwd_chunks<kInc, 1>(D, I, ph, reg, s);
  else if (D.max_in == 2)
    launch_fwd_chunks<kInc, 2>(D, I, ph, reg, s);
  else if (D.max_in == 3)
    launch_fwd_chunks<kInc, 3>(D, I, ph, reg, s);
  else
    launch_fwd_chunks<kInc, 4>(D, I, ph, reg, s);
  return hipGetLastError();
}

template <bool kInc>
static hipError_t backward_phase(const DevDesign &D, const IncArgs &I, int4 ph, hipStream_t s) {
  if (ph.z <= 0) return hipSuccess;
  const int per = kSweepBlock / kWave;
  constexpr int cpb = kInc ? 1 : kFullCpb;
  if (ph.x == kItemPiece)
    hipLaunchKernelGGL(k_backward_pieces<kInc>, dim3(blocks_for(ph.z, per)), dim3(kSweepBlock), sweep_lds_bytes(D),
                       s, D, ph.y, ph.y + ph.z, I);
  else
    hipLaunchKernelGGL((k_backward<kInc, cpb>), dim3(blocks_for(ph.z, cpb)), dim3(kSweepBlock * cpb),
                       sweep_lds_bytes(D, cpb), s, D, ph.y, ph.y + ph.z, I);
  return hipGetLastError();
}

hipError_t launch_forward_phase(const DevDesign &D, int4 ph, int4 reg, hipStream_t s) {
  return forward_phase<false>(D, IncArgs{}, ph, reg, s);
}

hipError_t launch_inc_forward_phase(const DevDesign &D, const IncArgs &I, int4 ph, int4 reg, hipStream_t s) {
  return forward_phase<true>(D, I, ph, reg, s);
}

hipError_t launch_inc_backward_phase(const DevDesign &D, const IncArgs &I, int4 ph, hipStream_t s) {
  return backward_phase<true>(D, I, ph, s);
}

hipError_t launch_backward(const DevDesign &D, int grid, bool coop, hipStream_t s) {
  return launch_sweep<kSweepBwd>(D, 0.0f, 0.0f, grid, coop, s);
}

template <int kSlots>
static void launch_bwd_push(const DevDesign &D, int4 ph, int4 reg, hipStream_t s) {
  hipLaunchKernelGGL((k_backward_push<kSlots, kFullCpb>), dim3(blocks_for(ph.z, kFullCpb)),
                     dim3(kSweepBlock * kFullCpb), span_sweep_lds_bytes(D, reg.z, kFullCpb), s, D, ph.y, reg.x,
                     reg.y, ph.z, reg.z);
}

template <int kSlots>
static hipError_t launch_flow_k(const DevDesign &D, const FlowArgs &F, bool fwd, int grid, hipStream_t s) {
  DevDesign a = D;
  FlowArgs b = F;
  void *args[] = {&a, &b};
  const void *k = fwd ? reinterpret_cast<const void *>(&k_flow_fwd<kSlots>)
                      : reinterpret_cast<const void *>(&k_flow_bwd<kSlots>);
  return hipLaunchCooperativeKernel(k, dim3(grid), dim3(kSweepBlock), args, (unsigned)sweep_lds_bytes(D), s);
}

hipError_t launch_flow(const DevDesign &D, const FlowArgs &F, bool fwd, int grid, hipStream_t s) {
  if (F.n_items <= 0) return hipSuccess;
  switch (D.max_in <= 1 ? 1 : D.max_in) {
    case 1: return launch_flow_k<1>(D, F, fwd, grid, s);
    case 2: return launch_flow_k<2>(D, F, fwd, grid, s);
    case 3: return launch_flow_k<3>(D, F, fwd, grid, s);
    default: return launch_flow_k<4>(D, F, fwd, grid, s);
  }
}

int flow_blocks_per_cu(const DevDesign &D) {
  int n = 1 << 30;
  const void *ks[] = {reinterpret_cast<const void *>(&k_flow_fwd<1>), reinterpret_cast<const void *>(&k_flow_bwd<1>),
                      reinterpret_cast<const void *>(&k_flow_fwd<2>), reinterpret_cast<const void *>(&k_flow_bwd<2>),
                      reinterpret_cast<const void *>(&k_flow_fwd<3>), reinterpret_cast<const void *>(&k_flow_bwd<3>),
                      reinterpret_cast<const void *>(&k_flow_fwd<4>), reinterpret_cast<const void *>(&k_flow_bwd<4>)};
  for (const void *k : ks) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k, kSweepBlock, sweep_lds_bytes(D)) != hipSuccess) return 0;
    n = std::min(n, b);
  }
  return n;
}

hipError_t launch_backward_phase(const DevDesign &D, int4 ph, int4 reg, hipStream_t s) {
  if (ph.z <= 0) return hipSuccess;
  if (ph.x == kItemPiece)
    hipLaunchKernelGGL(k_backward_push_pieces, dim3(blocks_for(ph.z, kSweepBlock / kWave)), dim3(kSweepBlock), 0, s,
                       D, ph.y, ph.y + ph.z);
  else if (!D.fanin4)
    launch_bwd_push<0>(D, ph, reg, s);
  else if (D.max_in <= 1)
    launch_bwd_push<1>(D, ph, reg, s);
  else if (D.max_in == 2)
    launch_bwd_push<2>(D, ph, reg, s);
  else if (D.max_in == 3)
    launch_bwd_push<3>(D, ph, reg, s);
  else
    launch_bwd_push<4>(D, ph, reg, s);
  return hipGetLastError();
}

// Plain device copy in 16-byte elements (bandwidth measurement): each
// thread moves four elements a round, all loads before the stores.
__global__ __launch_bounds__(256) void k_copy4(const float4 *__restrict__ src, float4 *__restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const float4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

// The dependent chain of one level kernel reduced to its memory accesses:
// an index load, a 32-byte gather at that index, a 32-byte store (latency
// floor measurement).
__global__ __launch_bounds__(256) void k_level_floor(const int32_t *__restrict__ idx, const PinState *__restrict__ src,
                                                     PinState *__restrict__ dst, int n, int off) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  PinState v = src[idx[off + i]];
  v.at.x += 1.0f;
  dst[off + i] = v;
}

hipError_t launch_level_floor(const int32_t *idx, const void *src, void *dst, int n, int off, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_level_floor, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, idx,
                     static_cast<const PinState *>(src), static_cast<PinState *>(dst), n, off);
  return hipGetLastError();
}

hipError_t launch_copy4(const void *src, void *dst, int64_t n16, hipStream_t s) {
  if (n16 <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n16 + 255) / 256, 256 * 32);
  hipLaunchKernelGGL(k_copy4, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const float4 *>(src),
                     static_cast<float4 *>(dst), n16);
  return hipGetLastError();
}

hipError_t launch_reduce_smooth(const DevDesign &D, double *partials, double *out, uint64_t *keys, int32_t *vals,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_smooth, dim3(kReduceBlocks), dim3(256), 0, s, D, partials, out, keys, vals);
  return hipGetLastError();
}


template <int kSlots>
static void launch_adjoint_k(const DevDesign &D, float g_tns, float g_wns, int4 ph, int lib_f4, hipStream_t s) {
  const size_t lds = span_lds_bytes(lib_f4, D.n_types) + sizeof(float2) * kChunk + sizeof(float4) * kSweepBlock;
  hipLaunchKernelGGL(k_adjoint<kSlots>, dim3(ph.z), dim3(kSweepBlock), lds, s, D, g_tns, g_wns, ph.y, ph.y + ph.z,
                     lib_f4);
}

hipError_t launch_adjoint_phase(const DevDesign &D, float g_tns, float g_wns, int4 ph, int lib_f4, hipStream_t s) {
  if (ph.z <= 0) return hipSuccess;
  if (!D.fanin4)
    launch_adjoint_k<0>(D, g_tns, g_wns, ph, lib_f4, s);
  else if (D.max_in <= 1)
    launch_adjoint_k<1>(D, g_tns, g_wns, ph, lib_f4, s);
  else if (D.max_in == 2)
    launch_adjoint_k<2>(D, g_tns, g_wns, ph, lib_f4, s);
  else if (D.max_in == 3)
    launch_adjoint_k<3>(D, g_tns, g_wns, ph, lib_f4, s);
  else
    launch_adjoint_k<4>(D, g_tns, g_wns, ph, lib_f4, s);
  return hipGetLastError();
}

hipError_t launch_rc_adjoint(const DevDesign &D, const int2 *chunks, int n_chunks, bool res, hipStream_t s) {
  if (n_chunks <= 0) return hipSuccess;
  if (res)
    hipLaunchKernelGGL(k_rc_adjoint<true>, dim3(xcd_grid(n_chunks)), dim3(kRcAdjBlock), 0, s, D, chunks, n_chunks);
  else
    hipLaunchKernelGGL(k_rc_adjoint<false>, dim3(xcd_grid(n_chunks)), dim3(kRcAdjBlock), 0, s, D, chunks, n_chunks);
  return hipGetLastError();
}

hipError_t launch_scatter_grads(const DevDesign &D, const int32_t *node_src, int64_t n_nodes, float *grad_cap,
                                float *grad_res, const int32_t *pin_loc, int n_pins, float *grad_load,
                                const int32_t *arc_src, int n_arcs, float4 *grad_arc, hipStream_t s) {
  int64_t n = n_nodes;
  if (n_pins > n) n = n_pins;
  if (n_arcs > n) n = n_arcs;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_grads, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, D, node_src, n_nodes,
                     grad_cap, grad_res, pin_loc, n_pins, grad_load, arc_src, n_arcs, grad_arc);
  return hipGetLastError();
}

template <int kKind>
static hipError_t launch_inc(const DevDesign &D, const IncArgs &I, int grid, int max_items, hipStream_t s) {
  DevDesign a = D;
  IncArgs b = I;
  int m = max_items;
  void *args[] = {&a, &b, &m};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_inc_sweep<kKind>), dim3(grid),
                                    dim3(kSweepBlock), args, (unsigned)sweep_lds_bytes(D), s);
}

hipError_t launch_inc_forward(const DevDesign &D, const IncArgs &I, int grid, int max_items, hipStream_t s) {
  return launch_inc<kSweepFwd>(D, I, grid, max_items, s);
}

hipError_t launch_inc_backward(const DevDesign &D, const IncArgs &I, int grid, int max_items, hipStream_t s) {
  return launch_inc<kSweepBwd>(D, I, grid, max_items, s);
}

hipError_t launch_inc_queues(const DevDesign &D, const IncArgs &I, bool backward, hipStream_t s) {
  const int n = backward ? D.n_ph_bwd : D.n_ph_fwd;
  if (n <= 0) return hipSuccess;
  if (backward)
    hipLaunchKernelGGL(k_inc_queues<kSweepBwd>, dim3(n), dim3(256), 0, s, D, I);
  else
    hipLaunchKernelGGL(k_inc_queues<kSweepFwd>, dim3(n), dim3(256), 0, s, D, I);
  return hipGetLastError();
}

int inc_blocks_per_cu(size_t lds_bytes) {
  int n = 1 << 30;
  const void *ks[] = {reinterpret_cast<const void *>(&k_inc_sweep<kSweepFwd>),
                      reinterpret_cast<const void *>(&k_inc_sweep<kSweepBwd>)};
  for (const void *k : ks) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k, kSweepBlock, lds_bytes) != hipSuccess) return 0;
    n = b < n ? b : n;
  }
  return n;
}

hipError_t launch_inc_maps(const DevDesign &D, const int32_t *chunk_of, int32_t *sink_cc, int4 *fanin_cc,
                           hipStream_t s) {
  const int n = D.n_sinks > D.n_drv ? D.n_sinks : D.n_drv;
  hipLaunchKernelGGL(k_inc_maps, dim3(blocks_for(n > 0 ? n : 1, 256)), dim3(256), 0, s, D, chunk_of, sink_cc,
                     fanin_cc);
  return hipGetLastError();
}

hipError_t launch_inc_seed(const DevDesign &D, const IncArgs &I, const int32_t *nets, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_inc_seed, dim3(blocks_for(n, 256)), dim3(256), 0, s, D, I, nets, n);
  return hipGetLastError();
}

hipError_t launch_reset_counters(uint32_t *counters, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_reset, dim3(blocks_for(n, 256)), dim3(256), 0, s, counters, n);
  return hipGetLastError();
}

hipError_t launch_reduce(const DevDesign &D, double *partials, double *out, uint64_t *keys, int32_t *vals,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(kReduceBlocks), dim3(256), 0, s, D, partials, out, keys, vals);
  return hipGetLastError();
}

// Endpoint orders: rocPRIM's stable onesweep radix sort at every size above
// one block (its default picks a merge-sort path below 2^20 items, about 20
// launches per sort on a million endpoints).  Both orders of an update are
// one sort of (early/late, [design,] slack) keys.
using EpSortConfig = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config,
                                                rocprim::default_config, 0>;

size_t sort_temp_bytes(int n) {
  size_t bytes = 0;
  (void)rocprim::radix_sort_pairs<EpSortConfig>(nullptr, bytes, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                                (const int32_t *)nullptr, (int32_t *)nullptr, (unsigned)n);
  return bytes;
}

hipError_t sort_endpoints(void *temp, size_t temp_bytes, const uint32_t *keys_in, uint32_t *keys_out,
                          const int32_t *vals_in, int32_t *vals_out, int n, hipStream_t s) {
  return rocprim::radix_sort_pairs<EpSortConfig>(temp, temp_bytes, keys_in, keys_out, vals_in, vals_out,
                                                 (unsigned)n, 0, 32, s);
}

hipError_t launch_reduce_batch(const DevDesign &D, const int32_t *ep_off, int n_designs, int dbits,
                               double *partials, double *out, uint64_t *keys, int32_t *vals, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_batch, dim3(kReduceBlocks, n_designs), dim3(256), 0, s, D, ep_off, partials, keys,
                     vals, dbits);
  hipLaunchKernelGGL(k_reduce_batch_final, dim3(blocks_for(n_designs, 256)), dim3(256), 0, s, partials, out,
                     n_designs);
  return hipGetLastError();
}

size_t sort_temp_bytes64(int n, int end_bit) {
  size_t bytes = 0;
  (void)rocprim::radix_sort_pairs<EpSortConfig>(nullptr, bytes, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                                (const int32_t *)nullptr, (int32_t *)nullptr, (unsigned)n, 0,
                                                (unsigned)end_bit);
  return bytes;
}

hipError_t sort_endpoints64(void *temp, size_t temp_bytes, const uint64_t *keys_in, uint64_t *keys_out,
                            const int32_t *vals_in, int32_t *vals_out, int n, int end_bit, hipStream_t s) {
  return rocprim::radix_sort_pairs<EpSortConfig>(temp, temp_bytes, keys_in, keys_out, vals_in, vals_out,
                                                 (unsigned)n, 0, (unsigned)end_bit, s);
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
                               const float *pc, int64_t n_small, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_permute_caps, dim3(blocks_for(n, 256)), dim3(256), 0, s, src, node_src, dst, n, pc,
                     n_small);
  return hipGetLastError();
}


__global__ void k_set_i32(int32_t *p, int32_t v) { *p = v; }

// The leading endpoints in slack order whose slack is below thr: the first
// failing position (cand when none fails).
__global__ void k_paths_count(const float2 *ep_slack, const int32_t *ord, int cand, int el, float thr, int32_t *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cand) return;
  const float2 e = ep_slack[ord[i]];
  if (!((el ? e.y : e.x) < thr)) atomicMin(out, i);
}

hipError_t launch_paths_count(const DevDesign &D, const int32_t *ord, int cand, int el, float thr, int32_t *out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, out, (int32_t)cand);
  if (cand > 0)
    hipLaunchKernelGGL(k_paths_count, dim3(blocks_for(cand, 256)), dim3(256), 0, s, D.ep_slack, ord, cand, el, thr,
                       out);
  return hipGetLastError();
}

size_t paths_queue_lds_bytes(const DevDesign &D, int m) {
  return lib_lds_bytes(D.n_types, D.tstride) + sizeof(int4) * (size_t)kWave * m;
}

hipError_t launch_paths_enum(const DevDesign &D, const PathArgs &A, hipStream_t s) {
  if (A.n_eps <= 0) return hipSuccess;
  if (A.items)
    hipLaunchKernelGGL(k_paths_enum<false>, dim3(blocks_for(A.n_eps, kWave)), dim3(kWave),
                       lib_lds_bytes(D.n_types, D.tstride), s, D, A);
  else
    hipLaunchKernelGGL(k_paths_enum<true>, dim3(blocks_for(A.n_eps, kWave)), dim3(kWave),
                       paths_queue_lds_bytes(D, A.m), s, D, A);
  return hipGetLastError();
}

hipError_t launch_paths_keys(const PathArgs &A, uint32_t *keys, int32_t *vals, hipStream_t s) {
  const int n = A.n_eps * A.m;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_paths_keys, dim3(blocks_for(n, 256)), dim3(256), 0, s, A, keys, vals);
  return hipGetLastError();
}

hipError_t launch_paths_lengths(const PathArgs &A, const int32_t *sel, int n_sel, int32_t *len, hipStream_t s) {
  if (n_sel <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_paths_lengths, dim3(blocks_for(n_sel, 256)), dim3(256), 0, s, A, sel, n_sel, len);
  return hipGetLastError();
}

hipError_t launch_paths_emit(const DevDesign &D, const PathArgs &A, const int32_t *sel, int n_sel,
                             const int32_t *ptr, int32_t *pin, int8_t *rf, float *slack, int32_t *ep,
                             hipStream_t s) {
  if (n_sel <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_paths_emit, dim3(blocks_for(n_sel, 256 / kWave)), dim3(256), 0, s, D, A, sel, n_sel, ptr,
                     pin, rf, slack, ep);
  return hipGetLastError();
}

hipError_t exclusive_sum(void *temp, size_t &temp_bytes, const int32_t *in, int32_t *out, int n, hipStream_t s) {
  return hipcub::DeviceScan::ExclusiveSum(temp, temp_bytes, in, out, n, s);
}

}  // namespace sta
