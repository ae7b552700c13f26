// RC trees estimated from pin positions (§III "Parasitics (RC) inputs": for
// placement flows the timer builds each net's RC tree itself from pin positions
// and unit resistance / capacitance along x and y).  Per net: a rectilinear
// minimum spanning tree grown by Prim's rule from the driver (Manhattan
// distances in FP32, ties to the lower pin index, a pin's parent the first
// tree pin at its distance), each tree edge wired as an L: along x from the
// parent to a corner node, then along y to the pin.  The t-th pin to join is
// RC nodes 2t-1 (corner) and 2t (pin); R and C of a piece are the unit values
// times its length, C lumped at the piece's far node.  A net of k sinks has
// 2k + 1 nodes, so net n starts at node n + 2 * (sinks of nets before n).
//
// Three kernels by net size, so that no pin waits on a slot it cannot use:
//   k_est_lane    one lane per net of at most 8 pins: the whole Prim loop in
//                 the lane's registers (most nets of a netlist)
//   k_est_wave    one wavefront per net of 9..64 pins, one pin per lane: each
//                 Prim step is a wave minimum of the distance bits, then of
//                 the lane indices holding it (DPP row shifts and row
//                 broadcasts, no LDS), no barrier
//   k_est_block   one 1024-thread block per larger net (up to kEstMaxPins
//                 pins, up to kEstPer per thread in registers, as many slots
//                 as the net needs): per step a thread, wave and block
//                 minimum, the 16 wave winners through double-buffered LDS
//                 with one barrier, then one branch-free pass that relaxes
//                 the distances and finds the next thread minimum; the RC
//                 nodes are written once the tree is complete
//
// A pin in the tree carries distance +inf; since positions are finite and
// bounded (checked first), every pin outside the tree has a finite distance,
// so the minimum never picks a tree pin.  In the lane and wave kernels a
// pin's owner keeps, besides its position and distance, the position and RC
// node of the tree pin that gives that distance, so the joining pin's owner
// writes both of its RC nodes without asking anyone.
#include <algorithm>
#include <mutex>
#include <vector>

#include "sta_est.h"
#include "sta_internal.h"

namespace sta {

namespace {

constexpr float kFar = __builtin_inff();
constexpr uint32_t kNone = 0xffffffffu;  // identity of the unsigned minimum
constexpr int kLanePins = 8;            // largest net of k_est_lane
constexpr int kEstPer = kEstMaxPins / 1024;  // pins per thread of k_est_block
constexpr float kMaxCoord = 1e18f;      // |x|, |y| bound: every distance stays finite

struct PinLoc {
  float x, y;
};

__device__ __forceinline__ float manhattan(float ax, float ay, float bx, float by) {
  return fabsf(ax - bx) + fabsf(ay - by);
}

// Unsigned minimum over the 64 lanes (all active), as a uniform value: an
// inclusive min-scan inside each row of 16 by row shifts 1, 2, 4, 8, then row
// broadcasts 15 and 31 carry rows 0-1 and 0-2 into rows 1-3; lane 63 ends
// with the minimum of the wave.  Lanes whose DPP source is outside the row
// (or whose row is masked off) take kNone, the identity.
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)kNone, (int)v, 0x111, 0xf, 0xf, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)kNone, (int)v, 0x112, 0xf, 0xf, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)kNone, (int)v, 0x114, 0xf, 0xf, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)kNone, (int)v, 0x118, 0xf, 0xf, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)kNone, (int)v, 0x142, 0xa, 0xf, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)kNone, (int)v, 0x143, 0xc, 0xf, false));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Minimum within each row of 16 lanes (all active), as a uniform value: the
// row-shift scan of wave_min, read at lane 15 (row 0; every row holds the
// same 16 values where this is used).
__device__ __forceinline__ uint32_t row_min16(uint32_t v) {
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)kNone, (int)v, 0x111, 0xf, 0xf, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)kNone, (int)v, 0x112, 0xf, 0xf, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)kNone, (int)v, 0x114, 0xf, 0xf, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)kNone, (int)v, 0x118, 0xf, 0xf, false));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
}

// Non-negative floats order like their bit patterns.
__device__ __forceinline__ uint32_t key_of(float d) { return __float_as_uint(d); }

__device__ __forceinline__ float lane_float(float v, uint32_t lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), (int)lane));
}

// Both RC nodes of the t-th pin to join, from its parent's position and node.
__device__ __forceinline__ void emit_pin(const EstArgs &A, int64_t base, int t, float x, float y, float px, float py,
                                         int pnode) {
  const float lx = fabsf(x - px), ly = fabsf(y - py);
  const int64_t a = base + 2 * t - 1, b = a + 1;
  A.parent[a] = pnode;
  A.res[a] = A.rx * lx;
  A.cap[a] = A.cx * lx;
  A.parent[b] = 2 * t - 1;
  A.res[b] = A.ry * ly;
  A.cap[b] = A.cy * ly;
}

__device__ __forceinline__ void emit_root(const EstArgs &A, int n, int64_t base) {
  A.parent[base] = -1;
  A.res[base] = 0.0f;
  A.cap[base] = 0.0f;
  A.node_ptr[n + 1] = base + 2 * (int64_t)(A.sink_ptr[n + 1] - A.sink_ptr[n]) + 1;
  if (n == 0) A.node_ptr[0] = 0;
}

// One lane per net of at most kLanePins pins (the rest return at once).
__global__ __launch_bounds__(256) void k_est_lane(EstArgs A) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= A.n_nets) return;
  const int s0 = A.sink_ptr[n], k = A.sink_ptr[n + 1] - s0;
  if (k + 1 > kLanePins) return;
  const int64_t base = (int64_t)n + 2 * (int64_t)s0;
  const int drv = A.driver[n];
  float x[kLanePins], y[kLanePins], dist[kLanePins], px[kLanePins], py[kLanePins];
  int pnode[kLanePins];
#pragma unroll
  for (int u = 0; u < kLanePins; ++u) {
    const int pin = (u >= 1 && u <= k) ? A.sink_pin[s0 + u - 1] : drv;
    x[u] = A.x[pin];
    y[u] = A.y[pin];
  }
#pragma unroll
  for (int u = 0; u < kLanePins; ++u) {
    dist[u] = (u >= 1 && u <= k) ? manhattan(x[u], y[u], x[0], y[0]) : kFar;
    px[u] = x[0];
    py[u] = y[0];
    pnode[u] = 0;
  }
  emit_root(A, n, base);
  for (int t = 1; t <= k; ++t) {
    float best = kFar;
    int j = 0;
#pragma unroll
    for (int u = 1; u < kLanePins; ++u)  // ascending u: the first minimum wins ties
      if (dist[u] < best) {
        best = dist[u];
        j = u;
      }
    float xj = x[1], yj = y[1], pxj = px[1], pyj = py[1];
    int pnj = pnode[1];
#pragma unroll
    for (int u = 2; u < kLanePins; ++u)
      if (u == j) {
        xj = x[u];
        yj = y[u];
        pxj = px[u];
        pyj = py[u];
        pnj = pnode[u];
      }
    emit_pin(A, base, t, xj, yj, pxj, pyj, pnj);
    A.sink_node[s0 + j - 1] = 2 * t;
#pragma unroll
    for (int u = 1; u < kLanePins; ++u) {
      if (u == j) {
        dist[u] = kFar;
      } else if (dist[u] < kFar) {
        const float d = manhattan(x[u], y[u], xj, yj);
        if (d < dist[u]) {
          dist[u] = d;
          px[u] = xj;
          py[u] = yj;
          pnode[u] = 2 * t;
        }
      }
    }
  }
}

// One wavefront per net of list[0 .. *count).
__global__ __launch_bounds__(256) void k_est_wave(EstArgs A, const int32_t *list, const uint32_t *count) {
  const int w = blockIdx.x * (256 / kWave) + (int)(threadIdx.x / kWave);
  if (w >= (int)*count) return;
  const int n = list[w];
  const int lane = threadIdx.x & (kWave - 1);
  const int s0 = A.sink_ptr[n], k = A.sink_ptr[n + 1] - s0;
  const int64_t base = (int64_t)n + 2 * (int64_t)s0;
  const bool valid = lane <= k;
  const int pin = (lane == 0 || !valid) ? A.driver[n] : A.sink_pin[s0 + lane - 1];
  const float x = A.x[pin], y = A.y[pin];
  const float x0 = lane_float(x, 0), y0 = lane_float(y, 0);
  float dist = (valid && lane > 0) ? manhattan(x, y, x0, y0) : kFar;
  float px = x0, py = y0;
  int pnode = 0;
  if (lane == 0) emit_root(A, n, base);
  for (int t = 1; t <= k; ++t) {
    const uint32_t kmin = wave_min(key_of(dist));
    const uint32_t j = wave_min(key_of(dist) == kmin ? (uint32_t)lane : kNone);
    const float xj = lane_float(x, j), yj = lane_float(y, j);
    if (lane == (int)j) {
      emit_pin(A, base, t, x, y, px, py, pnode);
      A.sink_node[s0 + j - 1] = 2 * t;
      dist = kFar;
    } else if (dist < kFar) {
      const float d = manhattan(x, y, xj, yj);
      if (d < dist) {
        dist = d;
        px = xj;
        py = yj;
        pnode = 2 * t;
      }
    }
  }
}

// One net of k_est_block with NL live register slots per thread (pin
// l = tid + 1024 u, u < NL).  Per step only distances and parent nodes move;
// the RC nodes are written after the last step, when every pin knows its join
// step and its parent's node (the parent's pin comes from the join table).
// Every pin's position is also kept in LDS, where each step reads the joining
// pin's (a per-slot select of the candidate's position would cost three more
// instructions per slot and step).
template <int NL>
__device__ __forceinline__ void est_block_net(const EstArgs &A, int n, int s0, int k, int64_t base,
                                              uint32_t (*s_key)[1024 / kWave], uint32_t (*s_idx)[1024 / kWave],
                                              PinLoc *s_pos, uint16_t *s_join) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const float x0 = A.x[A.driver[n]], y0 = A.y[A.driver[n]];
  const float kNaN = __builtin_nanf("");
  float x[NL], y[NL], dist[NL];
  int pnode[NL], tj[NL];
  float key = kFar;
  int ul = 0;
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int l = tid + u * 1024;  // pin index in the net: 0 driver, 1..k sinks
    const bool valid = l >= 1 && l <= k;
    const int pin = A.sink_pin[s0 + (valid ? l - 1 : 0)];
    x[u] = valid ? A.x[pin] : kNaN;  // NaN: never nearer than anything
    y[u] = valid ? A.y[pin] : kNaN;
    if (valid) s_pos[l] = PinLoc{x[u], y[u]};
    dist[u] = valid ? manhattan(x[u], y[u], x0, y0) : kFar;
    pnode[u] = 0;
    tj[u] = 0;
    const bool b = dist[u] < key;  // ascending l: the first minimum wins ties
    key = b ? dist[u] : key;
    ul = b ? u : ul;
  }
  __syncthreads();  // s_pos complete
  for (int t = 1; t <= k; ++t) {
    const uint32_t wk = wave_min(key_of(key));
    const uint32_t wi = wave_min(key_of(key) == wk && key < kFar ? (uint32_t)(tid + ul * 1024) : kNone);
    const int buf = t & 1;
    if (lane == 0) {
      s_key[buf][wave] = wk;
      s_idx[buf][wave] = wi;
    }
    __syncthreads();
    // the 16 wave winners, one per lane of each row: row minima by DPP, so
    // the reduction costs every wave a few vector instructions; every row
    // holds all 16, so the result is the same in every lane
    const int e = lane & (1024 / kWave - 1);
    const uint32_t ek = s_key[buf][e], ei = s_idx[buf][e];
    const uint32_t bk = row_min16(ek);
    const uint32_t bi = row_min16(ek == bk ? ei : kNone);
    const int j = (int)__builtin_amdgcn_readfirstlane((int)bi);  // a pin outside the tree is left
    const PinLoc pj = s_pos[j];
    const float xj = pj.x, yj = pj.y;
    const int ju = j >> 10;
    if (tid == (j & 1023)) {  // the joining pin leaves the candidates
#pragma unroll
      for (int u = 0; u < NL; ++u)
        if (u == ju) {
          x[u] = kNaN;
          dist[u] = kFar;
          tj[u] = t;
        }
    }
    if (tid == 0) s_join[t] = (uint16_t)j;
    key = kFar;
    ul = 0;
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const float d = manhattan(x[u], y[u], xj, yj);  // NaN for tree and padding pins
      const bool up = d < dist[u];
      dist[u] = up ? d : dist[u];
      pnode[u] = up ? 2 * t : pnode[u];
      const bool b = dist[u] < key;
      key = b ? dist[u] : key;
      ul = b ? u : ul;
    }
  }
  __syncthreads();  // s_join complete
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int l = tid + u * 1024;
    if (l >= 1 && l <= k) {
      const int pin = A.sink_pin[s0 + l - 1];
      const int lp = pnode[u] == 0 ? 0 : (int)s_join[pnode[u] / 2];
      const int ppin = lp == 0 ? A.driver[n] : A.sink_pin[s0 + lp - 1];
      emit_pin(A, base, tj[u], A.x[pin], A.y[pin], A.x[ppin], A.y[ppin], pnode[u]);
      A.sink_node[s0 + l - 1] = 2 * tj[u];
    }
  }
  if (tid == 0) emit_root(A, n, base);
}

// One block per net of list[0 .. *count), looping over the list with a
// fixed grid; the net's size picks how many register slots each thread runs.
__global__ __launch_bounds__(1024) void k_est_block(EstArgs A, const int32_t *list, const uint32_t *count) {
  __shared__ uint32_t s_key[2][1024 / kWave];
  __shared__ uint32_t s_idx[2][1024 / kWave];
  __shared__ PinLoc s_pos[kEstMaxPins];
  __shared__ uint16_t s_join[kEstMaxPins];
  const int nb = (int)*count;
  for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    const int n = list[b];
    const int s0 = A.sink_ptr[n], k = A.sink_ptr[n + 1] - s0;
    const int64_t base = (int64_t)n + 2 * (int64_t)s0;
    switch (k >> 10) {  // live slots - 1: pins 0..k over 1024 threads
#define STA_EST_NET(c) \
  case c - 1:          \
    est_block_net<c>(A, n, s0, k, base, s_key, s_idx, s_pos, s_join); \
    break;
      STA_EST_NET(1) STA_EST_NET(2) STA_EST_NET(3) STA_EST_NET(4) STA_EST_NET(5) STA_EST_NET(6)
      STA_EST_NET(7) STA_EST_NET(8) STA_EST_NET(9) STA_EST_NET(10) STA_EST_NET(11) STA_EST_NET(12)
#undef STA_EST_NET
      default:
        break;  // more than kEstMaxPins pins: refused by the host before launch
    }
    __syncthreads();  // the next net reuses the buffers
  }
}

// Input check and work split in one pass.  st[0] / st[1] count the nets of
// 9..64 pins / of more than 64 pins (listed in mid / big, in any order: a
// net's result depends on the net alone), st[2] is the largest sink count,
// st[3] / st[4] / st[5] the first net (CSR or driver), sink entry and pin
// position found malformed (kNone when none).  The host reads st before any
// estimation kernel runs, so those never see a bad index or position.
// Exclusive prefix of c over a 256-thread block (a scan per wavefront, then
// the wavefront totals); *total gets the block's sum.  Every thread calls it.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t c, uint32_t *s_w, uint32_t *total) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  int v = (int)c;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(v, o, kWave);
    v += lane >= o ? y : 0;
  }
  if (lane == kWave - 1) s_w[wave] = (uint32_t)v;
  __syncthreads();
  uint32_t off = 0, tot = 0;
  for (int w = 0; w < 256 / kWave; ++w) {
    off += w < wave ? s_w[w] : 0u;
    tot += s_w[w];
  }
  *total = tot;
  return off + (uint32_t)v - c;
}

__device__ __forceinline__ bool est_mid_net(const EstArgs &A, int n, int n_pins, int n_sinks) {
  const int a = A.sink_ptr[n], b = A.sink_ptr[n + 1], drv = A.driver[n];
  const bool ok = a >= 0 && b >= a && b <= n_sinks && (n > 0 || a == 0) && drv >= 0 && drv < n_pins;
  return ok && b - a + 1 <= kWave && b - a + 1 > kLanePins;
}

// The mid list is filled without one atomic per net on a single counter (tens
// of thousands of those serialized at one L2 address): each block counts its
// mid nets first, reserves their slots with one atomic, then writes them.
// The lists hold at most mid_cap and big_cap entries; the counts in st[0] and
// st[1] keep counting past them, so the host sees when a list was too short.
__global__ __launch_bounds__(256) void k_est_check(EstArgs A, int n_pins, int n_sinks, int32_t *mid, int32_t *big,
                                                   uint32_t *st, uint32_t mid_cap, uint32_t big_cap) {
  __shared__ uint32_t s_w[256 / kWave];
  __shared__ uint32_t s_base;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t top = max(max((int64_t)A.n_nets, (int64_t)n_sinks), (int64_t)n_pins);
  uint32_t cnt = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < A.n_nets; i += stride)
    cnt += est_mid_net(A, (int)i, n_pins, n_sinks) ? 1u : 0u;
  uint32_t tot;
  uint32_t pos = block_excl_scan(cnt, s_w, &tot);
  if (threadIdx.x == 0) s_base = tot > 0 ? atomicAdd(&st[0], tot) : 0u;
  __syncthreads();
  pos += s_base;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < top; i += stride) {
    if (i < A.n_nets) {
      const int n = (int)i;
      const int a = A.sink_ptr[n], b = A.sink_ptr[n + 1], drv = A.driver[n];
      const bool ok = a >= 0 && b >= a && b <= n_sinks && (n > 0 || a == 0) && drv >= 0 && drv < n_pins;
      if (!ok) {
        atomicMin(&st[3], (uint32_t)n);
      } else if (b - a + 1 > kWave) {
        const uint32_t k = atomicAdd(&st[1], 1u);
        if (k < big_cap) big[k] = n;
        atomicMax(&st[2], (uint32_t)(b - a));
      } else if (b - a + 1 > kLanePins) {
        if (pos < mid_cap) mid[pos] = n;
        ++pos;
      }
    }
    if (i < n_sinks) {
      const int p = A.sink_pin[i];
      if (p < 0 || p >= n_pins) atomicMin(&st[4], (uint32_t)i);
    }
    if (i < n_pins) {  // also false for NaN
      if (!(fabsf(A.x[i]) <= kMaxCoord && fabsf(A.y[i]) <= kMaxCoord)) atomicMin(&st[5], (uint32_t)i);
    }
  }
}

// ------------------------------------------------- gradient to positions
//
// With the tree fixed, the edge parent pin p -> pin c puts R = r_x |x_c - x_p|
// and C = c_x |x_c - x_p| on its corner node a and the y terms on its pin node
// b, so it adds v_x = sgn(x_c - x_p) (r_x dJ/dR_a + c_x dJ/dC_a) to dJ/dx_c and
// -v_x to dJ/dx_p, likewise along y (sgn(0) = 0).  A pin's gradient is its own
// edge's term plus the negated terms of its child edges.  The lane and wave
// kernels add them in FP32 in sink order; the block kernel adds them as
// integers (each term rounded to 2^-48 of the net's largest term), exact in
// any order, so every tier is reproducible bit for bit.

__device__ __forceinline__ float sgnf(float v) { return v > 0.0f ? 1.0f : (v < 0.0f ? -1.0f : 0.0f); }

// One lane per net of at most kLanePins pins.
__global__ __launch_bounds__(256) void k_estg_lane(EstGradArgs G) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= G.n_nets) return;
  const int s0 = G.sink_ptr[n], k = G.sink_ptr[n + 1] - s0;
  if (k + 1 > kLanePins) return;
  const int64_t base = (int64_t)n + 2 * (int64_t)s0;
  int pin[kLanePins], node[kLanePins];
  float x[kLanePins], y[kLanePins], gx[kLanePins], gy[kLanePins];
  pin[0] = G.driver[n];
  node[0] = 0;
#pragma unroll
  for (int u = 1; u < kLanePins; ++u) {
    pin[u] = u <= k ? G.sink_pin[s0 + u - 1] : pin[0];
    node[u] = u <= k ? G.sink_node[s0 + u - 1] : -1;
  }
#pragma unroll
  for (int u = 0; u < kLanePins; ++u) {
    x[u] = G.x[pin[u]];
    y[u] = G.y[pin[u]];
    gx[u] = gy[u] = 0.0f;
  }
#pragma unroll
  for (int u = 1; u < kLanePins; ++u) {
    if (u > k) break;
    const int b = node[u], a = b - 1;
    const int pn = G.parent[base + a];
    float px = x[0], py = y[0];
#pragma unroll
    for (int v = 1; v < kLanePins; ++v) {
      px = node[v] == pn ? x[v] : px;
      py = node[v] == pn ? y[v] : py;
    }
    const float vx = sgnf(x[u] - px) * (G.rx * G.g_res[base + a] + G.cx * G.g_cap[base + a]);
    const float vy = sgnf(y[u] - py) * (G.ry * G.g_res[base + b] + G.cy * G.g_cap[base + b]);
    gx[u] += vx;
    gy[u] += vy;
#pragma unroll
    for (int v = 0; v < kLanePins; ++v) {
      gx[v] -= node[v] == pn ? vx : 0.0f;
      gy[v] -= node[v] == pn ? vy : 0.0f;
    }
  }
#pragma unroll
  for (int u = 0; u < kLanePins; ++u)
    if (u <= k) {
      G.gx[pin[u]] = gx[u];
      G.gy[pin[u]] = gy[u];
    }
}

// One wavefront per net of list[0 .. *count) (9..64 pins), one pin per lane.
__global__ __launch_bounds__(256) void k_estg_wave(EstGradArgs G, const int32_t *list, const uint32_t *count) {
  __shared__ int32_t s_inv[256 / kWave][kWave];
  const int wv = threadIdx.x / kWave;
  const int w = blockIdx.x * (256 / kWave) + wv;
  if (w >= (int)*count) return;
  const int n = list[w];
  const int lane = threadIdx.x & (kWave - 1);
  const int s0 = G.sink_ptr[n], k = G.sink_ptr[n + 1] - s0;
  const int64_t base = (int64_t)n + 2 * (int64_t)s0;
  const bool valid = lane <= k;
  const int pin = (lane == 0 || !valid) ? G.driver[n] : G.sink_pin[s0 + lane - 1];
  const int node = (lane == 0 || !valid) ? 0 : G.sink_node[s0 + lane - 1];
  const float x = G.x[pin], y = G.y[pin];
  // lane of the pin at each pin node 2t (t = 1..k); slot 0 the driver
  s_inv[wv][lane] = 0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (valid && lane > 0) s_inv[wv][node >> 1] = lane;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  int q = 0;  // this pin's parent lane
  float vx = 0.0f, vy = 0.0f;
  if (valid && lane > 0) {
    const int b = node, a = b - 1;
    q = s_inv[wv][G.parent[base + a] >> 1];
    const float px = G.x[q == 0 ? G.driver[n] : G.sink_pin[s0 + q - 1]];
    const float py = G.y[q == 0 ? G.driver[n] : G.sink_pin[s0 + q - 1]];
    vx = sgnf(x - px) * (G.rx * G.g_res[base + a] + G.cx * G.g_cap[base + a]);
    vy = sgnf(y - py) * (G.ry * G.g_res[base + b] + G.cy * G.g_cap[base + b]);
  }
  float gx = vx, gy = vy;
  for (int l = 1; l <= k; ++l) {  // child terms in sink order
    const int ql = __builtin_amdgcn_readlane(q, l);
    const float ax = lane_float(vx, (uint32_t)l), ay = lane_float(vy, (uint32_t)l);
    gx -= lane == ql ? ax : 0.0f;
    gy -= lane == ql ? ay : 0.0f;
  }
  if (valid) {
    G.gx[pin] = gx;
    G.gy[pin] = gy;
  }
}

// Fixed-point exponent for terms of magnitude up to m: a slot sums at most
// kEstMaxPins terms, so 2^e m kEstMaxPins stays below 2^62.
__device__ __forceinline__ int fix_exp(float m) {
  return m > 0.0f ? 48 - ilogbf(m) : 0;
}

// One block per net of list[0 .. *count) (more than 64 pins), accumulating
// into acc[2 * (off[b] + slot)] (x) and [+1] (y), zeroed by the host.
__global__ __launch_bounds__(1024) void k_estg_block(EstGradArgs G, const int32_t *list, const uint32_t *count,
                                                     const int64_t *off, unsigned long long *acc) {
  __shared__ uint16_t s_inv[kEstMaxPins];  // slot of the pin at node 2t, by t (0: the driver)
  __shared__ uint32_t s_max[2][1024 / kWave];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int nb = (int)*count;
  for (int bi = blockIdx.x; bi < nb; bi += gridDim.x) {
    const int n = list[bi];
    const int s0 = G.sink_ptr[n], k = G.sink_ptr[n + 1] - s0;
    const int64_t base = (int64_t)n + 2 * (int64_t)s0;
    unsigned long long *ax = acc + 2 * off[bi];
    for (int t = tid; t <= k; t += 1024) s_inv[t] = 0;
    __syncthreads();
    for (int l = 1 + tid; l <= k; l += 1024) s_inv[G.sink_node[s0 + l - 1] >> 1] = (uint16_t)l;
    __syncthreads();
    // pass 1: every term, and the largest magnitude per axis
    float mx = 0.0f, my = 0.0f;
    for (int l = 1 + tid; l <= k; l += 1024) {
      const int b = G.sink_node[s0 + l - 1], a = b - 1;
      const int q = s_inv[G.parent[base + a] >> 1];
      const int pin = G.sink_pin[s0 + l - 1], ppin = q == 0 ? G.driver[n] : G.sink_pin[s0 + q - 1];
      const float vx = sgnf(G.x[pin] - G.x[ppin]) * (G.rx * G.g_res[base + a] + G.cx * G.g_cap[base + a]);
      const float vy = sgnf(G.y[pin] - G.y[ppin]) * (G.ry * G.g_res[base + b] + G.cy * G.g_cap[base + b]);
      mx = fmaxf(mx, fabsf(vx));
      my = fmaxf(my, fabsf(vy));
    }
    const uint32_t wx = kNone - wave_min(kNone - __float_as_uint(mx));  // max of non-negative floats
    const uint32_t wy = kNone - wave_min(kNone - __float_as_uint(my));
    if (lane == 0) {
      s_max[0][wave] = wx;
      s_max[1][wave] = wy;
    }
    __syncthreads();
    uint32_t bx = 0, by = 0;
#pragma unroll
    for (int w = 0; w < 1024 / kWave; ++w) {
      bx = max(bx, s_max[0][w]);
      by = max(by, s_max[1][w]);
    }
    const int ex = fix_exp(__uint_as_float(bx)), ey = fix_exp(__uint_as_float(by));
    // pass 2: integer sums (own term, and the negated term on the parent)
    for (int l = 1 + tid; l <= k; l += 1024) {
      const int b = G.sink_node[s0 + l - 1], a = b - 1;
      const int q = s_inv[G.parent[base + a] >> 1];
      const int pin = G.sink_pin[s0 + l - 1], ppin = q == 0 ? G.driver[n] : G.sink_pin[s0 + q - 1];
      const float vx = sgnf(G.x[pin] - G.x[ppin]) * (G.rx * G.g_res[base + a] + G.cx * G.g_cap[base + a]);
      const float vy = sgnf(G.y[pin] - G.y[ppin]) * (G.ry * G.g_res[base + b] + G.cy * G.g_cap[base + b]);
      const long long ix = __double2ll_rn(ldexp((double)vx, ex)), iy = __double2ll_rn(ldexp((double)vy, ey));
      atomicAdd(ax + 2 * l, (unsigned long long)ix);
      atomicAdd(ax + 2 * q, (unsigned long long)(-ix));
      atomicAdd(ax + 2 * l + 1, (unsigned long long)iy);
      atomicAdd(ax + 2 * q + 1, (unsigned long long)(-iy));
    }
    __threadfence();
    __syncthreads();
    for (int l = tid; l <= k; l += 1024) {
      const int pin = l == 0 ? G.driver[n] : G.sink_pin[s0 + l - 1];
      const long long sx = (long long)__hip_atomic_load(ax + 2 * l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const long long sy = (long long)__hip_atomic_load(ax + 2 * l + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      G.gx[pin] = (float)ldexp((double)sx, -ex);
      G.gy[pin] = (float)ldexp((double)sy, -ey);
    }
    __syncthreads();  // s_inv and s_max are reused by the next net
  }
}

// Checks of the tree arrays and the work split for the gradient: st[0] / st[1]
// count the nets of 9..64 / more than 64 pins (lists mid / big), st[2] is the
// first sink whose node or corner parent is not a valid estimated-tree entry
// (kNone when none), off[] gets each big net's accumulator offset and
// *total their sum.  The net CSR and positions are checked by k_est_check.
__global__ __launch_bounds__(256) void k_estg_check(EstGradArgs G, int n_sinks, int32_t *mid, int32_t *big,
                                                    int64_t *off, unsigned long long *total, uint32_t *st) {
  __shared__ uint32_t s_w[256 / kWave];
  __shared__ uint32_t s_base;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t top = max((int64_t)G.n_nets, (int64_t)n_sinks);
  uint32_t cnt = 0;  // mid nets of this thread, slots reserved per block as in k_est_check
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < G.n_nets; i += stride) {
    const int k = G.sink_ptr[i + 1] - G.sink_ptr[i];
    cnt += k + 1 <= kWave && k + 1 > kLanePins ? 1u : 0u;
  }
  uint32_t tot;
  uint32_t pos = block_excl_scan(cnt, s_w, &tot);
  if (threadIdx.x == 0) s_base = tot > 0 ? atomicAdd(&st[0], tot) : 0u;
  __syncthreads();
  pos += s_base;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < top; i += stride) {
    if (i < G.n_nets) {
      const int n = (int)i;
      const int k = G.sink_ptr[n + 1] - G.sink_ptr[n];
      if (k + 1 > kWave) {
        const uint32_t b = atomicAdd(&st[1], 1u);
        big[b] = n;
        off[b] = (int64_t)atomicAdd(total, (unsigned long long)(k + 1));
      } else if (k + 1 > kLanePins) {
        mid[pos++] = n;
      }
    }
  }
  // sinks: node 2t with 1 <= t <= k, corner parent an even node below the corner
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < G.n_nets; i += stride) {
    const int n = (int)i;
    const int s0 = G.sink_ptr[n], k = G.sink_ptr[n + 1] - s0;
    if (k + 1 > kWave) continue;  // checked by the block-wide pass below
    const int64_t base = (int64_t)n + 2 * (int64_t)s0;
    for (int s = s0; s < s0 + k; ++s) {
      const int b = G.sink_node[s];
      const bool ok = b >= 2 && b <= 2 * k && (b & 1) == 0 && G.parent[base + b - 1] >= 0 &&
                      G.parent[base + b - 1] <= b - 2 && (G.parent[base + b - 1] & 1) == 0;
      if (!ok) atomicMin(&st[2], (uint32_t)s);
    }
  }
}

// The same sink checks for the nets of more than 64 pins, one block per net.
__global__ __launch_bounds__(256) void k_estg_check_big(EstGradArgs G, const int32_t *big, const uint32_t *count,
                                                        uint32_t *st) {
  for (int bi = blockIdx.x; bi < (int)*count; bi += gridDim.x) {
    const int n = big[bi];
    const int s0 = G.sink_ptr[n], k = G.sink_ptr[n + 1] - s0;
    const int64_t base = (int64_t)n + 2 * (int64_t)s0;
    for (int s = s0 + threadIdx.x; s < s0 + k; s += blockDim.x) {
      const int b = G.sink_node[s];
      const bool ok = b >= 2 && b <= 2 * k && (b & 1) == 0 && G.parent[base + b - 1] >= 0 &&
                      G.parent[base + b - 1] <= b - 2 && (G.parent[base + b - 1] & 1) == 0;
      if (!ok) atomicMin(&st[2], (uint32_t)s);
    }
  }
}

inline int blocks_of(int64_t n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

hipError_t launch_est_check(const EstArgs &A, int n_pins, int n_sinks, int32_t *mid, int32_t *big, uint32_t *st,
                            hipStream_t s, uint32_t mid_cap, uint32_t big_cap) {
  const int64_t top = std::max<int64_t>(std::max(A.n_nets, n_sinks), n_pins);
  if (top <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((top + 255) / 256, 8192);
  const uint32_t all = (uint32_t)std::max(A.n_nets, 0);
  hipLaunchKernelGGL(k_est_check, dim3(grid), dim3(256), 0, s, A, n_pins, n_sinks, mid, big, st,
                     std::min(mid_cap, all), std::min(big_cap, all));
  return hipGetLastError();
}

// Fixed device scratch of sta_estimate_rc_noalloc: the six check words, then
// the two net lists.  Each device the library runs on holds its own copy (its
// address is looked up per device, below) until the process ends.
static __device__ __align__(256) unsigned char scratch[kEstScratchBytes];

hipError_t est_noalloc_scratch(int device, unsigned char **ptr) {
  static std::mutex mu;
  static std::vector<unsigned char *> addr;  // per device, filled on first use
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0) return hipErrorInvalidDevice;
  if ((size_t)device >= addr.size()) addr.resize((size_t)device + 1, nullptr);
  if (!addr[(size_t)device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes the device current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[(size_t)device] = static_cast<unsigned char *>(p);
  }
  *ptr = addr[(size_t)device];
  return hipSuccess;
}

hipError_t launch_est(const EstArgs &A, const int32_t *mid, const int32_t *big, const uint32_t *st, uint32_t n_mid,
                      uint32_t n_big, hipStream_t s) {
  if (A.n_nets <= 0) return hipSuccess;
  if (n_big > 0)  // first: the longest blocks start before the short work fills the chip
    hipLaunchKernelGGL(k_est_block, dim3(std::min<uint32_t>(n_big, 4096u)), dim3(1024), 0, s, A, big, st + 1);
  if (n_mid > 0)
    hipLaunchKernelGGL(k_est_wave, dim3(blocks_of(n_mid, 256 / kWave)), dim3(256), 0, s, A, mid, st);
  hipLaunchKernelGGL(k_est_lane, dim3(blocks_of(A.n_nets, 256)), dim3(256), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_estg_check(const EstGradArgs &G, int n_sinks, int32_t *mid, int32_t *big, int64_t *off,
                             unsigned long long *total, uint32_t *st, hipStream_t s) {
  const int64_t top = std::max<int64_t>(G.n_nets, n_sinks);
  if (top <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((top + 255) / 256, 8192);
  hipLaunchKernelGGL(k_estg_check, dim3(grid), dim3(256), 0, s, G, n_sinks, mid, big, off, total, st);
  return hipGetLastError();
}

hipError_t launch_estg_check_big(const EstGradArgs &G, const int32_t *big, uint32_t *st, hipStream_t s) {
  if (G.n_nets <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_estg_check_big, dim3(std::min(G.n_nets, 1024)), dim3(256), 0, s, G, big, st + 1, st);
  return hipGetLastError();
}

hipError_t launch_estg(const EstGradArgs &G, const int32_t *mid, const int32_t *big, const uint32_t *st,
                       const int64_t *off, unsigned long long *acc, uint32_t n_mid, uint32_t n_big, hipStream_t s) {
  if (G.n_nets <= 0) return hipSuccess;
  if (n_big > 0)
    hipLaunchKernelGGL(k_estg_block, dim3(std::min<uint32_t>(n_big, 4096u)), dim3(1024), 0, s, G, big, st + 1, off,
                       acc);
  if (n_mid > 0)
    hipLaunchKernelGGL(k_estg_wave, dim3(blocks_of(n_mid, 256 / kWave)), dim3(256), 0, s, G, mid, st);
  hipLaunchKernelGGL(k_estg_lane, dim3(blocks_of(G.n_nets, 256)), dim3(256), 0, s, G);
  return hipGetLastError();
}

}  // namespace sta
