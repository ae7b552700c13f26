// RC trees estimated from pin positions (§III "Parasitics (RC) inputs": for
// placement flows the timer builds each net's RC tree itself from pin positions
// and unit resistance / capacitance along x and y, as rectilinear Steiner
// trees).  Per net, the shortest-path heuristic of Takahashi and Matsuyama
// taken to the rectilinear plane: the tree starts as the driver's point; each
// step t joins the pin nearest to the tree's wires (FP32 Manhattan distance to
// the nearest point of a wire, ties to the lower pin index) along an L from
// that point q_t: segment 2t-1 along x to the corner (x_j, q_t.y), segment 2t
// along y to the pin.  A pin keeps its nearest distance, segment and point;
// a new segment replaces them only if strictly nearer (2t-1 before 2t).
//
// RC nodes: the driver D and per step the attach point S_t, the corner K_t
// and the pin J_t (3k + 1 per net of k sinks, so net n starts at node
// n + 3 * sink_ptr[n]).  The points on a segment (its start, the S of every
// later step attached to it, its end) form a chain by distance from the start,
// ties by step, each the parent of the next.  Nodes are numbered segment by
// segment (0, 1, ..., 2k), each segment's S points then its end: every start
// lies on an earlier segment, so parents precede children, and each index is
// closed-form from three counts per step (splits on the segments 0, 2t-1, 2t)
// and the step's rank on its own segment.  A node's R and C are its axis's unit
// values times the coordinate distance to its parent, C lumped at the node.
//
// Three kernels by net size (each pin a thread):
//   k_est_group<8>   one net of at most 8 pins per 8 lanes
//   k_est_group<64>  one net of 9..64 pins per wavefront
//   k_est_block      one 1024-thread block per larger net (up to kEstMaxPins
//                    pins, up to kEstPer per thread in registers)
// Each runs the join loop (a group minimum of the distance bits, then of the
// lowest pin holding it; the winner's attach point and position broadcast),
// records every step (attach point, segment, pin), and then numbers and
// writes the nodes with one thread per step: a pass over the net's steps (in
// the block kernel, over the steps on the same wire, found through a list
// ordered by wire) gives each step its rank and chain neighbours, a prefix sum
// over steps the segment offsets.
//
// The gradient mode (sta_estimate_rc_backward) rebuilds the trees the same
// way, checks them against the caller's, and sends each node's dJ/dR and
// dJ/dC to the two pins whose coordinates bound its piece: every node
// coordinate is a copy of one pin's (a clamp picks one of its candidates), so
// a piece |c_u - c_w| along x adds sgn(c_u - c_w) (r_x dJ/dR + c_x dJ/dC) to
// dJ/dx of c_u's pin and the negative to c_w's.  Terms are summed as integers
// (each rounded to 2^-44 of the net's largest term), exact in any order.
#include <algorithm>
#include <mutex>
#include <vector>

#include "sta_est.h"
#include "sta_internal.h"

namespace sta {

namespace {

constexpr float kFar = __builtin_inff();
constexpr uint32_t kNone = 0xffffffffu;  // identity of the unsigned minimum
constexpr int kLanePins = 8;            // largest net of k_est_group<8>
constexpr int kEstPer = kEstMaxPins / 1024;  // pins per thread of k_est_block
constexpr float kMaxCoord = 1e18f;      // |x|, |y| bound: every distance stays finite

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


// A pin's nearest point of the tree so far: distance, segment, the point and
// the net-local pins its two coordinates are copied from.
struct Near {
  float d, qx, qy;
  int seg, sqx, sqy;
};

// The step just made: its attach point (and sources), the joined pin's
// position and net-local index.
struct Join {
  float qx, qy, xj, yj;
  int sqx, sqy, j;
};

// The nearest point of [lo, hi] to v, and the pin it is copied from.
__device__ __forceinline__ void clamp_src(float v, int sv, float a, int sa, float b, int sb, float &c, int &sc) {
  const bool sw = b < a;
  const float lo = sw ? b : a, hi = sw ? a : b;
  const int slo = sw ? sb : sa, shi = sw ? sa : sb;
  const bool below = v < lo, above = v > hi;  // both false for NaN: c = NaN
  c = below ? lo : (above ? hi : v);
  sc = below ? slo : (above ? shi : sv);
}

// Offer pin (x, y) = net-local `self` the two segments of step t; a pin in the
// tree (or padding) carries x = NaN and never takes one.  Branch-free: the
// updates are selects.  Without kSrc (the estimation) the clamps are a max
// and a min: the same value as the compare form up to the sign of a zero,
// which no output depends on (pieces are absolute differences, keys compare
// -0 equal to +0); with kSrc (the gradient) the compare form also gives the
// pin each clamped coordinate is copied from.
template <bool kSrc>
__device__ __forceinline__ void sph_relax(float x, float y, int self, Near &n, const Join &J, int t) {
  float c;
  int sc = 0;
  if constexpr (kSrc) {
    clamp_src(x, self, J.qx, J.sqx, J.xj, J.j, c, sc);  // segment 2t-1: y = qy, x from qx to x_j
  } else {
    c = fminf(fmaxf(x, fminf(J.qx, J.xj)), fmaxf(J.qx, J.xj));
  }
  const float d1 = fabsf(x - c) + fabsf(y - J.qy);
  const bool b1 = d1 < n.d;
  n.d = b1 ? d1 : n.d;
  n.seg = b1 ? 2 * t - 1 : n.seg;
  n.qx = b1 ? c : n.qx;
  n.qy = b1 ? J.qy : n.qy;
  if constexpr (kSrc) {
    n.sqx = b1 ? sc : n.sqx;
    n.sqy = b1 ? J.sqy : n.sqy;
    clamp_src(y, self, J.qy, J.sqy, J.yj, J.j, c, sc);  // segment 2t: x = x_j, y from qy to y_j
  } else {
    c = fminf(fmaxf(y, fminf(J.qy, J.yj)), fmaxf(J.qy, J.yj));
  }
  const float d2 = fabsf(x - J.xj) + fabsf(y - c);
  const bool b2 = d2 < n.d;
  n.d = b2 ? d2 : n.d;
  n.seg = b2 ? 2 * t : n.seg;
  n.qx = b2 ? J.xj : n.qx;
  n.qy = b2 ? c : n.qy;
  if constexpr (kSrc) {
    n.sqx = b2 ? J.j : n.sqx;
    n.sqy = b2 ? sc : n.sqy;
  }
}

// A block barrier that orders LDS only: the join loop exchanges its winners
// through LDS, while its global stores (each step's record for the numbering)
// are read only after a full __syncthreads, so a step need not wait for them.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int G>
__device__ __forceinline__ uint32_t group_min(uint32_t v) {
  if constexpr (G == kWave) {
    return wave_min(v);
  } else {
#pragma unroll
    for (int m = 1; m < G; m <<= 1) v = min(v, (uint32_t)__shfl_xor((int)v, m, G));
    return v;
  }
}

template <int G>
__device__ __forceinline__ int group_incl_scan(int v) {
  const int lane = (int)(threadIdx.x % G);
#pragma unroll
  for (int o = 1; o < G; o <<= 1) {
    const int y = __shfl_up(v, o, G);
    v += lane >= o ? y : 0;
  }
  return v;
}

// Fixed-point exponent for terms of magnitude up to m: a pin receives at most
// 2 (3 kEstMaxPins) < 2^17 terms, so 2^e m 2^17 stays below 2^62.
__device__ __forceinline__ int fix_exp(double m) { return m > 0.0 ? 44 - ilogb(m) : 0; }

__device__ __forceinline__ long long to_fixed(double v, int e) { return __double2ll_rn(ldexp(v, e)); }

__device__ __forceinline__ double sgn_d(float v) { return v > 0.0f ? 1.0 : (v < 0.0f ? -1.0 : 0.0); }

// One net of at most G pins, a pin per lane of its group (G = 8: eight nets
// per wavefront; G = 64: one).  Nets come from list[0 .. *count) or, with no
// list, every net of at most G pins (the rest are skipped).
template <int G, bool kGrad>
__global__ __launch_bounds__(256) void k_est_group(EstArgs A, const int32_t *list, const uint32_t *count) {
  constexpr int NG = 256 / G;
  __shared__ float s_qx[NG][G], s_qy[NG][G], s_key[NG][G];
  __shared__ int32_t s_rec[NG][G];                             // segment | pin << 16, by step
  __shared__ uint32_t s_src[kGrad ? NG : 1][kGrad ? G : 1];    // source pins of q (x | y << 16), by step
  __shared__ unsigned long long s_acc[kGrad ? NG : 1][kGrad ? 2 * G : 1];
  const int grp = (int)(threadIdx.x / G), lane = (int)(threadIdx.x % G);
  const int w = (int)blockIdx.x * NG + grp;
  int n;
  if (list) {
    if (w >= (int)*count) return;
    n = list[w];
  } else {
    if (w >= A.n_nets) return;
    n = w;
  }
  const int s0 = A.sink_ptr[n], k = A.sink_ptr[n + 1] - s0;
  if (k + 1 > G) return;  // the whole group leaves together
  const int64_t base = (int64_t)n + 3 * (int64_t)s0;
  const bool valid = lane <= k;
  const int drv = A.driver[n];
  const int pin = (lane >= 1 && valid) ? A.sink_pin[s0 + lane - 1] : drv;
  const float px = A.x[pin], py = A.y[pin];  // this lane's pin (the driver for lane 0 and padding)
  const float x0 = A.x[drv], y0 = A.y[drv];
  const float kNaN = __builtin_nanf("");
  const bool live0 = valid && lane > 0;
  float x = live0 ? px : kNaN, y = live0 ? py : kNaN;
  Near nr{live0 ? manhattan(px, py, x0, y0) : kFar, x0, y0, 0, 0, 0};
  for (int t = 1; t <= k; ++t) {
    const uint32_t kmin = group_min<G>(key_of(nr.d));
    const int j = (int)group_min<G>(key_of(nr.d) == kmin ? (uint32_t)lane : kNone);
    Join J;
    J.qx = __shfl(nr.qx, j, G);
    J.qy = __shfl(nr.qy, j, G);
    J.sqx = __shfl(nr.sqx, j, G);
    J.sqy = __shfl(nr.sqy, j, G);
    J.xj = __shfl(px, j, G);
    J.yj = __shfl(py, j, G);
    J.j = j;
    if (lane == j) {
      s_qx[grp][t] = nr.qx;
      s_qy[grp][t] = nr.qy;
      s_rec[grp][t] = nr.seg | (j << 16);
      if constexpr (kGrad) s_src[grp][t] = (uint32_t)nr.sqx | ((uint32_t)nr.sqy << 16);
      x = kNaN;
      nr.d = kFar;
    } else {
      sph_relax<kGrad>(x, y, lane, nr, J, t);
    }
  }
  wave_sync();
  // ---- numbering: lane t handles step t
  const int t = lane;
  const bool act = t >= 1 && t <= k;
  const int rec = act ? s_rec[grp][t] : 0;
  // every step wrote its record; the clamps only keep each index in range
  const int sg = min(rec & 0xffff, max(2 * (t - 1), 0)), jt = act ? min(max(rec >> 16, 1), k) : 0;
  const float qx = act ? s_qx[grp][t] : 0.0f, qy = act ? s_qy[grp][t] : 0.0f;
  const float xj = __shfl(px, jt, G), yj = __shfl(py, jt, G);
  const int sc = (sg + 1) >> 1;  // the step that made segment sg (sg >= 1)
  const bool axy = sg != 0 && (sg & 1) == 0;
  const int js = sg != 0 ? min(s_rec[grp][sc] >> 16, k) : 0;
  const float pxs = __shfl(px, js, G), pys = __shfl(py, js, G);
  const float c0 = sg == 0 ? x0 : (axy ? s_qy[grp][sc] : s_qx[grp][sc]);  // start of segment sg along its axis
  const float cend = sg == 0 ? x0 : (axy ? pys : pxs);
  const float dir = cend < c0 ? -1.0f : 1.0f;
  const float c = axy ? qy : qx;  // S_t along its segment's axis
  const float key = dir * c;      // exact: distance order from the start
  const float dirA = xj < qx ? -1.0f : 1.0f, dirB = yj < qy ? -1.0f : 1.0f;
  if (act) s_key[grp][t] = key;
  wave_sync();
  int rank = 0, m0 = 0, mA = 0, mB = 0, predt = 0, bestAt = 0, bestBt = 0;
  float predk = 0.0f, bestA = 0.0f, bestB = 0.0f;
  for (int u = 1; u <= k; ++u) {  // ascending steps: ties in key go to the later step
    const int su = s_rec[grp][u] & 0xffff;
    const float ku = s_key[grp][u];
    m0 += su == 0 ? 1 : 0;
    if (su == sg && (ku < key || (ku == key && u < t))) {
      if (rank == 0 || ku >= predk) {
        predk = ku;
        predt = u;
      }
      ++rank;
    }
    if (su == 2 * t - 1) {
      if (mA == 0 || ku >= bestA) {
        bestA = ku;
        bestAt = u;
      }
      ++mA;
    }
    if (su == 2 * t && t > 0) {
      if (mB == 0 || ku >= bestB) {
        bestB = ku;
        bestBt = u;
      }
      ++mB;
    }
  }
  const int wv = act ? mA + mB + 2 : 0;
  const int W = group_incl_scan<G>(wv);
  const int offA = m0 + 1 + W - wv;  // first node of segment 2t-1
  const int idxK = offA + mA;        // K_t closes segment 2t-1
  const int idxJ = idxK + 1 + mB;    // J_t closes segment 2t
  const int offA_s = __shfl(offA, sc, G), idxK_s = __shfl(idxK, sc, G);
  const int offsg = sg == 0 ? 0 : ((sg & 1) ? offA_s : idxK_s + 1);
  const int idxS = offsg + (sg == 0 ? 1 : 0) + rank;
  const int idxS_s = __shfl(idxS, sc, G);
  const int pS = rank > 0 ? idxS - 1 : (sg == 0 ? 0 : ((sg & 1) ? idxS_s : idxK_s));
  const int pK = mA > 0 ? idxK - 1 : idxS;
  const int pJ = mB > 0 ? idxJ - 1 : idxK;
  const float cpS = rank > 0 ? dir * predk : c0;
  const float cpK = mA > 0 ? dirA * bestA : qx;
  const float cpJ = mB > 0 ? dirB * bestB : qy;
  const float LS = fabsf(c - cpS), LK = fabsf(xj - cpK), LJ = fabsf(yj - cpJ);
  const float ra = axy ? A.ry : A.rx, ca = axy ? A.cy : A.cx;
  const bool inr = act && idxS >= 1 && idxK >= 1 && idxJ <= 3 * k && idxS <= 3 * k && idxK <= 3 * k;
  if constexpr (!kGrad) {
    if (inr) {
      A.parent[base + idxS] = pS;
      A.res[base + idxS] = ra * LS;
      A.cap[base + idxS] = ca * LS;
      A.parent[base + idxK] = pK;
      A.res[base + idxK] = A.rx * LK;
      A.cap[base + idxK] = A.cx * LK;
      A.parent[base + idxJ] = pJ;
      A.res[base + idxJ] = A.ry * LJ;
      A.cap[base + idxJ] = A.cy * LJ;
      A.sink_node[s0 + jt - 1] = idxJ;
    }
    if (lane == 0) {
      A.parent[base] = -1;
      A.res[base] = 0.0f;
      A.cap[base] = 0.0f;
      A.node_ptr[n + 1] = base + 3 * (int64_t)k + 1;
      if (n == 0) A.node_ptr[0] = 0;
    }
  } else {
    // the caller's trees must be these
    const bool bad = act && (!inr || A.g_parent[base + idxS] != pS || A.g_parent[base + idxK] != pK ||
                             A.g_parent[base + idxJ] != pJ || A.g_sink_node[s0 + jt - 1] != idxJ);
    if (bad) atomicMin(A.err, (uint32_t)n);
    // the pins bounding each piece along its axis
    const uint32_t my = act ? s_src[grp][t] : 0u;
    const int mx_ = (int)(my & 0xffff), my_ = (int)(my >> 16);
    const uint32_t pr = s_src[grp][rank > 0 ? predt : (sg == 0 ? 0 : sc)];
    const int uS = axy ? my_ : mx_;
    const int wS = sg == 0 ? 0 : (axy ? (int)(pr >> 16) : (int)(pr & 0xffff));
    const int wK = mA > 0 ? (int)(s_src[grp][bestAt] & 0xffff) : mx_;
    const int wJ = mB > 0 ? (int)(s_src[grp][bestBt] >> 16) : my_;
    double vS = 0.0, vK = 0.0, vJ = 0.0;
    if (inr) {
      vS = sgn_d(c - cpS) * ((double)ra * A.g_res[base + idxS] + (double)ca * A.g_cap[base + idxS]);
      vK = sgn_d(xj - cpK) * ((double)A.rx * A.g_res[base + idxK] + (double)A.cx * A.g_cap[base + idxK]);
      vJ = sgn_d(yj - cpJ) * ((double)A.ry * A.g_res[base + idxJ] + (double)A.cy * A.g_cap[base + idxJ]);
    }
    // largest term per axis over the net, as the bits of a non-negative float
    const float mxf = (float)fmax(axy ? 0.0 : fabs(vS), fabs(vK));
    const float myf = (float)fmax(axy ? fabs(vS) : 0.0, fabs(vJ));
    const uint32_t bx = kNone - group_min<G>(kNone - __float_as_uint(mxf));
    const uint32_t by = kNone - group_min<G>(kNone - __float_as_uint(myf));
    // rounding up to float only raises the exponent by at most one: still in range
    const int ex = fix_exp((double)__uint_as_float(bx)), ey = fix_exp((double)__uint_as_float(by));
    s_acc[grp][2 * lane] = 0ull;
    s_acc[grp][2 * lane + 1] = 0ull;
    wave_sync();
    if (inr) {
      const int eS = axy ? ey : ex, oS = axy ? 1 : 0;
      const long long iS = to_fixed(vS, eS), iK = to_fixed(vK, ex), iJ = to_fixed(vJ, ey);
      atomicAdd(&s_acc[grp][2 * uS + oS], (unsigned long long)iS);
      atomicAdd(&s_acc[grp][2 * wS + oS], (unsigned long long)(-iS));
      atomicAdd(&s_acc[grp][2 * jt], (unsigned long long)iK);
      atomicAdd(&s_acc[grp][2 * wK], (unsigned long long)(-iK));
      atomicAdd(&s_acc[grp][2 * jt + 1], (unsigned long long)iJ);
      atomicAdd(&s_acc[grp][2 * wJ + 1], (unsigned long long)(-iJ));
    }
    wave_sync();
    if (valid) {
      A.gx[pin] = (float)ldexp((double)(long long)s_acc[grp][2 * lane], -ex);
      A.gy[pin] = (float)ldexp((double)(long long)s_acc[grp][2 * lane + 1], -ey);
    }
  }
}

// Exclusive prefix of c over a 1024-thread block; *total gets the block's
// sum.  Every thread calls it; s_w (16 words) is free again on return.
__device__ __forceinline__ uint32_t block_excl_scan1024(uint32_t c, uint32_t *s_w, uint32_t *total) {
  const int lane = (int)(threadIdx.x & (kWave - 1)), wave = (int)(threadIdx.x / kWave);
  int v = (int)c;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(v, o, kWave);
    v += lane >= o ? y : 0;
  }
  if (lane == kWave - 1) s_w[wave] = (uint32_t)v;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 1024 / kWave; ++w) {
    off += w < wave ? s_w[w] : 0u;
    tot += s_w[w];
  }
  __syncthreads();
  *total = tot;
  return off + (uint32_t)v - c;
}

// One net of k_est_block with NL live register slots per thread (pin
// l = tid + 1024 u, u < NL); step t is handled by thread (t - 1) % 1024 once
// the joins are done.  LDS per step: its record (segment | pin), its key and
// later its wire offsets; the step's attach point, its counters and the
// results of the passes go to the net's region of the global scratch tmp (16
// words per step), so no per-step state stays in registers between phases.
// The steps of each wire are found through a list ordered by wire (counts by
// atomics, slots from the node offsets), so the passes cost O(k) plus the
// squares of the wires' S-point counts.
template <int NL, bool kGrad>
__device__ __forceinline__ void est_block_net(const EstArgs &A, int n, int s0, int k, int64_t base, int b,
                                              uint32_t (*s_key)[1024 / kWave], uint32_t (*s_idx)[1024 / kWave],
                                              float (*s_win)[1024 / kWave][8], int32_t *s_rec, float *s_k,
                                              uint32_t *s_off, uint32_t *s_w) {
  const int tid = (int)threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int drv = A.driver[n];
  const float x0 = A.x[drv], y0 = A.y[drv];
  const float kNaN = __builtin_nanf("");
  uint32_t *tmp = A.big_tmp + 16 * A.acc_off[b];  // 16 words per step t at 16 t; t = 0: net counters
  {
    // The candidates: position p = tid + 1024 u holds a pin outside the tree
    // (its index in s_off[p], ascending with p, so the lowest position among
    // equal distances is the lowest index), the first nl slots of each thread
    // in use; whenever the pins left fit one slot fewer they are packed again
    // in position order (through words 6-14 of the scratch), so the work per
    // step follows the pins left rather than the net.
    float x[NL], y[NL];
    Near nr[NL];
    int li[kGrad ? NL : 1];  // the gradient mode's clamps name the pins
    int nl = NL;
    float key = kFar;
    int ul = 0;
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int l = tid + u * 1024;  // pin index in the net: 0 driver, 1..k sinks
      const bool live = l >= 1 && l <= k;
      const int pin = A.sink_pin[s0 + (live ? l - 1 : 0)];
      if constexpr (kGrad) li[u] = l;
      s_off[l] = (uint32_t)l;
      x[u] = live ? A.x[pin] : kNaN;  // NaN: never nearer than anything
      y[u] = live ? A.y[pin] : kNaN;
      nr[u] = Near{live ? manhattan(x[u], y[u], x0, y0) : kFar, x0, y0, 0, 0, 0};
      const bool bt = nr[u].d < key;  // ascending position: the first minimum wins ties
      key = bt ? nr[u].d : key;
      ul = bt ? u : ul;
    }
    __syncthreads();
    for (int t = 1; t <= k; ++t) {
      const uint32_t wk = wave_min(key_of(key));
      const uint32_t wi = wave_min(key_of(key) == wk && key < kFar ? (uint32_t)(tid + ul * 1024) : kNone);
      const int buf = t & 1;
      // the wave's winner publishes its attach point and position
      if (wi != kNone && (int)(wi & 1023) == tid) {
        float wqx = 0.0f, wqy = 0.0f, wx = 0.0f, wy = 0.0f;
        int wsx = 0, wsy = 0, wsg = 0;
#pragma unroll
        for (int u = 0; u < NL; ++u) {
          const bool me = u == ul;
          wqx = me ? nr[u].qx : wqx;
          wqy = me ? nr[u].qy : wqy;
          if constexpr (kGrad) {
            wsx = me ? nr[u].sqx : wsx;
            wsy = me ? nr[u].sqy : wsy;
          }
          wsg = me ? nr[u].seg : wsg;
          wx = me ? x[u] : wx;
          wy = me ? y[u] : wy;
        }
        s_win[buf][wave][0] = wqx;
        s_win[buf][wave][1] = wqy;
        s_win[buf][wave][2] = wx;
        s_win[buf][wave][3] = wy;
        s_win[buf][wave][6] = __int_as_float(wsg);
        if constexpr (kGrad) {
          s_win[buf][wave][4] = __int_as_float(wsx);
          s_win[buf][wave][5] = __int_as_float(wsy);
        }
      }
      if (lane == 0) {
        s_key[buf][wave] = wk;
        s_idx[buf][wave] = wi;
      }
      lds_barrier();
      const int e = lane & (1024 / kWave - 1);
      const uint32_t ek = s_key[buf][e], ei = s_idx[buf][e];
      const uint32_t bk = row_min16(ek);
      const uint32_t bi = row_min16(ek == bk ? ei : kNone);
      const int jp = min(max((int)__builtin_amdgcn_readfirstlane((int)bi), 0), NL * 1024 - 1);  // a pin is left
      const int jw = (jp & 1023) / kWave, ju = jp >> 10;
      const int j = (int)s_off[jp];  // its index in the net
      Join J;
      J.qx = s_win[buf][jw][0];
      J.qy = s_win[buf][jw][1];
      J.xj = s_win[buf][jw][2];
      J.yj = s_win[buf][jw][3];
      J.sqx = kGrad ? __float_as_int(s_win[buf][jw][4]) : 0;
      J.sqy = kGrad ? __float_as_int(s_win[buf][jw][5]) : 0;
      J.j = j;
      if (tid == 0) {  // the step's record, from the winner's published state
        s_rec[t] = __float_as_int(s_win[buf][jw][6]) | (j << 16);
        tmp[16 * t] = __float_as_uint(J.qx);
        tmp[16 * t + 1] = __float_as_uint(J.qy);
        if constexpr (kGrad) A.step_src[s0 + t - 1] = (uint32_t)J.sqx | ((uint32_t)J.sqy << 16);
      }
      key = kFar;
      ul = 0;
      const bool mine = tid == (jp & 1023);
#pragma unroll
      for (int u = 0; u < NL; ++u) {
        if (u < nl) {  // uniform: the slots in use
          const bool out = mine && u == ju;  // the joining pin leaves the candidates
          x[u] = out ? kNaN : x[u];
          nr[u].d = out ? kFar : nr[u].d;
          sph_relax<kGrad>(x[u], y[u], kGrad ? li[kGrad ? u : 0] : 0, nr[u], J, t);
          const bool bt = nr[u].d < key;
          key = bt ? nr[u].d : key;
          ul = bt ? u : ul;
        }
      }
      if (nl > 1 && k - t <= (nl - 1) * 1024) {  // uniform: pack the pins left into nl - 1 slots
        __syncthreads();  // the step's reads of s_off and s_win are done
        uint32_t carry = 0;
#pragma unroll
        for (int u = 0; u < NL; ++u) {
          if (u < nl) {
            const bool live = x[u] == x[u];  // not NaN
            uint32_t tot;
            const uint32_t pos = carry + block_excl_scan1024(live ? 1u : 0u, s_w, &tot);
            carry += tot;
            if (live) {
              uint32_t *o = tmp + 16 * (pos + 1) + 6;
              o[0] = __float_as_uint(x[u]);
              o[1] = __float_as_uint(y[u]);
              o[2] = __float_as_uint(nr[u].d);
              o[3] = __float_as_uint(nr[u].qx);
              o[4] = __float_as_uint(nr[u].qy);
              o[5] = (uint32_t)nr[u].seg;
              o[6] = s_off[tid + u * 1024];
              if constexpr (kGrad) {
                o[7] = (uint32_t)nr[u].sqx;
                o[8] = (uint32_t)nr[u].sqy;
              }
            }
          }
        }
        __syncthreads();  // every pin written (and every old index read)
        --nl;
        key = kFar;
        ul = 0;
#pragma unroll
        for (int u = 0; u < NL; ++u) {
          const int pos = tid + u * 1024;
          const bool live = u < nl && pos < k - t;
          const uint32_t *o = tmp + 16 * (min(pos, max(k - t - 1, 0)) + 1) + 6;  // in the net's region
          x[u] = live ? __uint_as_float(o[0]) : kNaN;
          y[u] = live ? __uint_as_float(o[1]) : kNaN;
          nr[u].d = live ? __uint_as_float(o[2]) : kFar;
          nr[u].qx = live ? __uint_as_float(o[3]) : 0.0f;
          nr[u].qy = live ? __uint_as_float(o[4]) : 0.0f;
          nr[u].seg = live ? (int)o[5] : 0;
          if (u < nl) s_off[pos] = live ? o[6] : 0u;
          if constexpr (kGrad) {
            li[u] = live ? (int)o[6] : 0;
            nr[u].sqx = live ? (int)o[7] : 0;
            nr[u].sqy = live ? (int)o[8] : 0;
          }
          const bool bt = nr[u].d < key;
          key = bt ? nr[u].d : key;
          ul = bt ? u : ul;
        }
        __syncthreads();  // the new indices in place
      }
    }
  }
  __syncthreads();  // every step recorded (LDS, and its point in tmp)
  auto pos_of = [&](int l, float &px, float &py) {
    const int p = l == 0 ? drv : A.sink_pin[s0 + l - 1];
    px = A.x[p];
    py = A.y[p];
  };
  // the record of step t, its clamps only keeping every index in range
  auto seg_of = [&](int t) { return min(s_rec[t] & 0xffff, 2 * (t - 1)); };
  auto pin_of = [&](int t) { return min(max(s_rec[t] >> 16, 1), k); };
  // ---- pass 1: each step's key (distance order on its wire: dir * coordinate),
  // and the step's counters cleared
  if (tid == 0) {
    tmp[4] = 0u;  // S points on wire 0
    tmp[5] = 0u;  // their fill counter
  }
  for (int t = tid + 1; t <= k; t += 1024) {
    const int sg = seg_of(t), sc = (sg + 1) >> 1;
    const bool axy = sg != 0 && (sg & 1) == 0;
    float c0 = x0, cend = x0;
    if (sg != 0) {
      float pxs, pys;
      pos_of(pin_of(sc), pxs, pys);
      c0 = __uint_as_float(tmp[16 * sc + (axy ? 1 : 0)]);
      cend = axy ? pys : pxs;
    }
    const float dir = cend < c0 ? -1.0f : 1.0f;
    s_k[t] = dir * __uint_as_float(tmp[16 * t + (axy ? 1 : 0)]);
    tmp[16 * t + 2] = __float_as_uint(c0);  // the step's own words: read back only by this step
    tmp[16 * t + 3] = __float_as_uint(dir);
#pragma unroll
    for (int w = 4; w < 10; ++w) tmp[16 * t + w] = 0u;
  }
  __syncthreads();
  // ---- pass 2: every S point reports to the step whose wire it lies on: a
  // count per wire and its last point (the largest key, ties to the later
  // step: an atomic maximum of the orderable key bits and the step)
  auto owner_word = [&](int sg, int w) -> uint32_t * { return tmp + 16 * ((sg + 1) >> 1) + w; };
  for (int t = tid + 1; t <= k; t += 1024) {
    const int sg = seg_of(t);
    if (sg == 0) {
      atomicAdd(tmp + 4, 1u);
      continue;
    }
    atomicAdd(owner_word(sg, 4), (sg & 1) ? 1u : 0x10000u);
    const uint32_t bits = __float_as_uint(s_k[t] + 0.0f);  // -0 reads as +0
    const uint32_t ok = (bits & 0x80000000u) ? ~bits : bits | 0x80000000u;
    atomicMax(reinterpret_cast<unsigned long long *>(owner_word(sg, (sg & 1) ? 6 : 8)),
              ((unsigned long long)ok << 32) | (unsigned long long)t);
  }
  __syncthreads();
  // ---- offsets: an exclusive prefix over steps of (S points on 2t-1 and 2t) + 2
  uint32_t carry = tmp[4] + 1u;
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int t = tid + 1 + u * 1024;
    const uint32_t cnt = t <= k ? tmp[16 * t + 4] : 0u;
    const uint32_t wv = t <= k ? (cnt & 0xffffu) + (cnt >> 16) + 2u : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan1024(wv, s_w, &tot);
    if (t <= k) s_off[t] = carry + ex;  // offset of wire 2t-1
    carry += tot;
  }
  __syncthreads();
  // first node of wire w, its S-point count, and its first slot in the list
  // of S points ordered by wire (the S points on earlier wires: off(w) - w)
  auto wire_off = [&](int w) -> int {
    if (w == 0) return 0;
    const int sc = (w + 1) >> 1;
    return (w & 1) ? (int)s_off[sc] : (int)s_off[sc] + (int)(tmp[16 * sc + 4] & 0xffffu) + 1;
  };
  auto wire_count = [&](int w) -> int {
    if (w == 0) return (int)tmp[4];
    const uint32_t cnt = tmp[16 * ((w + 1) >> 1) + 4];
    return (int)((w & 1) ? (cnt & 0xffffu) : (cnt >> 16));
  };
  // ---- pass 3: the S points into their wires' slots (list at word 10 of slot + 1)
  for (int t = tid + 1; t <= k; t += 1024) {
    const int sg = seg_of(t);
    uint32_t pos;
    if (sg == 0)
      pos = atomicAdd(tmp + 5, 1u);
    else
      pos = (atomicAdd(owner_word(sg, 5), (sg & 1) ? 1u : 0x10000u) >> ((sg & 1) ? 0 : 16)) & 0xffffu;
    const int slot = wire_off(sg) - sg + (int)pos;
    if (slot >= 0 && slot < k) tmp[16 * (slot + 1) + 10] = (uint32_t)t;
  }
  __syncthreads();
  // ---- pass 4: rank on the own wire (and the predecessor) from the wire's
  // slots; then the signed pieces (child minus parent coordinate) of S_t, K_t
  // and J_t
  for (int t = tid + 1; t <= k; t += 1024) {
    const int sg = seg_of(t), sc = (sg + 1) >> 1;
    const bool axy = sg != 0 && (sg & 1) == 0;
    const float kt = s_k[t];
    const int first = wire_off(sg) - sg, m = wire_count(sg);
    int rk = 0, pt = 0;
    float pk = 0.0f;
    for (int i = 0; i < m; ++i) {
      const int slot = first + i;
      const int v = (slot >= 0 && slot < k) ? min(max((int)tmp[16 * (slot + 1) + 10], 1), k) : t;
      const float kv = s_k[v];
      if (kv < kt || (kv == kt && v < t)) {
        if (rk == 0 || kv > pk || (kv == pk && v > pt)) {
          pk = kv;
          pt = v;
        }
        ++rk;
      }
    }
    const uint32_t cnt = tmp[16 * t + 4];
    const int ma = (int)(cnt & 0xffffu), mb = (int)(cnt >> 16);
    const int at = ma > 0 ? min(max((int)(uint32_t)*reinterpret_cast<unsigned long long *>(tmp + 16 * t + 6), 1), k) : 0;
    const int bt = mb > 0 ? min(max((int)(uint32_t)*reinterpret_cast<unsigned long long *>(tmp + 16 * t + 8), 1), k) : 0;
    const float qx = __uint_as_float(tmp[16 * t]), qy = __uint_as_float(tmp[16 * t + 1]);
    const float c0 = __uint_as_float(tmp[16 * t + 2]), dir = __uint_as_float(tmp[16 * t + 3]);
    const float c = axy ? qy : qx;
    float xj, yj;
    pos_of(pin_of(t), xj, yj);
    const float dirA = xj < qx ? -1.0f : 1.0f, dirB = yj < qy ? -1.0f : 1.0f;
    const float cpS = rk > 0 ? dir * pk : c0;
    const float cpK = ma > 0 ? dirA * s_k[at] : qx;
    const float cpJ = mb > 0 ? dirB * s_k[bt] : qy;
    if constexpr (kGrad) {  // the pins bounding the pieces along their axes
      const uint32_t my = A.step_src[s0 + t - 1];
      const int mx_ = (int)(my & 0xffff), my_ = (int)(my >> 16);
      const uint32_t pr = rk > 0 ? A.step_src[s0 + pt - 1] : (sg == 0 ? 0u : A.step_src[s0 + sc - 1]);
      const int uS = axy ? my_ : mx_;
      const int wS = sg == 0 ? 0 : (axy ? (int)(pr >> 16) : (int)(pr & 0xffff));
      const int wK = ma > 0 ? (int)(A.step_src[s0 + at - 1] & 0xffff) : mx_;
      const int wJ = mb > 0 ? (int)(A.step_src[s0 + bt - 1] >> 16) : my_;
      tmp[16 * t + 11] = (uint32_t)uS | (axy ? 0x8000u : 0u) | ((uint32_t)wS << 16);  // bit 15: S term to y
      tmp[16 * t + 12] = (uint32_t)wK | ((uint32_t)wJ << 16);
    }
    // the step's own words 0-3, read above; others read word 3 only after the next barrier
    tmp[16 * t] = __float_as_uint(c - cpS);
    tmp[16 * t + 1] = __float_as_uint(xj - cpK);
    tmp[16 * t + 2] = __float_as_uint(yj - cpJ);
    tmp[16 * t + 3] = (uint32_t)rk;
  }
  __syncthreads();
  // ---- the nodes
  auto idx_s = [&](int t) {  // node of S_t
    const int sg = seg_of(t);
    return wire_off(sg) + (sg == 0 ? 1 : 0) + (int)tmp[16 * t + 3];
  };
  // node indices, parents and pieces of step t (S_t, K_t, J_t)
  auto nodes_of = [&](int t, int &iS, int &iK, int &iJ, int &pS, int &pK, int &pJ) {
    const int sg = seg_of(t), sc = (sg + 1) >> 1;
    const uint32_t cnt = tmp[16 * t + 4];
    const int rk = (int)tmp[16 * t + 3], ma = (int)(cnt & 0xffffu), mb = (int)(cnt >> 16);
    iS = idx_s(t);
    iK = (int)s_off[t] + ma;
    iJ = iK + 1 + mb;
    pS = rk > 0 ? iS - 1 : (sg == 0 ? 0 : ((sg & 1) ? idx_s(sc) : (int)s_off[sc] + (int)(tmp[16 * sc + 4] & 0xffffu)));
    pK = ma > 0 ? iK - 1 : iS;
    pJ = mb > 0 ? iJ - 1 : iK;
    return iS >= 1 && iS <= 3 * k && iK >= 1 && iK <= 3 * k && iJ <= 3 * k;
  };
  // the three terms of step t in the gradient mode
  auto terms_of = [&](int t, int iS, int iK, int iJ, double &vS, double &vK, double &vJ) {
    const int sg = seg_of(t);
    const bool axy = sg != 0 && (sg & 1) == 0;
    const float ra = axy ? A.ry : A.rx, ca = axy ? A.cy : A.cx;
    vS = sgn_d(__uint_as_float(tmp[16 * t])) * ((double)ra * A.g_res[base + iS] + (double)ca * A.g_cap[base + iS]);
    vK = sgn_d(__uint_as_float(tmp[16 * t + 1])) * ((double)A.rx * A.g_res[base + iK] + (double)A.cx * A.g_cap[base + iK]);
    vJ = sgn_d(__uint_as_float(tmp[16 * t + 2])) * ((double)A.ry * A.g_res[base + iJ] + (double)A.cy * A.g_cap[base + iJ]);
    return axy;
  };
  double mxd = 0.0, myd = 0.0;
  for (int t = tid + 1; t <= k; t += 1024) {
    int iS, iK, iJ, pS, pK, pJ;
    if (!nodes_of(t, iS, iK, iJ, pS, pK, pJ)) {
      if constexpr (kGrad) atomicMin(A.err, (uint32_t)n);
      continue;
    }
    const int jt = pin_of(t);
    if constexpr (!kGrad) {
      const int sg = seg_of(t);
      const bool axy = sg != 0 && (sg & 1) == 0;
      const float ra = axy ? A.ry : A.rx, ca = axy ? A.cy : A.cx;
      const float LS = fabsf(__uint_as_float(tmp[16 * t])), LK = fabsf(__uint_as_float(tmp[16 * t + 1])),
                  LJ = fabsf(__uint_as_float(tmp[16 * t + 2]));
      A.parent[base + iS] = pS;
      A.res[base + iS] = ra * LS;
      A.cap[base + iS] = ca * LS;
      A.parent[base + iK] = pK;
      A.res[base + iK] = A.rx * LK;
      A.cap[base + iK] = A.cx * LK;
      A.parent[base + iJ] = pJ;
      A.res[base + iJ] = A.ry * LJ;
      A.cap[base + iJ] = A.cy * LJ;
      A.sink_node[s0 + jt - 1] = iJ;
    } else {
      const bool bad = A.g_parent[base + iS] != pS || A.g_parent[base + iK] != pK || A.g_parent[base + iJ] != pJ ||
                       A.g_sink_node[s0 + jt - 1] != iJ;
      if (bad) atomicMin(A.err, (uint32_t)n);
      double vS, vK, vJ;
      if (terms_of(t, iS, iK, iJ, vS, vK, vJ))
        myd = fmax(myd, fabs(vS));
      else
        mxd = fmax(mxd, fabs(vS));
      mxd = fmax(mxd, fabs(vK));
      myd = fmax(myd, fabs(vJ));
    }
  }
  if constexpr (!kGrad) {
    if (tid == 0) {
      A.parent[base] = -1;
      A.res[base] = 0.0f;
      A.cap[base] = 0.0f;
      A.node_ptr[n + 1] = base + 3 * (int64_t)k + 1;
      if (n == 0) A.node_ptr[0] = 0;
    }
  } else {
    // per-net exponents from the largest term per axis (as the bits of
    // non-negative floats: rounding up to float raises the exponent by at
    // most one, still in range)
    const uint32_t wx = kNone - wave_min(kNone - __float_as_uint((float)mxd));
    const uint32_t wy = kNone - wave_min(kNone - __float_as_uint((float)myd));
    __syncthreads();  // s_w free (the offsets scan is done)
    if (lane == 0) {
      s_w[wave] = wx;
      s_w[16 + wave] = wy;
    }
    __syncthreads();
    uint32_t bx = 0, by = 0;
#pragma unroll
    for (int v = 0; v < 1024 / kWave; ++v) {
      bx = max(bx, s_w[v]);
      by = max(by, s_w[16 + v]);
    }
    const int ex = fix_exp((double)__uint_as_float(bx)), ey = fix_exp((double)__uint_as_float(by));
    unsigned long long *acc = A.acc + 2 * A.acc_off[b];
    for (int t = tid + 1; t <= k; t += 1024) {
      int iS, iK, iJ, pS, pK, pJ;
      if (!nodes_of(t, iS, iK, iJ, pS, pK, pJ)) continue;
      double vS, vK, vJ;
      terms_of(t, iS, iK, iJ, vS, vK, vJ);
      const uint32_t w0 = tmp[16 * t + 11], w1 = tmp[16 * t + 12];
      const int oS = (w0 >> 15) & 1, us = (int)(w0 & 0x7fff), ws = (int)(w0 >> 16);
      const int wk = (int)(w1 & 0xffff), wj = (int)(w1 >> 16);
      const long long is = to_fixed(vS, oS ? ey : ex), ik = to_fixed(vK, ex), ij = to_fixed(vJ, ey);
      const int jt = pin_of(t);
      atomicAdd(acc + 2 * us + oS, (unsigned long long)is);
      atomicAdd(acc + 2 * ws + oS, (unsigned long long)(-is));
      atomicAdd(acc + 2 * jt, (unsigned long long)ik);
      atomicAdd(acc + 2 * wk, (unsigned long long)(-ik));
      atomicAdd(acc + 2 * jt + 1, (unsigned long long)ij);
      atomicAdd(acc + 2 * wj + 1, (unsigned long long)(-ij));
    }
    __threadfence();
    __syncthreads();
    for (int l = tid; l <= k; l += 1024) {
      const int p = l == 0 ? drv : A.sink_pin[s0 + l - 1];
      const long long sx = (long long)__hip_atomic_load(acc + 2 * l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const long long sy = (long long)__hip_atomic_load(acc + 2 * l + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      A.gx[p] = (float)ldexp((double)sx, -ex);
      A.gy[p] = (float)ldexp((double)sy, -ey);
    }
  }
}

// Picks the register-slot count NL of a net of k_est_block (pins 0..k over
// 1024 threads) among kLo..kHi.
template <bool kGrad, int NL, int kHi>
__device__ __forceinline__ void est_block_dispatch(int nl, const EstArgs &A, int n, int s0, int k, int64_t base, int b,
                                                   uint32_t (*s_key)[1024 / kWave], uint32_t (*s_idx)[1024 / kWave],
                                                   float (*s_win)[1024 / kWave][8], int32_t *s_rec, float *s_k,
                                                   uint32_t *s_off, uint32_t *s_w) {
  if constexpr (NL <= kHi) {
    if (nl == NL)
      est_block_net<NL, kGrad>(A, n, s0, k, base, b, s_key, s_idx, s_win, s_rec, s_k, s_off, s_w);
    else
      est_block_dispatch<kGrad, NL + 1, kHi>(nl, A, n, s0, k, base, b, s_key, s_idx, s_win, s_rec, s_k, s_off,
                                             s_w);
  }
}

// One block per net of list[0 .. *count) whose slot count lies in kLo..kHi,
// looping over the list with a fixed grid.  Separate kernels per slot range
// keep the register allocation of the small nets free of the large ones'.
template <bool kGrad, int kLo, int kHi>
__global__ __launch_bounds__(1024) void k_est_block(EstArgs A, const int32_t *list, const uint32_t *count) {
  __shared__ uint32_t s_key[2][1024 / kWave];
  __shared__ uint32_t s_idx[2][1024 / kWave];
  __shared__ float s_win[2][1024 / kWave][8];
  __shared__ uint32_t s_w[2 * (1024 / kWave)];
  __shared__ int32_t s_rec[kEstMaxPins];
  __shared__ float s_k[kEstMaxPins];
  __shared__ uint32_t s_off[kEstMaxPins];
  const int nb = (int)*count;
  for (int b = (int)blockIdx.x; b < nb; b += (int)gridDim.x) {
    const int n = list[b];
    const int s0 = A.sink_ptr[n], k = A.sink_ptr[n + 1] - s0;
    const int nl = (k >> 10) + 1;  // more than kEstMaxPins pins: refused by the host before launch
    if (nl < kLo || nl > kHi) continue;
    const int64_t base = (int64_t)n + 3 * (int64_t)s0;
    est_block_dispatch<kGrad, kLo, kHi>(nl, A, n, s0, k, base, b, s_key, s_idx, s_win, s_rec, s_k, s_off, s_w);
    __syncthreads();  // the next net reuses the buffers
  }
}

// The accumulator offsets of the gradient mode's large nets: off[b] = the
// pins of big[0 .. b), *total their sum (one thread; the list is short).
__global__ void k_est_acc_offsets(const EstArgs A, const int32_t *big, const uint32_t *count, int64_t *off,
                                  unsigned long long *total) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int64_t s = 0;
  for (int b = 0; b < (int)*count; ++b) {
    const int n = big[b];
    off[b] = s;
    s += (int64_t)(A.sink_ptr[n + 1] - A.sink_ptr[n]) + 1;
  }
  *total = (unsigned long long)s;
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

template <bool kGrad>
static hipError_t launch_tiers(const EstArgs &A, const int32_t *mid, const int32_t *big, const uint32_t *st,
                               uint32_t n_mid, uint32_t n_big, hipStream_t s, hipStream_t side) {
  if (A.n_nets <= 0) return hipSuccess;
  if (n_big > 0) {  // first: the longest blocks start before the short work fills the chip
    const dim3 grid(std::min<uint32_t>(n_big, 4096u));
    hipLaunchKernelGGL((k_est_block<kGrad, 1, kEstPer>), grid, dim3(1024), 0, s, A, big, st + 1);
  }
  hipStream_t t = side ? side : s;  // the tiers write other nets than the block kernel
  if (n_mid > 0)
    hipLaunchKernelGGL((k_est_group<kWave, kGrad>), dim3(blocks_of(n_mid, 256 / kWave)), dim3(256), 0, t, A, mid,
                       st);
  hipLaunchKernelGGL((k_est_group<kLanePins, kGrad>), dim3(blocks_of(A.n_nets, 256 / kLanePins)), dim3(256), 0, t,
                     A, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_est(const EstArgs &A, const int32_t *mid, const int32_t *big, const uint32_t *st, uint32_t n_mid,
                      uint32_t n_big, hipStream_t s, hipStream_t side) {
  return launch_tiers<false>(A, mid, big, st, n_mid, n_big, s, side);
}

hipError_t launch_est_acc_offsets(const EstArgs &A, const int32_t *big, const uint32_t *st, int64_t *off,
                                  unsigned long long *total, hipStream_t s) {
  hipLaunchKernelGGL(k_est_acc_offsets, dim3(1), dim3(64), 0, s, A, big, st + 1, off, total);
  return hipGetLastError();
}

hipError_t launch_est_grad(const EstArgs &A, const int32_t *mid, const int32_t *big, const uint32_t *st,
                           uint32_t n_mid, uint32_t n_big, hipStream_t s, hipStream_t side) {
  return launch_tiers<true>(A, mid, big, st, n_mid, n_big, s, side);
}

}  // namespace sta
