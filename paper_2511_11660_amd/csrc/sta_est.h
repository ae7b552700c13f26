// Internal interface of the RC estimator (sta_rc_estimate.hip), shared with
// the host entry point.  Kept apart from the timing kernels' header.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace sta {

// RC estimation from pin positions (sta_rc_estimate.hip)
constexpr int kEstMaxPins = 12288;  // largest net (driver + sinks) the estimator takes
struct EstArgs {
  int n_nets;
  const int32_t *driver, *sink_ptr, *sink_pin;  // caller net CSR
  const float *x, *y;                           // [n_pins] positions (um)
  float rx, ry, cx, cy;                         // kOhm / um and fF / um along x, y
  int64_t *node_ptr;                            // outputs: RC CSR of every net
  int32_t *parent;
  float *res, *cap;
  int32_t *sink_node;
  uint32_t *big_tmp;        // nets above 64 pins: 16 words per pin, at 16 acc_off[b] for big-list entry b
  const int64_t *acc_off;   // pins of the big-list entries before b
  // gradient mode (the trees rebuilt, checked and differentiated)
  const int32_t *g_parent, *g_sink_node;  // the caller's trees (net n at node n + 3 sink_ptr[n])
  const float *g_res, *g_cap;             // dJ/dR, dJ/dC per node
  float *gx, *gy;                         // [n_pins] outputs (pins on no net untouched)
  uint32_t *step_src;                     // [n_sinks] scratch: source pins of each step's attach point
  uint32_t *err;                          // lowest net whose tree differs from the caller's (~0 when none)
  unsigned long long *acc;                // integer accumulators of the nets above 64 pins (2 per pin)
};
// st[6] (caller-initialized to {0, 0, 0, ~0, ~0, ~0}): nets of 9..64 pins,
// nets above 64 pins, their largest sink count, first bad net, first bad sink
// entry, first pin position not finite or beyond 1e18 in magnitude.  The mid
// and big lists receive at most mid_cap and big_cap entries (the counts go on
// counting); by default they are as long as there are nets.
hipError_t launch_est_check(const EstArgs &A, int n_pins, int n_sinks, int32_t *mid, int32_t *big, uint32_t *st,
                            hipStream_t s, uint32_t mid_cap = UINT32_MAX, uint32_t big_cap = UINT32_MAX);

// Scratch of the allocation-free entry point: 256 bytes of check words, then
// kEstNoallocMid mid-list entries, kEstNoallocBig big-list entries, their
// kEstNoallocBig pin offsets (int64), and the big nets' per-pin scratch for
// at most kEstNoallocBigPins pins in all.
constexpr uint32_t kEstNoallocMid = 1u << 20, kEstNoallocBig = 1u << 16, kEstNoallocBigPins = 1u << 17;
constexpr size_t kEstScratchBytes =
    256 + 4 * ((size_t)kEstNoallocMid + kEstNoallocBig) + 8 * (size_t)kEstNoallocBig + 64 * (size_t)kEstNoallocBigPins;
// Device address of that scratch on `device`, which must be the current
// device; looked up once per device and kept.
hipError_t est_noalloc_scratch(int device, unsigned char **ptr);
// n_mid = st[0], n_big = st[1] as read back by the host; the kernels read
// the counts from st as well.  The block kernel of the nets above 64 pins
// runs on s; the two smaller tiers on `side` when given (the caller orders
// side after s's earlier work and s after side's), else on s after it.
hipError_t launch_est(const EstArgs &A, const int32_t *mid, const int32_t *big, const uint32_t *st, uint32_t n_mid,
                      uint32_t n_big, hipStream_t s, hipStream_t side = nullptr);

// off[b] / *total get the big nets' pin offsets and their pin total (count
// read from st[1] on the device): big_tmp needs 16 * total words, and the
// gradient mode's acc 2 * total zeroed ones.
hipError_t launch_est_acc_offsets(const EstArgs &A, const int32_t *big, const uint32_t *st, int64_t *off,
                                  unsigned long long *total, hipStream_t s);
hipError_t launch_est_grad(const EstArgs &A, const int32_t *mid, const int32_t *big, const uint32_t *st,
                           uint32_t n_mid, uint32_t n_big, hipStream_t s, hipStream_t side = nullptr);

}  // namespace sta
