/*
 * FP64 CPU oracle for the static-timing hot path.  TEST INFRASTRUCTURE ONLY:
 * only the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no code, header, table or helper with the GPU library.
 *
 * Plain single-threaded loops in double precision, each step written from its
 * definition.  The paper (HeteroSTA) names the steps but prints no formulas:
 *   - netlist as flattened CSR edge lists .......... §III "Heterogeneous netlist database"
 *   - RC trees as a flattened RC CSR ............... §III "Parasitics (RC) inputs"
 *   - Elmore net delay ............................. §II, §III "Delay models"
 *   - NLDM cell delay / slew tables ................ §IV-A, Table I ("NLDM+Arnoldi")
 *   - graph-based propagation, pin slacks, WNS/TNS . §I, §III "Report options"
 *   - STA itself ................................... §II (textbook STA, ref. [STABook])
 * so the formulas are the textbook ones:
 *   levels      level(p) = 0 without fanin, else 1 + max over fanin of level
 *   RC tree     load(k) = sum of C^ over sub(k); d(k) = d(parent) + R_k load(k)  (Elmore m1)
 *               ld(k) = sum over sub(k) of C^_j d(j); m2(k) = m2(parent) + R_k ld(k)
 *               q(k) = max(0, 2 m2(k) - d(k)^2)  (spread of the impulse response)
 *               sink slew = sqrt(driver slew^2 + q), sink AT = driver AT + d
 *   NLDM        bilinear interpolation, linear extrapolation on boundary segments
 *   forward     AT_out = max (late) / min (early) over unate-compatible fanin arcs
 *               of AT_in + delay; slew_out = the same merge over arc output slews
 *   backward    RAT = min (late) / max (early) over fanouts of RAT_fo - delay
 *   slack       late RAT - AT, early AT - RAT; WNS = min(0, min endpoint slack),
 *               TNS = sum of min(0, endpoint slack); Table IV prints both as zero
 *               for a design without violations
 * Views v = 2*el + rf with el 0 early / 1 late and rf 0 rise / 1 fall.
 * Parity pins for every function live in tests/test_oracle_pins.py.
 */
#include <time.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t n_pins, n_cells, n_nets, n_pi, n_po;
  const int32_t *pin_kind; /* 0 PI, 1 cell input, 2 cell output, 3 PO */
  const int32_t *cell_type, *cell_in_ptr, *cell_in_pin, *cell_out_pin;
  const int32_t *net_driver, *net_sink_ptr, *net_sink_pin;
  const int64_t *net_node_ptr;
  const int32_t *parent; /* net-local, -1 at the root */
  const float *res_kohm, *cap_ff;
  const int32_t *sink_node; /* net-local node of each sink */
  int32_t n_types, nx, ny;
  const int32_t *n_inputs, *sense; /* sense 0 positive, 1 negative, 2 non-unate */
  const float *pin_cap_ff, *slew_axis, *load_axis, *tables;
  float po_cap_ff;
  const float *pi_at, *pi_slew, *po_rat; /* [n_pi][4], [n_pi][4], [n_po][4] */
  float dangling_rat[4];
  int32_t dangling_policy; /* 1: cell outputs without fanout are endpoints */
  const double *res64;     /* FP64 segment resistances overriding res_kohm when non-NULL */
  const double *delay64;   /* per-sink net delays overriding the Elmore delay when non-NULL */
  /* Perturbation inputs of the smooth forward, for finite-difference pins of
   * its adjoint (NULL: none).  load64[n] is added to net n's load as the NLDM
   * lookups of its driver see it (not to the RC moments); arcd64[k][v] is
   * added to the delay of cell arc k (cell_in_pin order) in view v. */
  const double *load64;
  const double *arcd64;
} orc_design;

static double seg_res(const orc_design *D, int64_t k) {
  return D->res64 ? D->res64[k] : (double)D->res_kohm[k];
}

typedef struct {
  int32_t *level, *level_order;    /* [n_pins] */
  double *L_net;                   /* [n_nets] */
  double *d_sink, *q_sink;         /* [n_sinks] */
  double *at, *slew, *rat, *slack; /* [n_pins][4] */
  int8_t *crit;                    /* [n_pins][4] */
  int32_t *ep_pin;                 /* [n_ep] (capacity n_pins) */
  double *ep_slack;                /* [n_ep][2] */
  int32_t *ep_order;               /* [2][n_ep] */
  double wns[2], tns[2];
  int32_t n_ep, n_levels;
  double update_s; /* wall time of the update proper (below), for the host baseline */
} orc_result;

enum { PI_ = 0, CIN_ = 1, COUT_ = 2, PO_ = 3 };

/* ------------------------------------------------------------ pin roles */

typedef struct {
  int32_t *drv_net;  /* net driven by the pin, or -1 */
  int32_t *sink_idx; /* index into net_sink_* of a sink pin, or -1 */
  int32_t *sink_net; /* net of each sink index */
  int32_t *cell_of;  /* cell of a cell pin, or -1 */
  int32_t *rank;     /* PI rank / PO rank by pin id, or -1 */
} roles_t;

static void roles_build(const orc_design *D, roles_t *r) {
  int32_t NP = D->n_pins, NS = D->net_sink_ptr[D->n_nets];
  r->drv_net = malloc(sizeof(int32_t) * (size_t)NP);
  r->sink_idx = malloc(sizeof(int32_t) * (size_t)NP);
  r->sink_net = malloc(sizeof(int32_t) * (size_t)(NS > 0 ? NS : 1));
  r->cell_of = malloc(sizeof(int32_t) * (size_t)NP);
  r->rank = malloc(sizeof(int32_t) * (size_t)NP);
  for (int32_t p = 0; p < NP; p++) {
    r->drv_net[p] = -1; r->sink_idx[p] = -1; r->cell_of[p] = -1; r->rank[p] = -1;
  }
  for (int32_t n = 0; n < D->n_nets; n++) {
    r->drv_net[D->net_driver[n]] = n;
    for (int32_t s = D->net_sink_ptr[n]; s < D->net_sink_ptr[n + 1]; s++) {
      r->sink_idx[D->net_sink_pin[s]] = s;
      r->sink_net[s] = n;
    }
  }
  for (int32_t c = 0; c < D->n_cells; c++) {
    r->cell_of[D->cell_out_pin[c]] = c;
    for (int32_t k = D->cell_in_ptr[c]; k < D->cell_in_ptr[c + 1]; k++) r->cell_of[D->cell_in_pin[k]] = c;
  }
  int32_t npi = 0, npo = 0;
  for (int32_t p = 0; p < NP; p++) {
    if (D->pin_kind[p] == PI_) r->rank[p] = npi++;
    else if (D->pin_kind[p] == PO_) r->rank[p] = npo++;
  }
}

static void roles_free(roles_t *r) {
  free(r->drv_net); free(r->sink_idx); free(r->sink_net); free(r->cell_of); free(r->rank);
}

/* -------------------------------------------------------- levelization */

/* Longest-path levels over the timing graph (net arcs driver -> sink, cell arcs
 * input -> output) by Kahn's topological order, then the pins in ascending
 * (level, pin id).  Returns 1 if some pin is on a cycle. */
int orc_levelize(const orc_design *D, int32_t *level, int32_t *level_order, int32_t *n_levels) {
  roles_t R;
  roles_build(D, &R);
  int32_t NP = D->n_pins;
  int32_t *indeg = calloc((size_t)NP, sizeof(int32_t));
  for (int32_t p = 0; p < NP; p++) {
    level[p] = 0;
    if (D->pin_kind[p] == CIN_ || D->pin_kind[p] == PO_) indeg[p] = 1;
    else if (D->pin_kind[p] == COUT_) {
      int32_t c = R.cell_of[p];
      indeg[p] = D->cell_in_ptr[c + 1] - D->cell_in_ptr[c];
    }
  }
  int32_t *queue = malloc(sizeof(int32_t) * (size_t)NP);
  int32_t head = 0, tail = 0;
  for (int32_t p = 0; p < NP; p++)
    if (indeg[p] == 0) queue[tail++] = p;
  while (head < tail) {
    int32_t u = queue[head++];
    int32_t kind = D->pin_kind[u];
    if (kind == PI_ || kind == COUT_) {
      int32_t n = R.drv_net[u];
      if (n >= 0)
        for (int32_t s = D->net_sink_ptr[n]; s < D->net_sink_ptr[n + 1]; s++) {
          int32_t v = D->net_sink_pin[s];
          if (level[u] + 1 > level[v]) level[v] = level[u] + 1;
          if (--indeg[v] == 0) queue[tail++] = v;
        }
    } else if (kind == CIN_) {
      int32_t v = D->cell_out_pin[R.cell_of[u]];
      if (level[u] + 1 > level[v]) level[v] = level[u] + 1;
      if (--indeg[v] == 0) queue[tail++] = v;
    }
  }
  int cyc = tail < NP;
  int32_t maxl = 0;
  for (int32_t p = 0; p < NP; p++)
    if (level[p] > maxl) maxl = level[p];
  int32_t *cnt = calloc((size_t)maxl + 2, sizeof(int32_t));
  for (int32_t p = 0; p < NP; p++) cnt[level[p] + 1]++;
  for (int32_t l = 0; l <= maxl; l++) cnt[l + 1] += cnt[l];
  for (int32_t p = 0; p < NP; p++) level_order[cnt[level[p]]++] = p;
  *n_levels = maxl + 1;
  free(cnt); free(queue); free(indeg); roles_free(&R);
  return cyc;
}

/* ------------------------------------------------------------- RC trees */

/* Input cap of each sink pin: the receiving cell type's pin cap, or the PO cap. */
static void sink_pincaps(const orc_design *D, const roles_t *R, double *pc) {
  int32_t NS = D->net_sink_ptr[D->n_nets];
  for (int32_t s = 0; s < NS; s++) {
    int32_t pin = D->net_sink_pin[s];
    pc[s] = D->pin_kind[pin] == PO_ ? (double)D->po_cap_ff
                                    : (double)D->pin_cap_ff[D->cell_type[R->cell_of[pin]]];
  }
}

/* Elmore delay and second moment on one RC tree (nodes 0..m-1, parent[k] < k,
 * node 0 the root at the driver).  Chat[k] = wire cap + sink pin caps at k. */
void orc_rc_tree(int64_t m, const int32_t *parent, const double *R, const double *Chat,
                 double *load, double *d, double *ld, double *m2) {
  for (int64_t k = 0; k < m; k++) load[k] = Chat[k];
  for (int64_t k = m - 1; k >= 1; k--) load[parent[k]] += load[k];
  d[0] = 0.0;
  for (int64_t k = 1; k < m; k++) d[k] = d[parent[k]] + R[k] * load[k];
  for (int64_t k = 0; k < m; k++) ld[k] = Chat[k] * d[k];
  for (int64_t k = m - 1; k >= 1; k--) ld[parent[k]] += ld[k];
  m2[0] = 0.0;
  for (int64_t k = 1; k < m; k++) m2[k] = m2[parent[k]] + R[k] * ld[k];
}

/* All nets: L_net = load at the root; per sink d and q = max(0, 2 m2 - d^2).
 * wire_cap (FP64, caller node order) replaces the design's node caps if given. */
void orc_rc(const orc_design *D, const double *wire_cap, double *L_net, double *d_sink, double *q_sink) {
  roles_t RL;
  roles_build(D, &RL);
  int32_t NS = D->net_sink_ptr[D->n_nets];
  double *pc = malloc(sizeof(double) * (size_t)(NS > 0 ? NS : 1));
  sink_pincaps(D, &RL, pc);
  int64_t maxm = 1;
  for (int32_t n = 0; n < D->n_nets; n++) {
    int64_t m = D->net_node_ptr[n + 1] - D->net_node_ptr[n];
    if (m > maxm) maxm = m;
  }
  double *R = malloc(sizeof(double) * (size_t)maxm), *Chat = malloc(sizeof(double) * (size_t)maxm);
  double *load = malloc(sizeof(double) * (size_t)maxm), *d = malloc(sizeof(double) * (size_t)maxm);
  double *ld = malloc(sizeof(double) * (size_t)maxm), *m2 = malloc(sizeof(double) * (size_t)maxm);
  for (int32_t n = 0; n < D->n_nets; n++) {
    int64_t base = D->net_node_ptr[n], m = D->net_node_ptr[n + 1] - base;
    for (int64_t k = 0; k < m; k++) {
      R[k] = seg_res(D, base + k);
      Chat[k] = wire_cap ? wire_cap[base + k] : (double)D->cap_ff[base + k];
    }
    for (int32_t s = D->net_sink_ptr[n]; s < D->net_sink_ptr[n + 1]; s++) Chat[D->sink_node[s]] += pc[s];
    orc_rc_tree(m, D->parent + base, R, Chat, load, d, ld, m2);
    L_net[n] = load[0];
    for (int32_t s = D->net_sink_ptr[n]; s < D->net_sink_ptr[n + 1]; s++) {
      int32_t k = D->sink_node[s];
      double q = 2.0 * m2[k] - d[k] * d[k];
      d_sink[s] = D->delay64 ? D->delay64[s] : d[k];
      q_sink[s] = q > 0.0 ? q : 0.0;
    }
  }
  free(R); free(Chat); free(load); free(d); free(ld); free(m2); free(pc);
  roles_free(&RL);
}

/* ----------------------------------------------------------------- NLDM */

/* Bilinear table value at (X, Y).  Segment i is the largest i with x_i <= X,
 * kept inside [0, nx-2], so points off the table extrapolate linearly along the
 * boundary segment.  table is [nx][ny] row-major in (slew, load). */
double orc_nldm(int32_t nx, int32_t ny, const float *xa, const float *ya, const float *table,
                double X, double Y) {
  int32_t i = 0, j = 0;
  for (int32_t m = 1; m <= nx - 2; m++)
    if ((double)xa[m] <= X) i = m;
  for (int32_t m = 1; m <= ny - 2; m++)
    if ((double)ya[m] <= Y) j = m;
  double t = (X - xa[i]) / ((double)xa[i + 1] - xa[i]);
  double u = (Y - ya[j]) / ((double)ya[j + 1] - ya[j]);
  double T00 = table[i * ny + j], T10 = table[(i + 1) * ny + j];
  double T01 = table[i * ny + j + 1], T11 = table[(i + 1) * ny + j + 1];
  return (1 - t) * (1 - u) * T00 + t * (1 - u) * T10 + (1 - t) * u * T01 + t * u * T11;
}

/* Does an input transition r_i reach output transition r_o for this sense? */
static int arc_maps(int32_t sense, int r_i, int r_o) {
  if (sense == 0) return r_i == r_o;
  if (sense == 1) return r_i != r_o;
  return 1;
}

static double arc_delay(const orc_design *D, int32_t type, int r_o, double slew, double load) {
  const float *tb = D->tables + ((size_t)type * 4 + (size_t)r_o) * D->nx * D->ny;
  return orc_nldm(D->nx, D->ny, D->slew_axis + (size_t)type * D->nx, D->load_axis + (size_t)type * D->ny,
                  tb, slew, load);
}

static double arc_slew(const orc_design *D, int32_t type, int r_o, double slew, double load) {
  const float *tb = D->tables + ((size_t)type * 4 + 2 + (size_t)r_o) * D->nx * D->ny;
  return orc_nldm(D->nx, D->ny, D->slew_axis + (size_t)type * D->nx, D->load_axis + (size_t)type * D->ny,
                  tb, slew, load);
}

/* ------------------------------------------------------- full analysis */

static int is_endpoint(const orc_design *D, const roles_t *R, int32_t p) {
  if (D->pin_kind[p] == PO_) return 1;
  if (D->dangling_policy && D->pin_kind[p] == COUT_) {
    int32_t n = R->drv_net[p];
    return n < 0 || D->net_sink_ptr[n + 1] == D->net_sink_ptr[n];
  }
  return 0;
}

static const double *g_sort_key;
static const int32_t *g_sort_pin;
static int ep_cmp(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  if (g_sort_key[x] < g_sort_key[y]) return -1;
  if (g_sort_key[x] > g_sort_key[y]) return 1;
  return g_sort_pin[x] < g_sort_pin[y] ? -1 : (g_sort_pin[x] > g_sort_pin[y]);
}

/* Forward arrival/slew, backward required time, slack and endpoint reports.
 * wire_cap (caller node order, FP64) overrides the node caps when non-NULL.
 * Returns 1 on a combinational cycle. */
static double wall_s(void) {
  struct timespec t;
  clock_gettime(CLOCK_MONOTONIC, &t);
  return (double)t.tv_sec + 1e-9 * (double)t.tv_nsec;
}

int orc_sta(const orc_design *D, const double *wire_cap, orc_result *out) {
  int32_t NP = D->n_pins;
  if (orc_levelize(D, out->level, out->level_order, &out->n_levels)) return 1;
  roles_t R;
  roles_build(D, &R);
  /* the update proper starts here (levels and pin roles are what a timer
     builds once per netlist); only timed, nothing below depends on it */
  const double t_update = wall_s();
  orc_rc(D, wire_cap, out->L_net, out->d_sink, out->q_sink);
  double *at = out->at, *sl = out->slew, *rat = out->rat;

  /* forward, pins in level order */
  for (int32_t o = 0; o < NP; o++) {
    int32_t p = out->level_order[o];
    int32_t kind = D->pin_kind[p];
    for (int v = 0; v < 4; v++) out->crit[p * 4 + v] = -1;
    if (kind == PI_) {
      for (int v = 0; v < 4; v++) {
        at[p * 4 + v] = D->pi_at[R.rank[p] * 4 + v];
        sl[p * 4 + v] = D->pi_slew[R.rank[p] * 4 + v];
      }
    } else if (kind == CIN_ || kind == PO_) {
      int32_t s = R.sink_idx[p];
      int32_t drv = D->net_driver[R.sink_net[s]];
      for (int v = 0; v < 4; v++) {
        at[p * 4 + v] = at[drv * 4 + v] + out->d_sink[s];
        sl[p * 4 + v] = sqrt(sl[drv * 4 + v] * sl[drv * 4 + v] + out->q_sink[s]);
      }
    } else { /* cell output */
      int32_t c = R.cell_of[p], type = D->cell_type[c], sense = D->sense[type];
      double load = out->L_net[R.drv_net[p]];
      for (int el = 0; el < 2; el++)
        for (int r_o = 0; r_o < 2; r_o++) {
          int v = el * 2 + r_o;
          double best_at = el ? -INFINITY : INFINITY, best_sl = el ? -INFINITY : INFINITY;
          int best_k = -1;
          for (int32_t k = D->cell_in_ptr[c]; k < D->cell_in_ptr[c + 1]; k++) {
            int32_t in = D->cell_in_pin[k];
            for (int r_i = 0; r_i < 2; r_i++) {
              if (!arc_maps(sense, r_i, r_o)) continue;
              double x = sl[in * 4 + el * 2 + r_i];
              double cand = at[in * 4 + el * 2 + r_i] + arc_delay(D, type, r_o, x, load);
              double cs = arc_slew(D, type, r_o, x, load);
              if (el ? cand > best_at : cand < best_at) {
                best_at = cand;
                best_k = (k - D->cell_in_ptr[c]) * 2 + r_i;
              }
              if (el ? cs > best_sl : cs < best_sl) best_sl = cs;
            }
          }
          at[p * 4 + v] = best_at;
          sl[p * 4 + v] = best_sl;
          out->crit[p * 4 + v] = (int8_t)best_k;
        }
    }
  }

  /* backward, pins in reverse level order */
  for (int32_t o = NP - 1; o >= 0; o--) {
    int32_t p = out->level_order[o];
    int32_t kind = D->pin_kind[p];
    if (kind == PO_) {
      for (int v = 0; v < 4; v++) rat[p * 4 + v] = D->po_rat[R.rank[p] * 4 + v];
    } else if (kind == CIN_) {
      int32_t c = R.cell_of[p], type = D->cell_type[c], sense = D->sense[type];
      int32_t out_pin = D->cell_out_pin[c];
      double load = out->L_net[R.drv_net[out_pin]];
      for (int el = 0; el < 2; el++)
        for (int r_i = 0; r_i < 2; r_i++) {
          double best = el ? INFINITY : -INFINITY;
          double x = sl[p * 4 + el * 2 + r_i];
          for (int r_o = 0; r_o < 2; r_o++) {
            if (!arc_maps(sense, r_i, r_o)) continue;
            double cand = rat[out_pin * 4 + el * 2 + r_o] - arc_delay(D, type, r_o, x, load);
            if (el ? cand < best : cand > best) best = cand;
          }
          rat[p * 4 + el * 2 + r_i] = best;
        }
    } else { /* PI or cell output: a net driver */
      int32_t n = R.drv_net[p];
      int has_sinks = n >= 0 && D->net_sink_ptr[n + 1] > D->net_sink_ptr[n];
      if (!has_sinks && is_endpoint(D, &R, p)) {
        for (int v = 0; v < 4; v++) rat[p * 4 + v] = D->dangling_rat[v];
      } else {
        for (int v = 0; v < 4; v++) {
          int el = v / 2;
          double best = el ? INFINITY : -INFINITY;
          if (n >= 0)
            for (int32_t s = D->net_sink_ptr[n]; s < D->net_sink_ptr[n + 1]; s++) {
              double cand = rat[D->net_sink_pin[s] * 4 + v] - out->d_sink[s];
              if (el ? cand < best : cand > best) best = cand;
            }
          rat[p * 4 + v] = best;
        }
      }
    }
  }

  /* slack */
  for (int32_t p = 0; p < NP; p++)
    for (int v = 0; v < 4; v++) {
      double a = at[p * 4 + v], r = rat[p * 4 + v];
      out->slack[p * 4 + v] = (v / 2) ? r - a : a - r;
    }

  /* endpoints, ascending pin id */
  int32_t ne = 0;
  for (int32_t p = 0; p < NP; p++)
    if (is_endpoint(D, &R, p)) out->ep_pin[ne++] = p;
  out->n_ep = ne;
  for (int el = 0; el < 2; el++) {
    double wns = 0.0, tns = 0.0;
    for (int32_t e = 0; e < ne; e++) {
      int32_t p = out->ep_pin[e];
      double a = out->slack[p * 4 + el * 2 + 0], b = out->slack[p * 4 + el * 2 + 1];
      double s = a < b ? a : b;
      out->ep_slack[e * 2 + el] = s;
      if (s < wns) wns = s;
      if (s < 0.0) tns += s;
    }
    out->wns[el] = wns;
    out->tns[el] = tns;
  }
  /* endpoint order per el: ascending (slack, endpoint pin id) */
  double *key = malloc(sizeof(double) * (size_t)(ne > 0 ? ne : 1));
  for (int el = 0; el < 2; el++) {
    for (int32_t e = 0; e < ne; e++) {
      key[e] = out->ep_slack[e * 2 + el];
      out->ep_order[el * ne + e] = e;
    }
    g_sort_key = key;
    g_sort_pin = out->ep_pin;
    qsort(out->ep_order + el * ne, (size_t)ne, sizeof(int32_t), ep_cmp);
  }
  free(key);
  out->update_s = wall_s() - t_update;
  roles_free(&R);
  return 0;
}

/* ================================================================ smooth form
 *
 * Differentiable variant (not in the paper; it serves gradient-based
 * optimization loops of the kind §IV-C and §IV-D drive, where per-pin slacks
 * are fed back).  Late arrival merges use the log-sum-exp smooth maximum
 *     LSE_g(x) = m + g log sum exp((x_i - m) / g),  m = max x,
 * the late endpoint slack is the smooth minimum over rise/fall of RAT - AT,
 *     s = -LSE_g(AT_R - RAT_R, AT_F - RAT_F),
 * and the objective terms are
 *     TNS_g = sum_ep -g log(1 + exp(-s/g))            (smooth min(0, s))
 *     WNS_g = -g log(1 + sum_ep exp(-s/g))            (smooth min(0, min s)).
 * Early views and all slew merges stay hard.  The adjoint is reverse mode
 * through these definitions, the bilinear lookups and the RC moments. */

typedef struct {
  double *at, *slew;   /* [n_pins][4] */
  double *L_net;       /* [n_nets] */
  double *d_sink, *q_sink; /* [n_sinks] */
  int32_t *ep_pin;     /* [n_ep] (capacity n_pins) */
  double *ep_s;        /* [n_ep] smooth late slack */
  double tns, wns;
  int32_t n_ep;
  uint64_t sig;        /* hash of every discrete choice (table segments, slew winners) */
} orc_smooth_result;

static double lse2(double a, double b, double g) {
  double m = a > b ? a : b;
  return m + g * log(exp((a - m) / g) + exp((b - m) / g));
}

/* log(1 + exp(x)) without overflow */
static double softplus(double x) { return x > 0 ? x + log1p(exp(-x)) : log1p(exp(x)); }

static uint64_t mix(uint64_t h, uint64_t v) {
  h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
  return h;
}

/* Bilinear value and its partials in X and Y on the segment the lookup picks. */
static double nldm_d(int32_t nx, int32_t ny, const float *xa, const float *ya, const float *T, double X,
                     double Y, double *dX, double *dY, int32_t *seg) {
  int32_t i = 0, j = 0;
  for (int32_t m = 1; m <= nx - 2; m++)
    if ((double)xa[m] <= X) i = m;
  for (int32_t m = 1; m <= ny - 2; m++)
    if ((double)ya[m] <= Y) j = m;
  double hx = (double)xa[i + 1] - xa[i], hy = (double)ya[j + 1] - ya[j];
  double t = (X - xa[i]) / hx, u = (Y - ya[j]) / hy;
  double T00 = T[i * ny + j], T10 = T[(i + 1) * ny + j], T01 = T[i * ny + j + 1], T11 = T[(i + 1) * ny + j + 1];
  if (dX) *dX = ((1 - u) * (T10 - T00) + u * (T11 - T01)) / hx;
  if (dY) *dY = ((1 - t) * (T01 - T00) + t * (T11 - T10)) / hy;
  if (seg) *seg = i * 16 + j;
  return (1 - t) * (1 - u) * T00 + t * (1 - u) * T10 + (1 - t) * u * T01 + t * u * T11;
}

static const float *tab_of(const orc_design *D, int32_t type, int k) {
  return D->tables + ((size_t)type * 4 + (size_t)k) * D->nx * D->ny;
}

/* Smooth forward; returns 1 on a cycle.  level_order must come from
 * orc_levelize. */
static int smooth_forward(const orc_design *D, const roles_t *R, const int32_t *order, const double *wire_cap,
                          double gamma, orc_smooth_result *out) {
  int32_t NP = D->n_pins;
  double *at = out->at, *sl = out->slew;
  uint64_t sig = 1469598103934665603ull;
  orc_rc(D, wire_cap, out->L_net, out->d_sink, out->q_sink);
  for (int32_t o = 0; o < NP; o++) {
    int32_t p = order[o];
    int32_t kind = D->pin_kind[p];
    if (kind == PI_) {
      for (int v = 0; v < 4; v++) {
        at[p * 4 + v] = D->pi_at[R->rank[p] * 4 + v];
        sl[p * 4 + v] = D->pi_slew[R->rank[p] * 4 + v];
      }
    } else if (kind == CIN_ || kind == PO_) {
      int32_t s = R->sink_idx[p];
      int32_t drv = D->net_driver[R->sink_net[s]];
      for (int v = 0; v < 4; v++) {
        at[p * 4 + v] = at[drv * 4 + v] + out->d_sink[s];
        sl[p * 4 + v] = sqrt(sl[drv * 4 + v] * sl[drv * 4 + v] + out->q_sink[s]);
      }
    } else {
      int32_t c = R->cell_of[p], type = D->cell_type[c], sense = D->sense[type];
      double load = out->L_net[R->drv_net[p]] + (D->load64 ? D->load64[R->drv_net[p]] : 0.0);
      const float *xa = D->slew_axis + (size_t)type * D->nx, *ya = D->load_axis + (size_t)type * D->ny;
      for (int el = 0; el < 2; el++)
        for (int r_o = 0; r_o < 2; r_o++) {
          double best_sl = el ? -INFINITY : INFINITY, hard = el ? -INFINITY : INFINITY;
          int win = -1;
          /* candidate values */
          double z[16];
          int nz = 0;
          for (int32_t k = D->cell_in_ptr[c]; k < D->cell_in_ptr[c + 1]; k++) {
            int32_t in = D->cell_in_pin[k];
            for (int r_i = 0; r_i < 2; r_i++) {
              if (!arc_maps(sense, r_i, r_o)) continue;
              double x = sl[in * 4 + el * 2 + r_i];
              int32_t seg;
              double dl = nldm_d(D->nx, D->ny, xa, ya, tab_of(D, type, r_o), x, load, NULL, NULL, &seg);
              double cs = nldm_d(D->nx, D->ny, xa, ya, tab_of(D, type, 2 + r_o), x, load, NULL, NULL, NULL);
              if (el) sig = mix(sig, (uint64_t)seg);
              if (D->arcd64) dl += D->arcd64[(size_t)k * 4 + el * 2 + r_o];
              z[nz++] = at[in * 4 + el * 2 + r_i] + dl;
              if (el ? z[nz - 1] > hard : z[nz - 1] < hard) hard = z[nz - 1];
              if (el ? cs > best_sl : cs < best_sl) {
                best_sl = cs;
                win = (k - D->cell_in_ptr[c]) * 2 + r_i;
              }
            }
          }
          if (el) {
            double acc = 0.0;
            for (int i = 0; i < nz; i++) acc += exp((z[i] - hard) / gamma);
            at[p * 4 + el * 2 + r_o] = hard + gamma * log(acc);
            sig = mix(sig, (uint64_t)win);
          } else {
            at[p * 4 + el * 2 + r_o] = hard;
          }
          sl[p * 4 + el * 2 + r_o] = best_sl;
        }
    }
  }
  /* endpoints and the smooth objective */
  int32_t ne = 0;
  for (int32_t p = 0; p < NP; p++)
    if (is_endpoint(D, R, p)) out->ep_pin[ne++] = p;
  out->n_ep = ne;
  double tns = 0.0, mx = 0.0;
  for (int32_t e = 0; e < ne; e++) {
    int32_t p = out->ep_pin[e];
    double rr, rf;
    if (D->pin_kind[p] == PO_) {
      rr = D->po_rat[R->rank[p] * 4 + 2];
      rf = D->po_rat[R->rank[p] * 4 + 3];
    } else {
      rr = D->dangling_rat[2];
      rf = D->dangling_rat[3];
    }
    double s = -lse2(at[p * 4 + 2] - rr, at[p * 4 + 3] - rf, gamma);
    out->ep_s[e] = s;
    tns += -gamma * softplus(-s / gamma);
    if (-s / gamma > mx) mx = -s / gamma;
  }
  double acc = exp(-mx);
  for (int32_t e = 0; e < ne; e++) acc += exp(-out->ep_s[e] / gamma - mx);
  out->tns = tns;
  out->wns = -gamma * (mx + log(acc));
  out->sig = sig;
  return 0;
}

int orc_smooth_sta(const orc_design *D, const double *wire_cap, double gamma, orc_smooth_result *out) {
  int32_t NP = D->n_pins, nl;
  int32_t *level = malloc(sizeof(int32_t) * (size_t)NP), *order = malloc(sizeof(int32_t) * (size_t)NP);
  int cyc = orc_levelize(D, level, order, &nl);
  if (!cyc) {
    roles_t R;
    roles_build(D, &R);
    smooth_forward(D, &R, order, wire_cap, gamma, out);
    roles_free(&R);
  }
  free(level);
  free(order);
  return cyc;
}

/* Gradient of J = g_tns TNS_g + g_wns WNS_g with respect to every RC node's
 * ground cap and every segment's resistance (caller node order; grad_res may
 * be NULL), every cell output's NLDM load (the partial through the lookups
 * only, per pin) and every cell arc's additive delay per late output view
 * (arcs in cell_in_pin order, [n_arcs][4], early views 0).  Reverse mode over
 * the smooth forward, in reverse level order. */
int orc_smooth_adjoint(const orc_design *D, const double *wire_cap, double gamma, double g_tns, double g_wns,
                       double *grad_cap, double *grad_res, double *grad_load, double *grad_arc,
                       orc_smooth_result *fwd) {
  int32_t NP = D->n_pins, nl;
  int32_t NS = D->net_sink_ptr[D->n_nets];
  int32_t *level = malloc(sizeof(int32_t) * (size_t)NP), *order = malloc(sizeof(int32_t) * (size_t)NP);
  if (orc_levelize(D, level, order, &nl)) {
    free(level);
    free(order);
    return 1;
  }
  roles_t R;
  roles_build(D, &R);
  smooth_forward(D, &R, order, wire_cap, gamma, fwd);
  const double *at = fwd->at, *sl = fwd->slew;
  double *gA = calloc((size_t)NP * 2, sizeof(double)), *gS = calloc((size_t)NP * 2, sizeof(double));
  double *gL = calloc((size_t)D->n_nets, sizeof(double));
  double *gd = calloc((size_t)(NS > 0 ? NS : 1), sizeof(double)), *gq = calloc((size_t)(NS > 0 ? NS : 1), sizeof(double));
  int32_t n_arcs = D->cell_in_ptr[D->n_cells];
  memset(grad_arc, 0, sizeof(double) * (size_t)n_arcs * 4);
  memset(grad_load, 0, sizeof(double) * (size_t)NP);

  /* seeds at the endpoints */
  double mx = 0.0;
  for (int32_t e = 0; e < fwd->n_ep; e++)
    if (-fwd->ep_s[e] / gamma > mx) mx = -fwd->ep_s[e] / gamma;
  double den = exp(-mx);
  for (int32_t e = 0; e < fwd->n_ep; e++) den += exp(-fwd->ep_s[e] / gamma - mx);
  for (int32_t e = 0; e < fwd->n_ep; e++) {
    int32_t p = fwd->ep_pin[e];
    double s = fwd->ep_s[e];
    double sig_t = 1.0 / (1.0 + exp(s / gamma));               /* d TNS_g / d s */
    double sig_w = exp(-s / gamma - mx) / den;                  /* d WNS_g / d s */
    double gs = g_tns * sig_t + g_wns * sig_w;
    double rr, rf;
    if (D->pin_kind[p] == PO_) {
      rr = D->po_rat[R.rank[p] * 4 + 2];
      rf = D->po_rat[R.rank[p] * 4 + 3];
    } else {
      rr = D->dangling_rat[2];
      rf = D->dangling_rat[3];
    }
    /* s = -LSE(a_R, a_F), a = AT - RAT: ds/dAT_rf = -softmax_rf */
    double aR = at[p * 4 + 2] - rr, aF = at[p * 4 + 3] - rf, l = lse2(aR, aF, gamma);
    gA[p * 2 + 0] += -gs * exp((aR - l) / gamma);
    gA[p * 2 + 1] += -gs * exp((aF - l) / gamma);
  }

  /* reverse sweep over late views */
  for (int32_t o = NP - 1; o >= 0; o--) {
    int32_t p = order[o];
    int32_t kind = D->pin_kind[p];
    if (kind == CIN_ || kind == PO_) {
      int32_t s = R.sink_idx[p];
      int32_t drv = D->net_driver[R.sink_net[s]];
      for (int rf = 0; rf < 2; rf++) {
        double sp = sl[p * 4 + 2 + rf], sd = sl[drv * 4 + 2 + rf];
        gA[drv * 2 + rf] += gA[p * 2 + rf];
        gd[s] += gA[p * 2 + rf];
        gS[drv * 2 + rf] += gS[p * 2 + rf] * sd / sp;
        gq[s] += gS[p * 2 + rf] / (2.0 * sp);
      }
    } else if (kind == COUT_) {
      int32_t c = R.cell_of[p], type = D->cell_type[c], sense = D->sense[type];
      int32_t net = R.drv_net[p];
      double load = fwd->L_net[net];
      const float *xa = D->slew_axis + (size_t)type * D->nx, *ya = D->load_axis + (size_t)type * D->ny;
      for (int r_o = 0; r_o < 2; r_o++) {
        double gat = gA[p * 2 + r_o], gsl = gS[p * 2 + r_o];
        double best_sl = -INFINITY;
        int32_t win_in = -1, win_ri = -1;
        double win_dx = 0.0, win_dy = 0.0;
        for (int32_t k = D->cell_in_ptr[c]; k < D->cell_in_ptr[c + 1]; k++) {
          int32_t in = D->cell_in_pin[k];
          for (int r_i = 0; r_i < 2; r_i++) {
            if (!arc_maps(sense, r_i, r_o)) continue;
            double x = sl[in * 4 + 2 + r_i], ddx, ddy, sdx, sdy;
            double dl = nldm_d(D->nx, D->ny, xa, ya, tab_of(D, type, r_o), x, load, &ddx, &ddy, NULL);
            double cs = nldm_d(D->nx, D->ny, xa, ya, tab_of(D, type, 2 + r_o), x, load, &sdx, &sdy, NULL);
            double w = exp((at[in * 4 + 2 + r_i] + dl - at[p * 4 + 2 + r_o]) / gamma); /* softmax weight */
            gA[in * 2 + r_i] += w * gat;
            gS[in * 2 + r_i] += w * gat * ddx;
            gL[net] += w * gat * ddy;
            grad_arc[(size_t)k * 4 + 2 + r_o] += w * gat;
            if (cs > best_sl) {
              best_sl = cs;
              win_in = in;
              win_ri = r_i;
              win_dx = sdx;
              win_dy = sdy;
            }
          }
        }
        gS[win_in * 2 + win_ri] += gsl * win_dx;
        gL[net] += gsl * win_dy;
      }
      grad_load[p] = gL[net];
    }
  }

  /* RC adjoint per net: J depends on the node caps through L_net (every node),
   * d_s and q_s = 2 m2 - d^2.  With R_kj the shared path resistance:
   *   dd_v/dC_k = R_vk,   dm2_v/dC_k = R_vk d_k + sum_j C^_j R_vj R_jk,
   * so, with gd_v = dJ/dd_v - 2 d_v dJ/dq_v and gm_v = 2 dJ/dq_v at sink nodes,
   *   dJ/dC_k = gL + sum_{a on path(k)} R_a Gd(a) + d_k H_k + sum_{a on path(k)} R_a K(a)
   *   Gd(a) = subtree sum of gd, H_j = sum_{a on path(j)} R_a Gm(a),
   *   Gm(a) = subtree sum of gm, K(a) = subtree sum of C^ H.
   * A segment's resistance enters d_v as R_k S1_k (S1 = downstream cap) on
   * every path through k, and m2_v as R_k S2_k (S2 = subtree sum of C^ d)
   * plus through the d_j inside S2 of the segments above, which gives
   *   dJ/dR_k = S1_k (Gd(k) + K(k)) + S2_k Gm(k),   dJ/dR_root = 0. */
  double *pc = malloc(sizeof(double) * (size_t)(NS > 0 ? NS : 1));
  sink_pincaps(D, &R, pc);
  int64_t maxm = 1;
  for (int32_t n = 0; n < D->n_nets; n++) {
    int64_t m = D->net_node_ptr[n + 1] - D->net_node_ptr[n];
    if (m > maxm) maxm = m;
  }
  double *Rv = malloc(sizeof(double) * maxm), *Ch = malloc(sizeof(double) * maxm);
  double *load = malloc(sizeof(double) * maxm), *dd = malloc(sizeof(double) * maxm);
  double *ld = malloc(sizeof(double) * maxm), *m2 = malloc(sizeof(double) * maxm);
  double *Gd = malloc(sizeof(double) * maxm), *Gm = malloc(sizeof(double) * maxm);
  double *H = malloc(sizeof(double) * maxm), *K = malloc(sizeof(double) * maxm);
  double *PA = malloc(sizeof(double) * maxm), *PB = malloc(sizeof(double) * maxm);
  for (int32_t n = 0; n < D->n_nets; n++) {
    int64_t base = D->net_node_ptr[n], m = D->net_node_ptr[n + 1] - base;
    const int32_t *par = D->parent + base;
    for (int64_t k = 0; k < m; k++) {
      Rv[k] = seg_res(D, base + k);
      Ch[k] = wire_cap ? wire_cap[base + k] : (double)D->cap_ff[base + k];
      Gd[k] = Gm[k] = 0.0;
    }
    for (int32_t s = D->net_sink_ptr[n]; s < D->net_sink_ptr[n + 1]; s++) Ch[D->sink_node[s]] += pc[s];
    orc_rc_tree(m, par, Rv, Ch, load, dd, ld, m2);
    for (int32_t s = D->net_sink_ptr[n]; s < D->net_sink_ptr[n + 1]; s++) {
      int32_t k = D->sink_node[s];
      double qraw = 2.0 * m2[k] - dd[k] * dd[k];
      double gqs = qraw > 0.0 ? gq[s] : 0.0;
      Gd[k] += gd[s] - 2.0 * dd[k] * gqs;
      Gm[k] += 2.0 * gqs;
    }
    for (int64_t k = m - 1; k >= 1; k--) {
      Gd[par[k]] += Gd[k];
      Gm[par[k]] += Gm[k];
    }
    H[0] = 0.0;
    PA[0] = 0.0;
    for (int64_t k = 1; k < m; k++) {
      H[k] = H[par[k]] + Rv[k] * Gm[k];
      PA[k] = PA[par[k]] + Rv[k] * Gd[k];
    }
    for (int64_t k = 0; k < m; k++) K[k] = Ch[k] * H[k];
    for (int64_t k = m - 1; k >= 1; k--) K[par[k]] += K[k];
    if (grad_res) {
      grad_res[base] = 0.0;
      for (int64_t k = 1; k < m; k++) grad_res[base + k] = load[k] * (Gd[k] + K[k]) + ld[k] * Gm[k];
    }
    PB[0] = 0.0;
    for (int64_t k = 1; k < m; k++) PB[k] = PB[par[k]] + Rv[k] * K[k];
    for (int64_t k = 0; k < m; k++) grad_cap[base + k] = gL[n] + PA[k] + dd[k] * H[k] + PB[k];
  }
  free(Rv); free(Ch); free(load); free(dd); free(ld); free(m2); free(Gd); free(Gm); free(H); free(K);
  free(PA); free(PB); free(pc);
  free(gA); free(gS); free(gL); free(gd); free(gq);
  roles_free(&R);
  free(level);
  free(order);
  return 0;
}
