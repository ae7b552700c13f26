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
} orc_design;

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
      R[k] = (double)D->res_kohm[base + k];
      Chat[k] = wire_cap ? wire_cap[base + k] : (double)D->cap_ff[base + k];
    }
    for (int32_t s = D->net_sink_ptr[n]; s < D->net_sink_ptr[n + 1]; s++) Chat[D->sink_node[s]] += pc[s];
    orc_rc_tree(m, D->parent + base, R, Chat, load, d, ld, m2);
    L_net[n] = load[0];
    for (int32_t s = D->net_sink_ptr[n]; s < D->net_sink_ptr[n + 1]; s++) {
      int32_t k = D->sink_node[s];
      double q = 2.0 * m2[k] - d[k] * d[k];
      d_sink[s] = d[k];
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
int orc_sta(const orc_design *D, const double *wire_cap, orc_result *out) {
  int32_t NP = D->n_pins;
  if (orc_levelize(D, out->level, out->level_order, &out->n_levels)) return 1;
  roles_t R;
  roles_build(D, &R);
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
  roles_free(&R);
  return 0;
}
