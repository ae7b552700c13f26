/*
 * Seeded synthetic STA design generator.
 *
 * Stands in for the benchmark designs the paper evaluates on (TAU 2015 transpiled
 * to 14 nm in Table I, ICCAD 2015 in Table III, ISPD 2025 in Table IV), which are
 * not available here.  It produces, in the caller-facing flattened format:
 *   - a levelized random DAG netlist as cell CSR + net CSR arrays (the flattened
 *     netlist database of §III, "Heterogeneous netlist database"),
 *   - one RC tree per net as a flattened RC CSR (§III, "Parasitics (RC) inputs"),
 *   - a Liberty-style library of 7x7 NLDM tables (Table I uses NLDM),
 *   - PI arrival/slew and endpoint required-time constraints.
 *
 * It contains none of the timing arithmetic: no delay, slew, arrival, required
 * time or level is computed here.  Randomness comes from SplitMix64 (Steele, Lea
 * and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014),
 * written from its published definition.  Uniform doubles take the top 53 bits.
 *
 * Shared by the FP64 oracle tests and by the GPU path's tests and benchmark; it
 * depends on neither.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- PRNG */

typedef struct { uint64_t s; } sm64_t;

static uint64_t sm64_next(sm64_t *g) {
  uint64_t z = (g->s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double u01(sm64_t *g) { return (double)(sm64_next(g) >> 11) * 0x1.0p-53; }
static double unif(sm64_t *g, double a, double b) { return a + (b - a) * u01(g); }
/* integer uniform on [0, n) for n >= 1 */
static int64_t below(sm64_t *g, int64_t n) {
  int64_t r = (int64_t)(u01(g) * (double)n);
  return r >= n ? n - 1 : r;
}
/* independent stream per generation phase */
static sm64_t stream(uint64_t seed, uint64_t phase) {
  sm64_t g = {seed ^ (0xD1B54A32D192ED03ull * (phase + 1))};
  sm64_next(&g);
  return g;
}

/* ------------------------------------------------- Fenwick (weighted draw) */

typedef struct { int64_t n; int64_t *t; } fenwick_t;

static void fw_init(fenwick_t *f, const int64_t *w, int64_t n) {
  f->n = n;
  f->t = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  for (int64_t i = 1; i <= n; i++) {
    f->t[i] += w[i - 1];
    int64_t j = i + (i & -i);
    if (j <= n) f->t[j] += f->t[i];
  }
}
static void fw_add(fenwick_t *f, int64_t i, int64_t v) {
  for (i++; i <= f->n; i += i & -i) f->t[i] += v;
}
static int64_t fw_prefix(const fenwick_t *f, int64_t i) { /* sum of w[0..i) */
  int64_t s = 0;
  for (; i > 0; i -= i & -i) s += f->t[i];
  return s;
}
/* smallest index i with prefix(i+1) > r, for 0 <= r < total */
static int64_t fw_find(const fenwick_t *f, int64_t r) {
  int64_t pos = 0, step = 1;
  while (step * 2 <= f->n) step *= 2;
  for (; step > 0; step /= 2) {
    if (pos + step <= f->n && f->t[pos + step] <= r) {
      pos += step;
      r -= f->t[pos];
    }
  }
  return pos;
}

/* ---------------------------------------------------------- public types */

typedef struct {
  int64_t n_cells;
  int32_t n_levels, n_pi, n_po;
  double fanout_mu;
  int32_t fanout_cap;
  int32_t n_types;
  int32_t n_heavy;      /* number of heavy levels, drawn from 2..n_levels */
  double heavy_frac;    /* fraction of all cells in each heavy level */
  int32_t n_hf;         /* number of high-fanout nets */
  int32_t hf_min, hf_max;
  double rat_ps, rat_early_ps, pi_at_ps, pi_slew_ps, po_cap_ff;
  int32_t dangling_policy;
  int32_t shuffle;      /* permute pin ids, cell order and net order */
  uint64_t seed;
  uint64_t lib_seed;    /* library stream seed; 0 = the design seed */
} synth_cfg;

typedef struct {
  int32_t n_pins, n_cells, n_nets, n_pi, n_po, n_sinks, n_cell_in;
  int64_t n_nodes;
  int32_t *pin_kind;                 /* 0 PI, 1 cell input, 2 cell output, 3 PO */
  int32_t *cell_type, *cell_in_ptr, *cell_in_pin, *cell_out_pin;
  int32_t *net_driver, *net_sink_ptr, *net_sink_pin;
  int64_t *net_node_ptr;
  int32_t *parent;
  float *res_kohm, *cap_ff;
  int32_t *sink_node;
  int32_t n_types, nx, ny;
  int32_t *n_inputs, *sense;
  float *pin_cap_ff, *slew_axis, *load_axis, *tables;
  float po_cap_ff;
  float *pi_at, *pi_slew, *po_rat;
  float dangling_rat[4];
  int32_t dangling_policy;
} synth_design;

void synth_free(synth_design *d) {
  if (!d) return;
  free(d->pin_kind); free(d->cell_type); free(d->cell_in_ptr); free(d->cell_in_pin);
  free(d->cell_out_pin); free(d->net_driver); free(d->net_sink_ptr); free(d->net_sink_pin);
  free(d->net_node_ptr); free(d->parent); free(d->res_kohm); free(d->cap_ff);
  free(d->sink_node); free(d->n_inputs); free(d->sense); free(d->pin_cap_ff);
  free(d->slew_axis); free(d->load_axis); free(d->tables); free(d->pi_at);
  free(d->pi_slew); free(d->po_rat);
  free(d);
}

static void shuffle_i32(sm64_t *g, int32_t *a, int64_t n) {
  for (int64_t i = n - 1; i > 0; i--) {
    int64_t j = below(g, i + 1);
    int32_t t = a[i]; a[i] = a[j]; a[j] = t;
  }
}

/* Geometric on {1,2,...} with mean mu (p = 1/mu), by inversion. */
static int64_t geometric(sm64_t *g, double mu) {
  if (mu <= 1.0) return 1;
  double p = 1.0 / mu;
  double u = u01(g);
  return 1 + (int64_t)floor(log1p(-u) / log1p(-p));
}

/* Draw a driver in [lo, hi) with probability proportional to remaining sink
 * slots; when that range has no slot left, uniformly over the range. */
static int64_t draw_driver(sm64_t *g, fenwick_t *fw, int64_t *rem, int64_t lo, int64_t hi) {
  int64_t plo = fw_prefix(fw, lo), tot = fw_prefix(fw, hi) - plo;
  int64_t pick;
  if (tot > 0) {
    pick = fw_find(fw, plo + below(g, tot));
  } else {
    pick = lo + below(g, hi - lo);
  }
  if (rem[pick] > 0) {
    rem[pick]--;
    fw_add(fw, pick, -1);
  }
  return pick;
}

/* Table values a + b*slew + c*load + U[-1,1], then made monotone (non-decreasing)
 * along both axes with a running max. */
static void make_table(sm64_t *g, float *T, const float *xs, const float *ys, int nx, int ny,
                       double a0, double a1, double b0, double b1, double c0, double c1) {
  double a = unif(g, a0, a1), b = unif(g, b0, b1), c = unif(g, c0, c1);
  for (int i = 0; i < nx; i++)
    for (int j = 0; j < ny; j++)
      T[i * ny + j] = (float)(a + b * xs[i] + c * ys[j] + unif(g, -1.0, 1.0));
  for (int i = 1; i < nx; i++)
    for (int j = 0; j < ny; j++)
      if (T[i * ny + j] < T[(i - 1) * ny + j]) T[i * ny + j] = T[(i - 1) * ny + j];
  for (int i = 0; i < nx; i++)
    for (int j = 1; j < ny; j++)
      if (T[i * ny + j] < T[i * ny + j - 1]) T[i * ny + j] = T[i * ny + j - 1];
}

synth_design *synth_generate(const synth_cfg *cfg) {
  const int64_t NC = cfg->n_cells;
  const int L = cfg->n_levels;
  const int64_t NPI = cfg->n_pi, NPO = cfg->n_po;
  if (NC < 1 || L < 1 || NPI < 1 || NPO < 0 || cfg->n_types < 1 || NC < L) return NULL;
  sm64_t g_lvl = stream(cfg->seed, 1), g_top = stream(cfg->seed, 2), g_rc = stream(cfg->seed, 3);
  sm64_t g_lib = stream(cfg->lib_seed ? cfg->lib_seed : cfg->seed, 4), g_shuf = stream(cfg->seed, 5);

  /* 1. level sizes */
  int64_t *lvl_size = (int64_t *)calloc((size_t)L + 2, sizeof(int64_t));
  {
    int32_t *is_heavy = (int32_t *)calloc((size_t)L + 2, sizeof(int32_t));
    int nh = cfg->n_heavy;
    if (nh > L - 1) nh = L - 1;
    if (nh > 0) {
      int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)L);
      int nc = 0;
      for (int l = 2; l <= L; l++) cand[nc++] = l;
      for (int i = 0; i < nh; i++) { /* partial Fisher-Yates */
        int j = i + (int)below(&g_lvl, nc - i);
        int32_t t = cand[i]; cand[i] = cand[j]; cand[j] = t;
        is_heavy[cand[i]] = 1;
      }
      free(cand);
    }
    int64_t heavy_n = nh > 0 ? (int64_t)llround(cfg->heavy_frac * (double)NC) : 0;
    int64_t rest = NC - heavy_n * nh;
    int nl = L - nh;
    for (int l = 1, k = 0; l <= L; l++) {
      if (is_heavy[l]) { lvl_size[l] = heavy_n; continue; }
      lvl_size[l] = rest / nl + (k < rest % nl ? 1 : 0);
      k++;
    }
    free(is_heavy);
  }
  /* cells in level order: cell c (natural index) at level lvl_of */
  int64_t *lvl_start = (int64_t *)calloc((size_t)L + 2, sizeof(int64_t));
  for (int l = 1; l <= L; l++) lvl_start[l + 1] = lvl_start[l] + lvl_size[l];
  lvl_start[0] = 0; /* unused for cells */

  int32_t *ctype = (int32_t *)malloc(sizeof(int32_t) * (size_t)NC);
  int32_t *cnin = (int32_t *)malloc(sizeof(int32_t) * (size_t)NC);
  int64_t *cin_ptr = (int64_t *)malloc(sizeof(int64_t) * ((size_t)NC + 1));
  cin_ptr[0] = 0;
  for (int64_t c = 0; c < NC; c++) {
    ctype[c] = (int32_t)below(&g_top, cfg->n_types);
    cnin[c] = 1 + ctype[c] % 3;
    cin_ptr[c + 1] = cin_ptr[c] + cnin[c];
  }
  const int64_t NCIN = cin_ptr[NC];

  /* 2. drivers: PIs then cells (natural order); fanout targets */
  const int64_t ND = NPI + NC;
  int64_t *rem = (int64_t *)malloc(sizeof(int64_t) * (size_t)ND);
  for (int64_t i = 0; i < ND; i++) {
    int64_t f = geometric(&g_top, cfg->fanout_mu);
    if (f > cfg->fanout_cap) f = cfg->fanout_cap;
    rem[i] = f;
  }
  if (cfg->n_hf > 0) { /* high-fanout nets, driven by PIs or level-1 cells */
    int64_t pool = NPI + lvl_size[1];
    int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)pool);
    for (int64_t i = 0; i < pool; i++) cand[i] = i;
    int64_t nh = cfg->n_hf < pool ? cfg->n_hf : pool;
    for (int64_t i = 0; i < nh; i++) {
      int64_t j = i + below(&g_top, pool - i);
      int64_t t = cand[i]; cand[i] = cand[j]; cand[j] = t;
      rem[cand[i]] = (int64_t)llround(exp(unif(&g_top, log((double)cfg->hf_min), log((double)cfg->hf_max))));
    }
    free(cand);
  }
  fenwick_t fw;
  fw_init(&fw, rem, ND);
  /* driver index range of cell level l: [NPI + lvl_start[l], NPI + lvl_start[l+1]) ; level 0: [0, NPI) */

  /* 3. connect cell inputs */
  int64_t *cin_drv = (int64_t *)malloc(sizeof(int64_t) * (size_t)(NCIN > 0 ? NCIN : 1));
  for (int l = 1; l <= L; l++) {
    int64_t prev_lo = (l == 1) ? 0 : NPI + lvl_start[l - 1];
    int64_t prev_hi = (l == 1) ? NPI : NPI + lvl_start[l];
    for (int64_t c = lvl_start[l]; c < lvl_start[l + 1]; c++) {
      for (int k = 0; k < cnin[c]; k++) {
        int64_t lo = (k == 0) ? prev_lo : 0;
        cin_drv[cin_ptr[c] + k] = draw_driver(&g_top, &fw, rem, lo, prev_hi);
      }
    }
  }
  /* 4. primary outputs on drivers of the last level */
  int64_t *po_drv = (int64_t *)malloc(sizeof(int64_t) * (size_t)(NPO > 0 ? NPO : 1));
  for (int64_t o = 0; o < NPO; o++)
    po_drv[o] = draw_driver(&g_top, &fw, rem, NPI + lvl_start[L], NPI + lvl_start[L + 1]);
  free(fw.t);
  free(rem);

  /* 5. pin ids.  natural: PIs, then per cell (inputs..., output), then POs */
  const int64_t NP = NPI + NCIN + NC + NPO;
  if (NP > INT32_MAX) return NULL;
  int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)NP);
  for (int64_t i = 0; i < NP; i++) perm[i] = (int32_t)i;
  if (cfg->shuffle) shuffle_i32(&g_shuf, perm, NP);
  /* natural pin index helpers */
#define PIN_PI(i) ((int64_t)(i))
#define PIN_CIN(c, k) (NPI + cin_ptr[c] + (c) + (k))
#define PIN_COUT(c) (NPI + cin_ptr[(c) + 1] + (c))
#define PIN_PO(o) (NPI + NCIN + NC + (o))

  synth_design *d = (synth_design *)calloc(1, sizeof(synth_design));
  d->n_pins = (int32_t)NP; d->n_cells = (int32_t)NC; d->n_nets = (int32_t)ND;
  d->n_pi = (int32_t)NPI; d->n_po = (int32_t)NPO; d->n_cell_in = (int32_t)NCIN;
  d->n_sinks = (int32_t)(NCIN + NPO);
  d->dangling_policy = cfg->dangling_policy;
  d->pin_kind = (int32_t *)malloc(sizeof(int32_t) * (size_t)NP);
  for (int64_t i = 0; i < NPI; i++) d->pin_kind[perm[PIN_PI(i)]] = 0;
  for (int64_t c = 0; c < NC; c++) {
    for (int k = 0; k < cnin[c]; k++) d->pin_kind[perm[PIN_CIN(c, k)]] = 1;
    d->pin_kind[perm[PIN_COUT(c)]] = 2;
  }
  for (int64_t o = 0; o < NPO; o++) d->pin_kind[perm[PIN_PO(o)]] = 3;

  /* cell order (optionally shuffled) */
  int32_t *corder = (int32_t *)malloc(sizeof(int32_t) * (size_t)NC);
  for (int64_t c = 0; c < NC; c++) corder[c] = (int32_t)c;
  if (cfg->shuffle) shuffle_i32(&g_shuf, corder, NC);
  d->cell_type = (int32_t *)malloc(sizeof(int32_t) * (size_t)NC);
  d->cell_in_ptr = (int32_t *)malloc(sizeof(int32_t) * ((size_t)NC + 1));
  d->cell_in_pin = (int32_t *)malloc(sizeof(int32_t) * (size_t)(NCIN > 0 ? NCIN : 1));
  d->cell_out_pin = (int32_t *)malloc(sizeof(int32_t) * (size_t)NC);
  d->cell_in_ptr[0] = 0;
  for (int64_t i = 0; i < NC; i++) {
    int64_t c = corder[i];
    d->cell_type[i] = ctype[c];
    int32_t p = d->cell_in_ptr[i];
    for (int k = 0; k < cnin[c]; k++) d->cell_in_pin[p + k] = perm[PIN_CIN(c, k)];
    d->cell_in_ptr[i + 1] = p + cnin[c];
    d->cell_out_pin[i] = perm[PIN_COUT(c)];
  }

  /* 6. nets: one per driver; sinks in creation order */
  int64_t *fo = (int64_t *)calloc((size_t)ND + 1, sizeof(int64_t));
  for (int64_t i = 0; i < NCIN; i++) fo[cin_drv[i] + 1]++;
  for (int64_t o = 0; o < NPO; o++) fo[po_drv[o] + 1]++;
  for (int64_t i = 0; i < ND; i++) fo[i + 1] += fo[i];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ND);
  memcpy(fill, fo, sizeof(int64_t) * (size_t)ND);
  int64_t *sink_nat = (int64_t *)malloc(sizeof(int64_t) * (size_t)(fo[ND] > 0 ? fo[ND] : 1));
  for (int64_t c = 0; c < NC; c++)
    for (int k = 0; k < cnin[c]; k++) sink_nat[fill[cin_drv[cin_ptr[c] + k]]++] = PIN_CIN(c, k);
  for (int64_t o = 0; o < NPO; o++) sink_nat[fill[po_drv[o]]++] = PIN_PO(o);
  free(fill);

  int32_t *norder = (int32_t *)malloc(sizeof(int32_t) * (size_t)ND);
  for (int64_t i = 0; i < ND; i++) norder[i] = (int32_t)i;
  if (cfg->shuffle) shuffle_i32(&g_shuf, norder, ND);
  d->net_driver = (int32_t *)malloc(sizeof(int32_t) * (size_t)ND);
  d->net_sink_ptr = (int32_t *)malloc(sizeof(int32_t) * ((size_t)ND + 1));
  d->net_sink_pin = (int32_t *)malloc(sizeof(int32_t) * (size_t)(d->n_sinks > 0 ? d->n_sinks : 1));
  d->net_sink_ptr[0] = 0;
  for (int64_t i = 0; i < ND; i++) {
    int64_t drv = norder[i];
    d->net_driver[i] = perm[drv < NPI ? PIN_PI(drv) : PIN_COUT(drv - NPI)];
    int32_t p = d->net_sink_ptr[i];
    for (int64_t s = fo[drv]; s < fo[drv + 1]; s++) d->net_sink_pin[p++] = perm[sink_nat[s]];
    d->net_sink_ptr[i + 1] = p;
  }

  /* 7. RC trees: root = driver (node 0, no segment).  Each sink hangs a chain of
   * U{2..6} internal nodes off a uniformly chosen existing non-sink node and ends
   * in its own leaf.  Per segment R ~ U[1,50] ohm, C ~ U[0.1,2] fF at the child.
   * Nodes are appended, so parent < child. */
  int64_t nn = 0;
  d->net_node_ptr = (int64_t *)malloc(sizeof(int64_t) * ((size_t)ND + 1));
  /* exact node count needs the chain lengths: draw them first, per sink */
  int8_t *chain = (int8_t *)malloc((size_t)(d->n_sinks > 0 ? d->n_sinks : 1));
  for (int64_t s = 0; s < d->n_sinks; s++) chain[s] = (int8_t)(2 + below(&g_rc, 5));
  d->net_node_ptr[0] = 0;
  for (int64_t i = 0; i < ND; i++) {
    int64_t cnt = 1;
    for (int32_t s = d->net_sink_ptr[i]; s < d->net_sink_ptr[i + 1]; s++) cnt += chain[s] + 1;
    d->net_node_ptr[i + 1] = d->net_node_ptr[i] + cnt;
  }
  nn = d->net_node_ptr[ND];
  d->n_nodes = nn;
  d->parent = (int32_t *)malloc(sizeof(int32_t) * (size_t)nn);
  d->res_kohm = (float *)malloc(sizeof(float) * (size_t)nn);
  d->cap_ff = (float *)malloc(sizeof(float) * (size_t)nn);
  d->sink_node = (int32_t *)malloc(sizeof(int32_t) * (size_t)(d->n_sinks > 0 ? d->n_sinks : 1));
  {
    int64_t maxn = 1;
    for (int64_t i = 0; i < ND; i++) {
      int64_t m = d->net_node_ptr[i + 1] - d->net_node_ptr[i];
      if (m > maxn) maxn = m;
    }
    int32_t *elig = (int32_t *)malloc(sizeof(int32_t) * (size_t)maxn);
    for (int64_t i = 0; i < ND; i++) {
      int64_t base = d->net_node_ptr[i];
      int32_t n = 0, ne = 0;
      d->parent[base] = -1; d->res_kohm[base] = 0.0f; d->cap_ff[base] = 0.0f;
      n = 1; elig[ne++] = 0;
      for (int32_t s = d->net_sink_ptr[i]; s < d->net_sink_ptr[i + 1]; s++) {
        int32_t at = elig[below(&g_rc, ne)];
        for (int k = 0; k <= chain[s]; k++) {
          d->parent[base + n] = at;
          d->res_kohm[base + n] = (float)(unif(&g_rc, 1.0, 50.0) / 1000.0);
          d->cap_ff[base + n] = (float)unif(&g_rc, 0.1, 2.0);
          if (k < chain[s]) elig[ne++] = n;
          at = n;
          n++;
        }
        d->sink_node[s] = at;
      }
    }
    free(elig);
  }
  free(chain);

  /* 8. library: type t has 1 + (t mod 3) inputs; unateness cycles negative,
   * positive, negative, non-unate; geometric axes slew 5..300 ps, load 0.5..50 fF */
  const int T = cfg->n_types, NX = 7, NY = 7;
  d->n_types = T; d->nx = NX; d->ny = NY; d->po_cap_ff = (float)cfg->po_cap_ff;
  d->n_inputs = (int32_t *)malloc(sizeof(int32_t) * (size_t)T);
  d->sense = (int32_t *)malloc(sizeof(int32_t) * (size_t)T);
  d->pin_cap_ff = (float *)malloc(sizeof(float) * (size_t)T);
  d->slew_axis = (float *)malloc(sizeof(float) * (size_t)T * NX);
  d->load_axis = (float *)malloc(sizeof(float) * (size_t)T * NY);
  d->tables = (float *)malloc(sizeof(float) * (size_t)T * 4 * NX * NY);
  static const int32_t sense_cycle[4] = {1, 0, 1, 2};
  for (int t = 0; t < T; t++) {
    d->n_inputs[t] = 1 + t % 3;
    d->sense[t] = sense_cycle[t % 4];
    d->pin_cap_ff[t] = (float)unif(&g_lib, 0.5, 3.0);
    for (int i = 0; i < NX; i++) d->slew_axis[t * NX + i] = (float)(5.0 * pow(60.0, i / 6.0));
    for (int j = 0; j < NY; j++) d->load_axis[t * NY + j] = (float)(0.5 * pow(100.0, j / 6.0));
    const float *xs = d->slew_axis + t * NX, *ys = d->load_axis + t * NY;
    float *tb = d->tables + (size_t)t * 4 * NX * NY;
    make_table(&g_lib, tb + 0 * NX * NY, xs, ys, NX, NY, 5, 25, 0.05, 0.25, 0.5, 2.5); /* cell_rise */
    make_table(&g_lib, tb + 1 * NX * NY, xs, ys, NX, NY, 5, 25, 0.05, 0.25, 0.5, 2.5); /* cell_fall */
    make_table(&g_lib, tb + 2 * NX * NY, xs, ys, NX, NY, 3, 12, 0.02, 0.15, 1.0, 4.0); /* rise_tr */
    make_table(&g_lib, tb + 3 * NX * NY, xs, ys, NX, NY, 3, 12, 0.02, 0.15, 1.0, 4.0); /* fall_tr */
  }

  /* 9. constraints, per PI / PO ranked by pin id */
  d->pi_at = (float *)malloc(sizeof(float) * (size_t)NPI * 4);
  d->pi_slew = (float *)malloc(sizeof(float) * (size_t)NPI * 4);
  d->po_rat = (float *)malloc(sizeof(float) * (size_t)(NPO > 0 ? NPO : 1) * 4);
  for (int64_t i = 0; i < NPI * 4; i++) { d->pi_at[i] = (float)cfg->pi_at_ps; d->pi_slew[i] = (float)cfg->pi_slew_ps; }
  /* views 0,1 early (rise, fall); 2,3 late */
  for (int64_t i = 0; i < NPO * 4; i++) d->po_rat[i] = (float)((i % 4) < 2 ? cfg->rat_early_ps : cfg->rat_ps);
  for (int v = 0; v < 4; v++) d->dangling_rat[v] = (float)(v < 2 ? cfg->rat_early_ps : cfg->rat_ps);

  free(perm); free(corder); free(norder); free(fo); free(sink_nat); free(cin_drv); free(po_drv);
  free(ctype); free(cnin); free(cin_ptr); free(lvl_size); free(lvl_start);
  return d;
#undef PIN_PI
#undef PIN_CIN
#undef PIN_COUT
#undef PIN_PO
}
