"""Pins for the FP64 oracle: closed forms, brute force, hand derivations and
invariants that do not reuse the oracle's own formulation.

RC (Elmore, §III "Delay models"): uniform-chain closed form, single-pole case,
O(n^2) shared-path-resistance sums on random trees, non-negative spread.
NLDM (Table I): exactness on bilinear surfaces including extrapolation.
Propagation (§I/§III graph-based STA, "Report options" slacks and WNS/TNS):
hand-derived 3-gate chain, brute-force path enumeration on tiny DAGs, slack
identities, constant slack along the worst critical path, monotonicity.
"""
import numpy as np
import pytest

import oracle
from designs import (CIN, COUT, PI, PO, LOAD_AXIS, SLEW_AXIS, make_design, planar_table,
                     random_tree, single_segment_net)
from paper_2511_11660_amd import synth



# ------------------------------------------------------------------ RC pins

def test_rc_uniform_chain_closed_form():
    """Chain of n segments (R, C at each child): load(k) = (n-k+1)C and
    d(k) = RC(k(n+1) - k(k+1)/2), so d(n) = RC n(n+1)/2 and L_net = nC."""
    for n in (1, 2, 5, 17):
        R, C = 0.013, 1.7
        parent = [-1] + list(range(n))
        Rv = [0.0] + [R] * n
        Cv = [0.0] + [C] * n
        load, d, _, _ = oracle.rc_tree(parent, Rv, Cv)
        for k in range(1, n + 1):
            assert load[k] == pytest.approx((n - k + 1) * C, rel=1e-14)
            assert d[k] == pytest.approx(R * C * (k * (n + 1) - k * (k + 1) / 2), rel=1e-13)
        assert load[0] == pytest.approx(n * C, rel=1e-14)
        assert d[n] == pytest.approx(R * C * n * (n + 1) / 2, rel=1e-13)


def test_rc_single_pole():
    """One segment: d = RC, m2 = (RC)^2, spread q = 2 m2 - d^2 = (RC)^2."""
    R, C = 0.04, 3.5
    load, d, ld, m2 = oracle.rc_tree([-1, 0], [0.0, R], [0.0, C])
    assert d[1] == pytest.approx(R * C, rel=1e-15)
    assert m2[1] == pytest.approx((R * C) ** 2, rel=1e-15)
    assert 2 * m2[1] - d[1] ** 2 == pytest.approx((R * C) ** 2, rel=1e-14)


def _brute_moments(parent, R, Chat):
    """d_k = sum_j R_kj Chat_j and m2_k = sum_j R_kj Chat_j d_j, with R_kj the
    resistance of the segments shared by the root->k and root->j paths."""
    n = len(parent)
    paths = []
    for k in range(n):
        s, x = set(), k
        while x > 0:
            s.add(x)
            x = parent[x]
        paths.append(s)
    Rkj = np.zeros((n, n))
    for k in range(n):
        for j in range(n):
            Rkj[k, j] = sum(R[a] for a in paths[k] & paths[j])
    d = Rkj @ np.asarray(Chat)
    m2 = Rkj @ (np.asarray(Chat) * d)
    return d, m2


@pytest.mark.parametrize("seed", range(12))
def test_rc_random_tree_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 31))
    parent = random_tree(rng, n)
    R = [0.0] + list(rng.uniform(0.001, 0.05, n - 1))
    Chat = list(rng.uniform(0.1, 3.0, n))
    load, d, ld, m2 = oracle.rc_tree(parent, R, Chat)
    bd, bm2 = _brute_moments(parent, R, Chat)
    np.testing.assert_allclose(d, bd, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m2, bm2, rtol=1e-12, atol=1e-18)
    assert load[0] == pytest.approx(sum(Chat), rel=1e-14)
    # the impulse-response spread is non-negative before any clamp
    assert np.all(2 * m2 - d * d >= -1e-12 * np.maximum(1.0, d * d))


def test_rc_net_load_is_total_cap():
    """L_net = wire caps + receiving pin caps of the net, on a generated design."""
    d = synth.generate(synth.tiny_config())
    L, dd, q = oracle.rc(d)
    cell_of = np.full(d.n_pins, -1)
    for c in range(d.n_cells):
        cell_of[d.cell_in_pin[d.cell_in_ptr[c]:d.cell_in_ptr[c + 1]]] = c
    for n in range(0, d.n_nets, 37):
        a, b = d.net_node_ptr[n], d.net_node_ptr[n + 1]
        tot = float(d.cap_ff[a:b].astype(np.float64).sum())
        for s in range(d.net_sink_ptr[n], d.net_sink_ptr[n + 1]):
            p = d.net_sink_pin[s]
            tot += d.po_cap_ff if d.pin_kind[p] == PO else float(d.pin_cap_ff[d.cell_type[cell_of[p]]])
        assert L[n] == pytest.approx(tot, rel=1e-12)
    assert np.all(q >= 0)


# ---------------------------------------------------------------- NLDM pins

def test_nldm_exact_on_bilinear_surfaces():
    rng = np.random.default_rng(7)
    for _ in range(5):
        a, b, c, e = rng.uniform(-10, 10), rng.uniform(-1, 1), rng.uniform(-3, 3), rng.uniform(-0.01, 0.01)
        T = planar_table(a, b, c, e)
        f = lambda X, Y: a + b * X + c * Y + e * X * Y  # noqa: E731
        # grid nodes
        for i in range(7):
            for j in range(7):
                X, Y = float(SLEW_AXIS[i]), float(LOAD_AXIS[j])
                assert oracle.nldm(SLEW_AXIS, LOAD_AXIS, T, X, Y) == pytest.approx(T[i, j], abs=1e-9)
        # inside and outside the table (boundary-segment extrapolation)
        for X, Y in [(1.0, 0.1), (3.0, 70.0), (400.0, 0.2), (500.0, 120.0), (42.0, 7.7),
                     (5.0, 50.0), (299.0, 0.6), (-3.0, -1.0)]:
            got = oracle.nldm(SLEW_AXIS, LOAD_AXIS, T, X, Y)
            # the float32 table holds f rounded at the grid; compare to f itself
            assert got == pytest.approx(f(X, Y), rel=2e-6, abs=2e-4)


def test_nldm_monotone_for_monotone_table():
    """Monotone in each axis (extrapolation included) while the other axis stays
    on the table; outside it, bilinear weights turn negative and no claim holds."""
    d = synth.generate(synth.tiny_config())
    T = d.tables[3, 0]
    wide_x, in_x = np.linspace(1.0, 400.0, 60), np.linspace(5.0, 300.0, 40)
    wide_y, in_y = np.linspace(0.1, 80.0, 60), np.linspace(0.5, 50.0, 40)
    f = lambda x, y: oracle.nldm(d.slew_axis[3], d.load_axis[3], T, x, y)  # noqa: E731
    vx = np.array([[f(x, y) for y in in_y] for x in wide_x])
    vy = np.array([[f(x, y) for y in wide_y] for x in in_x])
    assert np.all(np.diff(vx, axis=0) >= -1e-9)
    assert np.all(np.diff(vy, axis=1) >= -1e-9)


# ------------------------------------------------------- worked 3-gate chain

def _chain_design():
    # pins: 0 PI1, 1 PI2, 2 INV.A, 3 INV.Y, 4 NAND.A, 5 NAND.B, 6 NAND.Y, 7 BUF.A, 8 BUF.Y, 9 PO
    kinds = [PI, PI, CIN, COUT, CIN, CIN, COUT, CIN, COUT, PO]
    cells = [(0, [2], 3), (1, [4, 5], 6), (2, [7], 8)]
    R, C = 0.015625, 1.5  # exactly representable in float32
    nets = [single_segment_net(0, [2], R, C), single_segment_net(1, [5], R, C),
            single_segment_net(3, [4], R, C), single_segment_net(6, [7], R, C),
            single_segment_net(8, [9], R, C)]
    coef = {  # per type: (delay a,b,c) rise/fall and (slew a,b,c) rise/fall
        0: [(8.0, 0.10, 1.2), (6.0, 0.12, 1.0), (4.0, 0.05, 2.0), (3.5, 0.04, 1.8)],
        1: [(12.0, 0.15, 1.5), (10.0, 0.11, 1.7), (5.0, 0.06, 2.5), (4.5, 0.07, 2.2)],
        2: [(15.0, 0.08, 0.9), (14.0, 0.09, 0.8), (3.0, 0.03, 1.5), (2.5, 0.02, 1.4)],
    }
    tables = np.stack([np.stack([planar_table(*coef[t][k]) for k in range(4)]) for t in range(3)])
    pin_cap = [1.125, 1.625, 0.875]
    d = make_design(kinds, cells, nets, n_inputs=[1, 2, 1], sense=[1, 1, 0], pin_cap=pin_cap,
                    tables=tables, pi_at=0.0, pi_slew=20.0, po_rat=500.0, po_cap=2.0)
    return d, coef, pin_cap, R, C


def test_worked_three_gate_chain():
    """PI1 -> INV -> NAND2 (B from PI2) -> BUF -> PO with planar tables and
    one-segment nets, propagated by hand below (closed forms per stage).  The
    tables are float32 samples of planes, so the tolerance is the float32
    rounding of the table entries (a few 1e-6 ps), not the FP64 arithmetic."""
    d, coef, pin_cap, R, C = _chain_design()
    r = oracle.sta(d)

    def lin(t, k, X, Y):
        a, b, c = coef[t][k]
        return a + b * X + c * Y

    # one-segment net with receiving cap p: load = C + p, d = R(C+p), q = d^2
    def net(p):
        load = C + p
        dd = R * load
        return load, dd, dd * dd

    L_inv, d_inv_a, q_inv_a = net(pin_cap[0])       # PI1 -> INV.A
    _, d_nand_b, q_nand_b = net(pin_cap[1])         # PI2 -> NAND.B
    L_nand_in, d_nand_a, q_nand_a = net(pin_cap[1])  # INV.Y -> NAND.A (load of INV.Y)
    L_buf_in, d_buf_a, q_buf_a = net(pin_cap[2])     # NAND.Y -> BUF.A (load of NAND.Y)
    L_po, d_po, q_po = net(2.0)                      # BUF.Y -> PO
    # output loads: INV.Y drives NAND.A, NAND.Y drives BUF.A, BUF.Y drives PO
    L_invY, L_nandY, L_bufY = L_nand_in, L_buf_in, L_po

    E = {}
    for el in (0, 1):
        for rf in (0, 1):
            v = 2 * el + rf
            E[("pi", v)] = (0.0, 20.0)
    AT = np.zeros((10, 4))
    SL = np.zeros((10, 4))
    AT[0] = AT[1] = 0.0
    SL[0] = SL[1] = 20.0
    AT[2] = AT[0] + d_inv_a
    SL[2] = np.sqrt(20.0 ** 2 + q_inv_a)
    AT[5] = AT[1] + d_nand_b
    SL[5] = np.sqrt(20.0 ** 2 + q_nand_b)
    for el in (0, 1):
        for ro in (0, 1):
            ri = 1 - ro  # INV negative unate
            x = SL[2, 2 * el + ri]
            AT[3, 2 * el + ro] = AT[2, 2 * el + ri] + lin(0, ro, x, L_invY)
            SL[3, 2 * el + ro] = lin(0, 2 + ro, x, L_invY)
    AT[4] = AT[3] + d_nand_a
    SL[4] = np.sqrt(SL[3] ** 2 + q_nand_a)
    crit_nand = np.zeros(4, int)
    for el in (0, 1):
        for ro in (0, 1):
            ri = 1 - ro  # NAND2 negative unate
            cands = []
            for k, pin in enumerate((4, 5)):
                x = SL[pin, 2 * el + ri]
                cands.append((AT[pin, 2 * el + ri] + lin(1, ro, x, L_nandY), lin(1, 2 + ro, x, L_nandY),
                              2 * k + ri))
            pick = max if el else min
            best = pick(cands, key=lambda c: c[0])
            AT[6, 2 * el + ro] = best[0]
            crit_nand[2 * el + ro] = best[2]
            SL[6, 2 * el + ro] = pick(c[1] for c in cands)
    AT[7] = AT[6] + d_buf_a
    SL[7] = np.sqrt(SL[6] ** 2 + q_buf_a)
    for el in (0, 1):
        for ro in (0, 1):
            x = SL[7, 2 * el + ro]  # BUF positive unate
            AT[8, 2 * el + ro] = AT[7, 2 * el + ro] + lin(2, ro, x, L_bufY)
            SL[8, 2 * el + ro] = lin(2, 2 + ro, x, L_bufY)
    AT[9] = AT[8] + d_po
    SL[9] = np.sqrt(SL[8] ** 2 + q_po)
    tol = dict(rtol=0, atol=2e-5)
    np.testing.assert_allclose(r["at"], AT, **tol)
    np.testing.assert_allclose(r["slew"], SL, **tol)
    np.testing.assert_array_equal(r["crit"][6], crit_nand)

    # backward
    RAT = np.zeros((10, 4))
    RAT[9] = 500.0
    RAT[8] = RAT[9] - d_po
    for el in (0, 1):
        for ri in (0, 1):
            x = SL[7, 2 * el + ri]
            RAT[7, 2 * el + ri] = RAT[8, 2 * el + ri] - lin(2, ri, x, L_bufY)
    RAT[6] = RAT[7] - d_buf_a
    for pin in (4, 5):
        for el in (0, 1):
            for ri in (0, 1):
                ro = 1 - ri
                x = SL[pin, 2 * el + ri]
                RAT[pin, 2 * el + ri] = RAT[6, 2 * el + ro] - lin(1, ro, x, L_nandY)
    RAT[3] = RAT[4] - d_nand_a
    RAT[1] = RAT[5] - d_nand_b
    for el in (0, 1):
        for ri in (0, 1):
            ro = 1 - ri
            x = SL[2, 2 * el + ri]
            RAT[2, 2 * el + ri] = RAT[3, 2 * el + ro] - lin(0, ro, x, L_invY)
    RAT[0] = RAT[2] - d_inv_a
    np.testing.assert_allclose(r["rat"], RAT, **tol)
    SLK = RAT - AT
    SLK[:, :2] = AT[:, :2] - RAT[:, :2]
    np.testing.assert_allclose(r["slack"], SLK, **tol)
    # one endpoint (the PO); WNS/TNS clamp at zero
    assert r["n_ep"] == 1 and r["ep_pin"][0] == 9
    for el in (0, 1):
        s = min(SLK[9, 2 * el], SLK[9, 2 * el + 1])
        assert r["ep_slack"][0, el] == pytest.approx(s, abs=2e-5)
        assert r["wns"][el] == pytest.approx(min(0.0, s), abs=2e-5)
        assert r["tns"][el] == pytest.approx(min(0.0, s), abs=2e-5)
    # levels: PIs 0, INV.A 1, INV.Y 2, NAND.A 3, NAND.B 1, NAND.Y 4, BUF.A 5, BUF.Y 6, PO 7
    np.testing.assert_array_equal(r["level"], [0, 0, 1, 2, 3, 1, 4, 5, 6, 7])
    np.testing.assert_array_equal(r["level_order"], [0, 1, 2, 5, 3, 4, 6, 7, 8, 9])


# --------------------------------------------- brute-force path enumeration

def _const_tables(rng, n_types):
    """Delay and slew tables that do not depend on slew or load."""
    t = np.zeros((n_types, 4, 7, 7), np.float32)
    for ty in range(n_types):
        for k in range(4):
            t[ty, k] = np.float32(rng.uniform(1.0, 30.0))
    return t


def _tiny_dag(seed, dangling):
    cfg = synth.SynthConfig(n_cells=int(6 + seed % 7), n_levels=3 + seed % 2, n_pi=3, n_po=2,
                            fanout_mu=2.0, fanout_cap=4, n_types=8, rat_ps=90.0,
                            rat_early_ps=30.0, dangling_policy=dangling, shuffle=1, seed=100 + seed)
    d = synth.generate(cfg)
    rng = np.random.default_rng(seed)
    d.tables = _const_tables(rng, d.n_types)
    d.res_kohm[:] = 0.0  # no wire delay, no net spread
    d.pi_at[:] = rng.uniform(0, 5, d.pi_at.shape).astype(np.float32)
    return d


def _arcs(d):
    """Timing arcs as (from_pin, from_rf, to_pin, to_rf, delay)."""
    cell_of = {}
    for c in range(d.n_cells):
        for k in range(d.cell_in_ptr[c], d.cell_in_ptr[c + 1]):
            cell_of[int(d.cell_in_pin[k])] = c
    arcs = []
    for n in range(d.n_nets):
        for s in range(d.net_sink_ptr[n], d.net_sink_ptr[n + 1]):
            for rf in (0, 1):
                arcs.append((int(d.net_driver[n]), rf, int(d.net_sink_pin[s]), rf, 0.0))
    for c in range(d.n_cells):
        t = d.cell_type[c]
        sense = d.sense[t]
        for k in range(d.cell_in_ptr[c], d.cell_in_ptr[c + 1]):
            for ri in (0, 1):
                for ro in (0, 1):
                    ok = (sense == 0 and ri == ro) or (sense == 1 and ri != ro) or sense == 2
                    if ok:
                        arcs.append((int(d.cell_in_pin[k]), ri, int(d.cell_out_pin[c]), ro,
                                     float(d.tables[t, ro, 0, 0])))
    return arcs


def _enumerate_paths(d):
    """All paths, as lists of arcs, starting at a PI (either transition)."""
    arcs = _arcs(d)
    out = {}
    for a in arcs:
        out.setdefault((a[0], a[1]), []).append(a)
    paths = []

    def walk(node, acc):
        paths.append((node, acc))
        for a in out.get(node, []):
            walk((a[2], a[3]), acc + [a])

    for p in range(d.n_pins):
        if d.pin_kind[p] == PI:
            for rf in (0, 1):
                walk((p, rf), [])
    return paths


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("dangling", [0, 1])
def test_brute_force_paths(seed, dangling):
    d = _tiny_dag(seed, dangling)
    r = oracle.sta(d)
    paths = _enumerate_paths(d)
    pi_rank = {int(p): i for i, p in enumerate(np.flatnonzero(d.pin_kind == PI))}
    # arrival: late = max, early = min over all PI -> (pin, rf) paths
    late, early, longest = {}, {}, {}
    for (pin, rf), acc in paths:
        start = acc[0][0] if acc else pin
        t = float(d.pi_at[pi_rank[start], 2 + (acc[0][1] if acc else rf)]) + sum(a[4] for a in acc)
        te = float(d.pi_at[pi_rank[start], (acc[0][1] if acc else rf)]) + sum(a[4] for a in acc)
        late[(pin, rf)] = max(late.get((pin, rf), -np.inf), t)
        early[(pin, rf)] = min(early.get((pin, rf), np.inf), te)
        longest[pin] = max(longest.get(pin, 0), len(acc))
    for (pin, rf), v in late.items():
        assert r["at"][pin, 2 + rf] == pytest.approx(v, abs=1e-9)
        assert r["at"][pin, rf] == pytest.approx(early[(pin, rf)], abs=1e-9)
    for p in range(d.n_pins):
        assert r["level"][p] == longest[p]
    # required time: dual enumeration from each (pin, rf) to an endpoint
    eps = set(int(p) for p in r["ep_pin"])
    rat_of = {}
    po_rank = {int(p): i for i, p in enumerate(np.flatnonzero(d.pin_kind == PO))}
    for p in eps:
        for v in range(4):
            rat_of[(p, v)] = float(d.po_rat[po_rank[p], v]) if d.pin_kind[p] == PO else float(d.dangling_rat[v])
    arcs = _arcs(d)
    out = {}
    for a in arcs:
        out.setdefault((a[0], a[1]), []).append(a)

    def suffixes(node):
        """(endpoint, rf, summed delay) for every path from node to an endpoint."""
        res = []
        if node[0] in eps:
            res.append((node[0], node[1], 0.0))
        for a in out.get(node, []):
            for (e, erf, s) in suffixes((a[2], a[3])):
                res.append((e, erf, s + a[4]))
        return res

    for p in range(d.n_pins):
        for rf in (0, 1):
            suf = suffixes((p, rf))
            want_l = min((rat_of[(e, 2 + erf)] - s for e, erf, s in suf), default=np.inf)
            want_e = max((rat_of[(e, erf)] - s for e, erf, s in suf), default=-np.inf)
            assert r["rat"][p, 2 + rf] == pytest.approx(want_l, abs=1e-9)
            assert r["rat"][p, rf] == pytest.approx(want_e, abs=1e-9)


def test_levelize_detects_cycle():
    # PI0 -> A.in0 ; A(out 3) -> B.in (4) ; B(out 5) -> A.in1 (2); A has inputs 1, 2
    kinds = [PI, CIN, CIN, COUT, CIN, COUT]
    cells = [(1, [1, 2], 3), (0, [4], 5)]
    nets = [single_segment_net(0, [1], 0.01, 1.0), single_segment_net(3, [4], 0.01, 1.0),
            single_segment_net(5, [2], 0.01, 1.0)]
    tables = np.stack([np.stack([planar_table(5, 0.1, 1.0)] * 4)] * 2)
    d = make_design(kinds, cells, nets, n_inputs=[1, 2], sense=[0, 1], pin_cap=[1.0, 1.0],
                    tables=tables)
    with pytest.raises(ValueError):
        oracle.levelize(d)


# ------------------------------------------------------------- identities

@pytest.fixture(scope="module")
def tiny_result():
    d = synth.generate(synth.tiny_config())
    return d, oracle.sta(d)


@pytest.fixture(scope="module")
def small_mid_result():
    d = synth.generate(synth.mid_config(n_cells=20_000, n_levels=30, seed=11))
    return d, oracle.sta(d)


@pytest.mark.parametrize("which", ["tiny_result", "small_mid_result"])
def test_slack_identities(which, request):
    d, r = request.getfixturevalue(which)
    at, rat, slk = r["at"], r["rat"], r["slack"]
    fin = np.isfinite(rat)
    np.testing.assert_allclose(slk[:, 2:][fin[:, 2:]], (rat - at)[:, 2:][fin[:, 2:]], rtol=0, atol=1e-9)
    np.testing.assert_allclose(slk[:, :2][fin[:, :2]], (at - rat)[:, :2][fin[:, :2]], rtol=0, atol=1e-9)
    assert np.all(slk[~fin] == np.inf)
    es = r["ep_slack"]
    for el in (0, 1):
        assert r["wns"][el] <= 0.0
        assert r["tns"][el] <= r["wns"][el] + 1e-9
        assert np.all(es[:, el] >= r["wns"][el] - 1e-9)
        neg = es[:, el][es[:, el] < 0]
        assert r["tns"][el] == pytest.approx(neg.sum(), rel=1e-12, abs=1e-9)
        if np.all(es[:, el] >= 0):
            assert r["wns"][el] == 0.0
        # endpoint order: ascending (slack, pin id)
        o = r["ep_order"][el]
        keys = list(zip(es[o, el], r["ep_pin"][o]))
        assert keys == sorted(keys)
        assert sorted(o.tolist()) == list(range(r["n_ep"]))


@pytest.mark.parametrize("which", ["tiny_result", "small_mid_result"])
def test_worst_critical_path_has_constant_slack(which, request):
    """Following critical fanins back from the worst late endpoint, every pin's
    late slack equals the endpoint's (AT and RAT are consistent)."""
    d, r = request.getfixturevalue(which)
    drv_of_sink = {}
    for n in range(d.n_nets):
        for s in range(d.net_sink_ptr[n], d.net_sink_ptr[n + 1]):
            drv_of_sink[int(d.net_sink_pin[s])] = int(d.net_driver[n])
    cell_of_out = {int(p): c for c, p in enumerate(d.cell_out_pin)}
    e = r["ep_order"][1][0]
    p = int(r["ep_pin"][e])
    v = 2 + int(np.argmin(r["slack"][p, 2:]))
    target = r["slack"][p, v]
    steps = 0
    while d.pin_kind[p] != PI:
        assert r["slack"][p, v] == pytest.approx(target, abs=1e-7)
        if d.pin_kind[p] in (CIN, PO):
            p = drv_of_sink[p]
        else:
            c = cell_of_out[p]
            k = int(r["crit"][p, v])
            assert k >= 0
            p = int(d.cell_in_pin[d.cell_in_ptr[c] + k // 2])
            v = 2 + k % 2
        steps += 1
    assert r["slack"][p, v] == pytest.approx(target, abs=1e-7)
    assert steps > 5


# ---------------------------------------------------------- monotonicity

def test_late_at_monotone_in_arc_delay_slew_and_load():
    base = synth.generate(synth.tiny_config(seed=5))
    r0 = oracle.sta(base)
    # arc delay: raise one type's delay tables
    d1 = base.copy()
    d1.tables[3, 0:2] += np.float32(4.0)
    r1 = oracle.sta(d1)
    assert np.all(r1["at"][:, 2:] >= r0["at"][:, 2:] - 1e-9)
    assert np.any(r1["at"][:, 2:] > r0["at"][:, 2:] + 1e-6)
    # PI slew
    d2 = base.copy()
    d2.pi_slew[:] = 60.0
    r2 = oracle.sta(d2)
    assert np.all(r2["at"][:, 2:] >= r0["at"][:, 2:] - 1e-9)
    # load with no wire resistance (only the driver's NLDM load changes)
    d3 = base.copy()
    d3.res_kohm[:] = 0.0
    r3 = oracle.sta(d3)
    d4 = d3.copy()
    d4.cap_ff[d4.cap_ff > 0] += np.float32(0.5)
    r4 = oracle.sta(d4)
    assert np.all(r4["at"][:, 2:] >= r3["at"][:, 2:] - 1e-9)
    assert np.any(r4["at"][:, 2:] > r3["at"][:, 2:] + 1e-6)


def test_wire_cap_override_matches_design_caps():
    d = synth.generate(synth.tiny_config())
    r0 = oracle.sta(d)
    r1 = oracle.sta(d, wire_cap=d.cap_ff.astype(np.float64))
    np.testing.assert_array_equal(r0["at"], r1["at"])


def test_critical_fanin_tie_rule():
    """Exact ties go to the lowest fanin position, then to the rising input
    transition (R17): NAND2 inputs on identical branches, a non-unate cell
    whose rise and fall candidates coincide, and an AND3 whose B and C tie for
    the latest arrival while A is the earliest."""
    from designs import tie_design
    d = tie_design()
    r = oracle.sta(d)
    at = r["at"]
    np.testing.assert_array_equal(at[2], at[3])   # identical branches
    np.testing.assert_array_equal(at[8], at[9])
    assert at[5, 0] == at[5, 1] and at[5, 2] == at[5, 3]
    for v in range(4):
        ro = v % 2
        assert r["crit"][4, v] == 0 * 2 + (1 - ro)    # NAND2: input A, opposite transition
        assert r["crit"][6, v] == 0                  # non-unate: rise before fall
    assert list(r["crit"][10, 2:]) == [2 * 1 + 0, 2 * 1 + 1]   # AND3 late: B (tie with C)
    assert list(r["crit"][10, :2]) == [0, 1]                  # AND3 early: A
    assert at[7, 2] < at[8, 2]
