"""Arnoldi reduced-order net delay, CPU oracle.  TEST INFRASTRUCTURE ONLY
(same rule as the rest of ``oracle/``: only tests, the smoke check and the
benchmark's CPU baseline may use it).

§III "Delay models": besides Elmore the timer offers a reduced-order model
built by Arnoldi iterations, the more accurate choice late in a flow.  The
paper gives no formulas; this is the reading documented with the build, a
Krylov projection of the RC tree written out with dense FP64 matrices:

* unknowns are the non-root nodes of a net's tree (the root is driven by an
  ideal unit step); C = diag of the node caps (wire cap plus receiving pin
  caps), and G^-1 is the tree's resistance matrix, (G^-1)_ij = resistance
  shared by the root->i and root->j paths, so A = G^-1 C needs no division by a
  segment resistance and zero-resistance segments are allowed;
* the step response is Y(t) = 1 - z(t) with z(s) = (I + s A)^-1 d, d = A 1 the
  Elmore delays;
* the Arnoldi process on A in the G inner product (where A is self-adjoint,
  so it is the Lanczos three-term recurrence) from q1 = d / |d|_G builds the
  G-orthonormal basis Q of the Krylov space {d, A d} and T = Q^T G A Q; for
  vectors in the range of A, <A x, A y>_G = x^T C A y, so G itself is never
  formed;
* the projected response z_i(s) = |d|_G e_i^T Q (I + s T)^-1 e_1 gives, with
  T = U diag(tau) U^T, 1 - Y_i(t) = sum_j a_ij exp(-t / tau_j),
  a_ij = |d|_G (Q u_j)_i u_1j / tau_j; its first two time moments are exactly
  the node's Elmore delay d_i and second moment m2_i = (A d)_i;
* the delay is the first time the response reaches one half: 0 if
  Y_i(0) >= 1/2, else found by bisection (64 halvings of [0, t_hi], t_hi the
  first doubling of tau_max with 1 - Y_i(t_hi) < 1/2);
* an invariant Krylov space of dimension 1 (|r|_G = 0 after the first step,
  e.g. a single RC) gives the one-pole model; a net without resistance or
  capacitance (d = 0) has delay 0.
"""
from __future__ import annotations

import numpy as np


def shared_resistance(parent, R):
    """Dense (m-1) x (m-1) matrix of resistances shared by root paths of the
    non-root nodes 1..m-1 (parent[k] < k, node 0 the root): with P[i, k] = 1
    when segment k lies on the root->i path, Rs = P diag(R) P^T."""
    m = len(parent)
    P = np.zeros((m, m))
    for k in range(1, m):
        P[k] = P[parent[k]]
        P[k, k] = 1.0
    R = np.asarray(R, np.float64)
    return (P[1:] * R[None, :]) @ P[1:].T


def model(parent, R, Chat):
    """(a [n, J], tau [J]) of the reduced step response of every non-root
    node, J <= 2 poles; None when d = 0 everywhere."""
    R = np.asarray(R, np.float64)
    Cv = np.asarray(Chat, np.float64)[1:]
    A = shared_resistance(parent, R) @ np.diag(Cv)
    n = A.shape[0]
    one = np.ones(n)
    d = A @ one

    def ip(x, y):  # <A x, A y>_G from the pre-images x, y
        return float(x @ (Cv * (A @ y)))

    b0sq = ip(one, one)
    if b0sq <= 0.0:
        return None
    b0 = np.sqrt(b0sq)
    # q1 = d / b0 = A (1 / b0); pre-image p1
    p1 = one / b0
    q1 = A @ p1
    alpha1 = ip(p1, q1)  # <q1, A q1>_G, with A q1 = A (q1) as the pre-image
    # r1 = A q1 - alpha1 q1 = A (q1 - alpha1 p1)
    pr = q1 - alpha1 * p1
    b1sq = ip(pr, pr)
    if b1sq <= 1e-24 * alpha1 * alpha1:  # invariant: one pole
        T = np.array([[alpha1]])
        Q = q1[:, None]
    else:
        b1 = np.sqrt(b1sq)
        p2 = pr / b1
        q2 = A @ p2
        alpha2 = ip(p2, q2)
        T = np.array([[alpha1, b1], [b1, alpha2]])
        Q = np.stack([q1, q2], axis=1)
    tau, U = np.linalg.eigh(T)
    keep = tau > 0.0
    a = b0 * (Q @ U)[:, keep] * U[0, keep][None, :] / tau[keep][None, :]
    return a, tau[keep]


def half_time(a_i, tau):
    """First t >= 0 with sum_j a_ij exp(-t/tau_j) <= 1/2 (see the module
    docstring for the bracket and the bisection)."""
    f = lambda t: float(np.sum(a_i * np.exp(-t / tau))) - 0.5  # noqa: E731
    if f(0.0) <= 0.0:
        return 0.0
    hi = float(tau.max())
    while f(hi) > 0.0:
        hi *= 2.0
    lo = 0.0
    for _ in range(64):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def net_delays(parent, R, Chat, nodes):
    """Reduced-order 50% delays at the given net-local nodes."""
    mdl = model(parent, R, Chat)
    out = np.zeros(len(nodes))
    if mdl is None:
        return out
    a, tau = mdl
    for i, k in enumerate(nodes):
        if k > 0:
            out[i] = half_time(a[k - 1], tau)
    return out


def sink_delays(d, wire_cap=None):
    """Reduced-order delay of every sink of design ``d`` (caller sink order),
    with the receiving pin caps added at the sink nodes."""
    nsp = np.asarray(d.net_sink_ptr)
    ptr = np.asarray(d.net_node_ptr)
    caps = np.asarray(d.cap_ff if wire_cap is None else wire_cap, np.float64)
    kind = np.asarray(d.pin_kind)
    cell_of = np.full(d.n_pins, -1)
    cell_of[np.asarray(d.cell_in_pin)] = np.repeat(np.arange(d.n_cells), np.diff(d.cell_in_ptr))
    out = np.zeros(max(int(nsp[-1]), 1))
    for n in range(d.n_nets):
        a, b = ptr[n], ptr[n + 1]
        if nsp[n + 1] == nsp[n]:
            continue
        Chat = caps[a:b].copy()
        for s in range(nsp[n], nsp[n + 1]):
            pin = d.net_sink_pin[s]
            pc = d.po_cap_ff if kind[pin] == 3 else d.pin_cap_ff[d.cell_type[cell_of[pin]]]
            Chat[d.sink_node[s]] += pc
        out[nsp[n]:nsp[n + 1]] = net_delays(d.parent[a:b], d.res_kohm[a:b].astype(np.float64), Chat,
                                            d.sink_node[nsp[n]:nsp[n + 1]])
    return out[: int(nsp[-1])]
