"""Pins of the reduced-order (Arnoldi) net delay oracle (oracle/arnoldi.py):
the single-RC closed form, exactness when the Krylov space is the whole
state space (two unknown nodes, against the exact step response by the
matrix exponential), the first two time moments at every node (Elmore d and
m2), zero-resistance segments behaving as merged nodes, and the Elmore upper
bound of the exact 50% delay that the model approaches."""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import arnoldi as AR


def _exact_half(parent, R, Chat, node):
    """50% time of the exact step response at a node (bisection on expm)."""
    Rs = AR.shared_resistance(parent, np.asarray(R, np.float64))
    A = Rs @ np.diag(np.asarray(Chat, np.float64)[1:])
    Ainv = np.linalg.inv(A)
    one = np.ones(A.shape[0])
    y = lambda t: 1.0 - (expm(-Ainv * t) @ one)[node - 1]  # noqa: E731
    hi = float(np.max(np.abs(np.linalg.eigvals(A))))
    while y(hi) < 0.5:
        hi *= 2
    lo = 0.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if y(mid) < 0.5 else (lo, mid)
    return 0.5 * (lo + hi)


def _random_tree(rng, m):
    parent = np.array([-1] + [int(rng.integers(0, k)) for k in range(1, m)], np.int32)
    R = np.concatenate([[0.0], rng.uniform(0.01, 0.05, m - 1)])
    C = np.concatenate([[0.0], rng.uniform(0.1, 2.0, m - 1)])
    return parent, R, C


def test_single_rc_is_exact():
    for Rv, Cv in ((0.02, 3.0), (1.5, 0.01), (0.3, 7.5)):
        t = AR.net_delays([-1, 0], [0.0, Rv], [0.0, Cv], [1])[0]
        assert t == pytest.approx(Rv * Cv * np.log(2.0), rel=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_two_unknown_nodes_are_exact(seed):
    """A chain or a star of two nodes: the Krylov space {d, A d} is all of
    the state space, so the model is the exact response."""
    rng = np.random.default_rng(seed)
    for parent in ([-1, 0, 1], [-1, 0, 0]):
        R = [0.0, *rng.uniform(0.01, 0.1, 2)]
        C = [0.0, *rng.uniform(0.2, 3.0, 2)]
        for node in (1, 2):
            got = AR.net_delays(parent, R, C, [node])[0]
            assert got == pytest.approx(_exact_half(parent, R, C, node), rel=1e-9)


@pytest.mark.parametrize("seed", range(5))
def test_model_keeps_the_first_two_moments(seed):
    """1 - Y_i(t) = sum_j a_ij exp(-t/tau_j) integrates to the Elmore delay
    d_i and its first moment to m2_i = (A d)_i, at every node."""
    rng = np.random.default_rng(seed)
    parent, R, C = _random_tree(rng, int(rng.integers(4, 30)))
    a, tau = AR.model(parent, R, C)
    A = AR.shared_resistance(parent, R) @ np.diag(C[1:])
    d = A @ np.ones(A.shape[0])
    m2 = A @ d
    np.testing.assert_allclose(a @ tau, d, rtol=1e-9)
    np.testing.assert_allclose(a @ tau ** 2, m2, rtol=1e-9)


def test_zero_resistance_segments_merge_nodes():
    """A zero-resistance segment joins two nodes into one: the same delays as
    the tree with the pair merged (caps added)."""
    R = [0.0, 0.04, 0.0, 0.03, 0.05]
    C = [0.0, 1.0, 0.7, 0.4, 1.3]
    parent = [-1, 0, 1, 2, 2]  # node 2 hangs on node 1 through R = 0
    merged_parent = [-1, 0, 1, 1]
    merged_R = [0.0, 0.04, 0.03, 0.05]
    merged_C = [0.0, 1.7, 0.4, 1.3]
    got = AR.net_delays(parent, R, C, [1, 2, 3, 4])
    ref = AR.net_delays(merged_parent, merged_R, merged_C, [1, 1, 2, 3])
    np.testing.assert_allclose(got, ref, rtol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_delays_are_positive_and_below_elmore_for_far_sinks(seed):
    """For the node farthest from the driver the exact 50% delay lies below
    the Elmore delay (an upper bound on RC trees); the order-2 model stays
    within 10% of the exact value there."""
    rng = np.random.default_rng(10 + seed)
    parent, R, C = _random_tree(rng, 12)
    A = AR.shared_resistance(parent, R) @ np.diag(C[1:])
    d = A @ np.ones(A.shape[0])
    far = int(np.argmax(d)) + 1
    exact = _exact_half(parent, R, C, far)
    got = AR.net_delays(parent, R, C, [far])[0]
    assert 0.0 < exact <= d[far - 1]
    assert got == pytest.approx(exact, rel=0.1)


@pytest.mark.parametrize("seed", range(4))
def test_half_level_is_crossed_once(seed):
    """At every node the two-pole response crosses one half exactly once on
    t > 0 (the impulse response, a sum of two exponentials, changes sign at
    most once), so any bracketing root finder of the half-time equation
    lands on the root the bisection finds."""
    rng = np.random.default_rng(40 + seed)
    parent, R, C = _random_tree(rng, int(rng.integers(5, 40)))
    a, tau = AR.model(parent, R, C)
    t = np.linspace(0.0, 40.0 * float(tau.max()), 40001)
    for i in range(a.shape[0]):
        f = (a[i][None, :] * np.exp(-t[:, None] / tau[None, :])).sum(axis=1) - 0.5
        s = np.sign(f)
        s = s[s != 0]
        assert np.count_nonzero(np.diff(s)) <= 1
        th = AR.half_time(a[i], tau)
        if f[0] > 0.0:
            assert abs(float(np.sum(a[i] * np.exp(-th / tau))) - 0.5) < 1e-12
        else:
            assert th == 0.0
