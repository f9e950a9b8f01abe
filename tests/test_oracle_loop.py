"""Pins of the oracle's main loop (Alg. 4: the check every tau iterations, the best labels
kept only on a strictly lower conductance, and the stops of Eqs. (tcond-1) and (tcond-2)).

The loop is driven by scripts: the orthogonal-iteration step returns blocks whose successive
differences have scripted Frobenius norms, Discretize returns labels that name the iteration
that produced them, and the conductance of those labels is a scripted value.  Each script has
one stopping iteration, stop reason and returned labels that the paper's loop admits; the
mutations a reader could make (a non-strict comparison, a history that misses phi_0 or starts
late, the convergence test at iterations that are not checks, a loop that never breaks) each
change one of them.
"""
import numpy as np
import pytest

import oracle
import oracle.ancka as oa

N, K = 12, 3


class _Op:
    n = N


def run_script(monkeypatch, phis, dqs=None, tau=5, T_a=1000, eps_q=0.005):
    """Run oracle.cluster with phi_t = phis[t] at every check t (phis[0] = phi of the initial
    labels) and ||Q(t) - Q(t-1)||_F = dqs.get(t, 1.0).  Every labels array handed to the loop
    is a fresh object whose iteration of origin is kept in a side table, so the returned labels
    name the check that produced them.  Returns (that iteration, report)."""
    dqs = dqs or {}
    marker = {}

    def labels_of(t):
        y = np.zeros(N, dtype=np.int64)
        y[1:] = np.arange(1, N) % K
        marker[id(y)] = t
        return y

    y0 = labels_of(0)

    def fake_init_bcm(op, k, alpha, T_i):
        return y0, None

    def fake_mhc(op, labels, k, alpha, gamma):
        return phis[marker[id(labels)]]

    state = {"t": 0, "c": 0.0}
    E = np.zeros((N, K + 1))
    E[0, 0] = 1.0                        # unit Frobenius norm direction

    def fake_initial_q(C):
        return np.zeros((N, K + 1))

    def fake_apply_P(op, Q):
        return Q

    def fake_qr_pos(Z):
        state["t"] += 1
        state["c"] += dqs.get(state["t"], 1.0)
        return state["c"] * E, None

    def fake_discretize(Qk, max_iter=30):
        return labels_of(state["t"]), None, None, None

    monkeypatch.setattr(oa, "init_bcm", fake_init_bcm)
    monkeypatch.setattr(oa, "mhc", fake_mhc)
    monkeypatch.setattr(oa, "initial_q", fake_initial_q)
    monkeypatch.setattr(oa, "apply_P", fake_apply_P)
    monkeypatch.setattr(oa, "qr_pos", fake_qr_pos)
    monkeypatch.setattr(oa, "discretize", fake_discretize)
    labels, rep = oracle.cluster(_Op(), K, tau=tau, T_a=T_a, eps_q=eps_q)
    return marker[id(labels)], rep


def test_rising_conductance_stops_at_third_value(monkeypatch):
    # phi_0 < phi_5 < phi_10: Eq. (tcond-2) holds on the history [phi_0, phi_5, phi_10]
    src, rep = run_script(monkeypatch, {0: 0.50, 5: 0.60, 10: 0.70, 15: 0.10})
    assert rep.iterations == 10 and rep.reason == "early_stop"
    assert src == 0 and rep.best_t == 0 and rep.best_phi == 0.50
    assert rep.phi_trace == [(0, 0.50), (5, 0.60), (10, 0.70)]


def test_dip_then_rise(monkeypatch):
    # the best labels are those of the dip; the stop comes once three values rise after it
    phis = {0: 0.50, 5: 0.60, 10: 0.40, 15: 0.45, 20: 0.47, 25: 0.01}
    src, rep = run_script(monkeypatch, phis)
    assert rep.iterations == 20 and rep.reason == "early_stop"
    assert src == 10 and rep.best_t == 10 and rep.best_phi == 0.40


def test_equal_conductance_keeps_earlier_labels_and_does_not_stop(monkeypatch):
    # phi_10 == phi_5: not strictly lower, so the labels of t = 5 stay; [phi_5, phi_10,
    # phi_15] is not strictly rising, so the first stop is at t = 20
    phis = {0: 0.50, 5: 0.40, 10: 0.40, 15: 0.45, 20: 0.50, 25: 0.01}
    src, rep = run_script(monkeypatch, phis)
    assert rep.iterations == 20 and rep.reason == "early_stop"
    assert src == 5 and rep.best_t == 5


def test_converged_at_first_check(monkeypatch):
    # ||Q(5) - Q(4)||_F < eps_Q at the first check: Eq. (tcond-1) stops the run there
    src, rep = run_script(monkeypatch, {0: 0.5, 5: 0.45, 10: 0.3}, dqs={5: 1e-3})
    assert rep.iterations == 5 and rep.reason == "converged"
    assert src == 5 and rep.best_phi == 0.45


def test_small_step_between_checks_does_not_stop(monkeypatch):
    # a small step at t = 3 or t = 4 is not looked at (the test runs only when t mod tau = 0)
    phis = {0: 0.5, 5: 0.45, 10: 0.44, 15: 0.43, 20: 0.42}
    src, rep = run_script(monkeypatch, phis, dqs={3: 1e-6, 4: 1e-6, 14: 1e-6, 15: 1e-3})
    assert rep.iterations == 15 and rep.reason == "converged"
    assert src == 15


def test_max_iterations(monkeypatch):
    # strictly falling conductance and large steps: T_a ends the run (T_a not a multiple of tau)
    phis = {t: 1.0 - 0.01 * t for t in range(0, 60, 5)}
    src, rep = run_script(monkeypatch, phis, T_a=23)
    assert rep.iterations == 23 and rep.reason == "max_iter"
    assert src == 20 and rep.best_t == 20
    assert [t for t, _ in rep.phi_trace] == [0, 5, 10, 15, 20]


def test_check_period(monkeypatch):
    # tau = 3: checks at 3, 6, 9; rising from phi_3 on stops at t = 9
    phis = {0: 0.9, 3: 0.2, 6: 0.3, 9: 0.4, 12: 0.0}
    src, rep = run_script(monkeypatch, phis, tau=3)
    assert rep.iterations == 9 and rep.reason == "early_stop"
    assert src == 3 and [t for t, _ in rep.phi_trace] == [0, 3, 6, 9]


@pytest.mark.parametrize("eps,stops", [(0.5, True), (0.25, False)])
def test_convergence_threshold_is_strict(monkeypatch, eps, stops):
    # ||Q(5) - Q(4)||_F = 0.25 (exact in binary): stops only when it is below eps_Q
    src, rep = run_script(monkeypatch, {0: 0.5, 5: 0.45, 10: 0.44, 15: 0.43}, dqs={5: 0.25}, eps_q=eps, T_a=12)
    assert (rep.reason == "converged") == stops
    assert rep.iterations == (5 if stops else 12)
