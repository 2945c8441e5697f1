"""Pins of the oracle's double-and-restart branch (CPU only).

Sec. 3 doubles the number of training states when the generalisation test fails
(c_val / c_train - 1 > overtrain_ratio) and restarts the iteration from the gates
reached so far; App. A says the restart keeps the gates and that training states are
columns of a Haar unitary. The checks below take the oracle's record of each doubling
(every start's gates before and after it, the new training set and U psi, the plateau
reference on the new set) and test it against what those passages fix, through
independent routes: numpy's QR of the Ginibre draw, the dense brute-force circuit
matrices of ``tests/brute`` and the paper's overtraining rule applied to the recorded
costs.
"""
import numpy as np
import pytest

import oracle as O
from brute import dense as D
from paper_2405_12866_amd import inputs as I


def _haar_columns_by_numpy_qr(n, m, seed):
    """Mezzadri's construction with numpy's Householder QR (an independent route): the
    first m columns of the Q factor of the N x m Ginibre draw, phases fixed so that
    diag(R) is real and positive. Returned as [m][N] rows."""
    G = O.ginibre(1 << n, m, seed=seed, role=O.ROLE_TRAIN, stream=0).T  # N x m
    Q, R = np.linalg.qr(G)
    ph = np.diag(R) / np.abs(np.diag(R))
    return (Q * ph[None, :]).T


def _cost(U, C, psi):
    """Eq. 9 left side by dense matrices: (1/M) sum_j ||U psi_j - C psi_j||^2."""
    return float(np.mean([np.linalg.norm((U - C) @ s) ** 2 for s in psi]))


def _c1_run(**kw):
    """C1 (3 qubits, pairs (0,1),(1,2) x 3, Haar target from the template), doubling on."""
    w = I.workload_3q()
    p = O.default_params(**{**dict(dist_tol=1e-10, multistarts=4, seed=5, max_iter=400,
                                   m_init=2), **kw})
    gates, info = O.instantiate(3, w["pairs"], target_pairs=w["target_pairs"],
                                target_gates=w["target_gates"], params=p,
                                trace_capacity=20000, doubling_capacity=8)
    return w, p, gates, info


def test_doubling_record_exists_on_c1():
    """The 3-qubit workload overtrains at M = 2 and M = 4 (four states fix U only on a
    four-dimensional subspace) and doubles up to M = 8 = 2^n (Sec. 3: doubling stops
    at 2^n)."""
    _, _, _, info = _c1_run()
    dbl = info["trace"]["doublings"]
    assert info["restarts"] == len(dbl) >= 1
    assert [d["m_new"] for d in dbl] == [2 * d["m_old"] for d in dbl]
    assert dbl[-1]["m_new"] <= 8 and info["m_final"] == dbl[-1]["m_new"]


def test_extended_states_are_haar_columns_orthonormal_to_the_old_ones():
    """Sec. 3 / App. A: after a doubling the training set is still orthonormal and the
    old states are kept; the new ones are the next columns of the same Haar unitary.
    Checked against numpy's QR of the Ginibre draw (not the oracle's Gram-Schmidt), and
    U psi of the new set against the dense target matrix."""
    w, p, _, info = _c1_run()
    U = D.circuit_matrix(3, w["target_pairs"], w["target_gates"])
    prev = O.draw_states(3, p["m_init"], seed=p["seed"])
    for d in info["trace"]["doublings"]:
        psi, phi, m_old, m_new = d["psi"], d["phi"], d["m_old"], d["m_new"]
        assert psi.shape == (m_new, 8)
        # the old states are kept bit for bit
        assert np.array_equal(psi[:m_old], prev)
        # the whole set is orthonormal, in particular the new states against the old
        gram = psi.conj() @ psi.T
        assert np.max(np.abs(gram - np.eye(m_new))) < 1e-13
        assert np.max(np.abs(psi[m_old:].conj() @ psi[:m_old].T)) < 1e-13
        # and equals the Q factor of the Ginibre draw with m_new columns
        ref = _haar_columns_by_numpy_qr(3, m_new, p["seed"])
        assert np.max(np.abs(psi - ref)) < 1e-12
        # U psi formed for the new columns (Fig. pre-comp: A is recomputed)
        assert np.max(np.abs(phi - (U @ psi.T).T)) < 1e-13
        prev = psi


def test_gates_are_kept_across_each_doubling():
    """App. A: the restart continues from the gates reached so far. Every start's gates
    (running or stopped) are bit-identical just before and just after the doubling."""
    _, _, _, info = _c1_run(multistarts=6)
    for d in info["trace"]["doublings"]:
        assert np.array_equal(d["gates_before"], d["gates_after"])
        assert np.any(d["gates_before"] != 0)


def test_first_plateau_reference_is_the_cost_of_the_kept_gates_on_the_new_set():
    """Sec. 3 with App. A's Eq. 13: after a restart the improvement test compares the
    first sweep on the new set with the cost of the kept gates on that set. Checked by
    dense matrices: (1/M) sum ||U psi - C psi||^2 over the new training set."""
    w, _, _, info = _c1_run()
    U = D.circuit_matrix(3, w["target_pairs"], w["target_gates"])
    for d in info["trace"]["doublings"]:
        for s, g in enumerate(d["gates_after"]):
            if np.isnan(d["c_prev"][s]):
                continue  # a start that had stopped before the doubling
            C = D.circuit_matrix(3, w["pairs"], g.reshape(-1, 4, 4))
            assert abs(d["c_prev"][s] - _cost(U, C, d["psi"])) < 1e-12


def test_counters_restart_and_the_new_set_is_used():
    """After a doubling the sweep index since the restart starts again at 1, every row
    reports the new M, and the first sweep is not tested for overtraining before
    min_iter (the overtraining test needs i >= min_iter)."""
    _, p, _, info = _c1_run()
    tr = info["trace"]
    for d in info["trace"]["doublings"]:
        rows = np.nonzero(tr["m"] == d["m_new"])[0]
        first = rows[: np.unique(tr["start"][rows]).size]
        assert np.all(tr["iter"][first] == 1)
        over = rows[tr["event"][rows] == O.EV_OVERTRAINED]
        assert np.all(tr["iter"][over] >= p["min_iter"])


def _duplicate_validation_problem():
    """Fixed sample set whose validation rows are copies of the first two training
    rows: at M = 2 the validation cost equals the training cost up to rounding. The
    one-gate template cannot express the entangling target, so the cost stays well
    above dist_tol."""
    g = np.random.default_rng(44)
    psi = I.orthonormal_samples(3, 4, g)
    tg = I.haar_gates(1, g)
    phi = O.apply_circuit(3, psi, [(1, 2)], tg)
    return np.concatenate([psi, psi[:2]]), np.concatenate([phi, phi[:2]])


@pytest.mark.parametrize("otr", [1e-9, -1e-9])
def test_overtraining_fires_only_when_validation_cost_exceeds_the_ratio(otr):
    """Sec. 3: a start is overtrained when c_val / c_train - 1 > overtrain_ratio. With
    c_val = c_train (to rounding) a ratio of +1e-9 must never fire and -1e-9 must fire
    at the first sweep allowed to test (i = min_iter), which pins the direction of the
    comparison. On every recorded row with i >= min_iter and M below its cap the
    decision is then checked against the rule on the recorded costs."""
    psi, phi = _duplicate_validation_problem()
    p = O.default_params(multistarts=2, seed=9, m_init=2, max_iter=14, dist_tol=1e-30,
                         diff_tol_r=0.0, plateau_window=1000, overtrain_ratio=otr)
    _, info = O.instantiate(3, [(0, 1)], psi=psi, phi=phi, n_val=2, params=p,
                            trace_capacity=1000, doubling_capacity=4)
    tr = info["trace"]
    at_m2 = tr["m"] == 2
    assert np.all(np.abs(tr["c_val"][at_m2] - tr["c_train"][at_m2]) <= 1e-12 * tr["c_train"][at_m2])
    assert np.all(tr["c_train"] > 1e-3)
    if otr > 0:
        assert info["restarts"] == 0 and info["m_final"] == 2
        assert not np.any(tr["event"] == O.EV_OVERTRAINED)
    else:
        assert info["restarts"] >= 1
        over = np.nonzero(tr["event"] == O.EV_OVERTRAINED)[0]
        assert tr["iter"][over[0]] == p["min_iter"] and tr["m"][over[0]] == 2
        assert not np.any((tr["event"] == O.EV_OVERTRAINED) & (tr["iter"] < p["min_iter"]))
    m_cap = 4
    testable = (tr["iter"] >= p["min_iter"]) & (tr["m"] < m_cap)
    fired = tr["event"] == O.EV_OVERTRAINED
    rule = tr["c_val"] > (1.0 + otr) * tr["c_train"]
    assert np.array_equal(fired[testable], rule[testable])


def test_overtraining_at_the_cap_stops_without_doubling():
    """Sec. 3: M never grows past 2^n (here the 4 training rows of a sample set); a
    start that fails the generalisation test there is not doubled again."""
    psi, phi = _duplicate_validation_problem()
    p = O.default_params(multistarts=1, seed=9, m_init=4, max_iter=12, dist_tol=1e-30,
                         diff_tol_r=0.0, plateau_window=1000, overtrain_ratio=-0.5)
    _, info = O.instantiate(3, [(0, 1)], psi=psi, phi=phi, n_val=2, params=p,
                            trace_capacity=100, doubling_capacity=2)
    assert info["restarts"] == 0 and info["m_final"] == 4
    assert not np.any(info["trace"]["event"] == O.EV_OVERTRAINED)
