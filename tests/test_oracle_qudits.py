"""Pins of the oracle's qudit functions (Sec. 5: the method on d-level gates; CPU only).

With d = 2 the qudit functions must reproduce the pinned qubit oracle exactly; for d = 3
they are checked against tensor-reshape brute force, LAPACK's SVD, SciPy's polar
decomposition, the dense full-unitary QFactor sweep on base-3 axes, Haar moments and the
recovery of a reachable target.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle as O
from brute import dense as D
from paper_2405_12866_amd import inputs as I


def _rand_c(g, *shape):
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def _samples(d, n, M, g):
    N = d ** n
    z = _rand_c(g, N, M)
    q, _ = np.linalg.qr(z)
    return np.ascontiguousarray(q.T)


def test_d2_reduces_to_qubit_functions():
    n, M = 4, 3
    g = np.random.default_rng(1)
    a, b = _rand_c(g, M, 1 << n), _rand_c(g, M, 1 << n)
    for qa, qb in [(0, 1), (3, 1), (2, 0)]:
        u = I.haar_unitary(4, g)
        assert np.allclose(O.qd_apply_gate(2, n, a, qa, qb, u), O.apply_gate(n, a, qa, qb, u), atol=1e-14)
        assert np.allclose(O.qd_apply_gate(2, n, a, qa, qb, u, dagger=True),
                           O.apply_gate(n, a, qa, qb, u, dagger=True), atol=1e-14)
        assert np.allclose(O.qd_environment(2, n, a, b, qa, qb), O.environment(n, a, b, qa, qb), atol=1e-13)
    pairs = I.random_pair_template(n, 6, g)
    tg, g0 = I.haar_gates(6, g), I.haar_gates(6, g)
    psi = I.orthonormal_samples(n, 5, g)
    phi = O.apply_circuit(n, psi, pairs, tg)
    x, cx = O.qd_sweep(2, n, pairs, psi, phi, g0)
    y, cy = O.sweep(n, pairs, psi, phi, g0)
    assert np.allclose(x, y, atol=1e-12) and abs(cx - cy) < 1e-13


def test_d2_instantiate_follows_qubit_instantiate():
    n = 3
    g = np.random.default_rng(2)
    pairs = [(0, 1), (1, 2), (0, 2)]
    tg = I.haar_gates(3, g)
    psi = I.orthonormal_samples(n, 8, g)
    phi = O.apply_circuit(n, psi, pairs, tg)
    gi = np.stack([I.haar_gates(3, g) for _ in range(3)])
    p = O.default_params(multistarts=3, m_init=2, dist_tol=1e-11, max_iter=500, diff_tol_r=1e-7)
    ga, ia = O.qd_instantiate(2, n, pairs, psi, phi, n_val=2, params=p, gates_in=gi)
    gb, ib = O.instantiate(n, pairs, psi=psi, phi=phi, n_val=2, params=p, gates_in=gi)
    for k in ("reason_name", "best_start", "sweeps", "restarts", "m_final"):
        assert ia[k] == ib[k], k
    assert abs(ia["c_train"] - ib["c_train"]) <= 1e-10 * max(ib["c_train"], 1e-12)
    assert np.allclose(ga, gb, atol=1e-10)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_qutrit_apply_matches_tensor_brute_force(n):
    g = np.random.default_rng(n)
    st = _rand_c(g, 2, 3 ** n)
    for a in range(n):
        for b in range(n):
            if a == b:
                continue
            u = I.haar_unitary(9, g)
            assert np.allclose(O.qd_apply_gate(3, n, st, a, b, u), D.apply_gate_tensor_d(3, n, st, a, b, u),
                               atol=1e-13)
            assert np.allclose(O.qd_apply_gate(3, n, st, a, b, u, dagger=True),
                               D.apply_gate_tensor_d(3, n, st, a, b, u.conj().T), atol=1e-13)


def test_qutrit_environment_linear_functional():
    """Tr(G^dag X) = sum_j <a_j| X_ab |b_j> for arbitrary complex 9 x 9 X on (qa, qb)."""
    n, M = 3, 2
    g = np.random.default_rng(4)
    a, b = _rand_c(g, M, 27), _rand_c(g, M, 27)
    for qa, qb in [(0, 1), (2, 0), (1, 2)]:
        G = O.qd_environment(3, n, a, b, qa, qb)
        for _ in range(3):
            X = _rand_c(g, 9, 9)
            rhs = np.sum(a.conj() * (b @ D.gate_matrix_d(3, n, qa, qb, X).T))
            assert abs(np.sum(G.conj() * X) - rhs) < 1e-12 * (1 + abs(rhs))


@pytest.mark.parametrize("Dm", [4, 9, 16])
def test_qd_svd_against_lapack(Dm):
    g = np.random.default_rng(Dm)
    for rank in (Dm, Dm - 2, 1):
        A = _rand_c(g, Dm, rank) @ _rand_c(g, rank, Dm)
        W, s, V = O.qd_svd(A)
        assert np.allclose(s, np.linalg.svd(A, compute_uv=False), atol=1e-12 * s[0])
        assert np.allclose(W @ np.diag(s) @ V.conj().T, A, atol=1e-11 * s[0])
        assert np.allclose(W.conj().T @ W, np.eye(Dm), atol=1e-12)
        assert np.allclose(V.conj().T @ V, np.eye(Dm), atol=1e-12)


def test_qd_update_is_scipy_polar_and_beta_one_keeps():
    g = np.random.default_rng(5)
    for _ in range(10):
        G = _rand_c(g, 9, 9)
        u = O.qd_update_gate(G)
        assert np.allclose(u, scipy.linalg.polar(G, side="right")[0], atol=1e-12)
        w = I.haar_unitary(9, g)
        assert np.real(np.sum(G.conj() * w)) <= np.real(np.sum(G.conj() * u)) + 1e-12
    u0 = I.haar_unitary(9, g)
    assert np.allclose(O.qd_update_gate(_rand_c(g, 9, 9), 1.0, u0), u0, atol=1e-13)


def test_qd_haar_gate_moments():
    """Haar on U(9): unitary, E |Tr U|^2 = 1 (within 5 standard errors)."""
    tr2 = []
    for s in range(4):
        for k in range(250):
            u = O.qd_haar_gate(3, 7, s, k)
            assert np.max(np.abs(u.conj().T @ u - np.eye(9))) < 1e-13
            tr2.append(abs(np.trace(u)) ** 2)
    tr2 = np.array(tr2)
    assert abs(tr2.mean() - 1.0) < 5 * tr2.std() / np.sqrt(len(tr2))


def test_full_basis_qutrit_sweep_is_dense_qfactor():
    n = 3
    g = np.random.default_rng(6)
    pairs = [(0, 1), (1, 2), (0, 2), (2, 1)]
    tg = np.stack([I.haar_unitary(9, g) for _ in pairs])
    U = D.circuit_matrix_d(3, n, pairs, tg)
    psi = _samples(3, n, 27, g)
    phi = psi @ U.T
    gs = np.stack([I.haar_unitary(9, g) for _ in pairs])
    gd = gs.copy()
    for _ in range(3):
        gs, _ = O.qd_sweep(3, n, pairs, psi, phi, gs)
        gd = D.dense_qfactor_sweep_d(3, n, pairs, gd, U)
        assert np.allclose(gs, gd, atol=1e-11)


def test_qutrit_sweep_monotone_and_cost():
    n, M = 4, 5
    g = np.random.default_rng(7)
    pairs = I.random_pair_template(n, 5, g)
    tg = np.stack([I.haar_unitary(9, g) for _ in range(5)])
    psi = _samples(3, n, M, g)
    phi = O.qd_apply_circuit(3, n, psi, pairs, tg)
    gates = np.stack([I.haar_unitary(9, g) for _ in range(5)])
    for _ in range(4):
        new, c, fb, fa = O.qd_sweep(3, n, pairs, psi, phi, gates, record=True)
        assert np.all(fa >= fb - 1e-12 * M)
        assert np.allclose(fb[:-1], fa[1:], atol=1e-12 * M)
        Cpsi = O.qd_apply_circuit(3, n, psi, pairs, new)
        assert abs(c - np.sum(np.abs(Cpsi - phi) ** 2) / M) < 1e-12
        gates = new


def test_qutrit_target_recovered():
    """3 qutrits, 3 gates, target from the same template. With the full basis as training
    set (M = 27, no validation set) c_train is the full distance, and the run succeeds.
    With 9 .. 18 training and 9 validation samples the residual concentrates in the
    untrained directions (c_val stays about 3 c_train), so at the M cap the run ends
    NOT_GENERALIZED with c_train < dist_tol; the full distance is still small."""
    n = 3
    g = np.random.default_rng(8)
    pairs = [(0, 1), (1, 2), (0, 1)]
    tg = np.stack([I.haar_unitary(9, g) for _ in pairs])
    U = D.circuit_matrix_d(3, n, pairs, tg)
    psi = _samples(3, n, 27, g)
    phi = psi @ U.T
    p = O.default_params(multistarts=4, m_init=27, seed=3, dist_tol=1e-11, max_iter=3000)
    gates, info = O.qd_instantiate(3, n, pairs, psi, phi, n_val=0, params=p)
    assert info["reason_name"] == "SUCCESS", info
    C = D.circuit_matrix_d(3, n, pairs, gates)
    d_full = np.linalg.norm(U - C) ** 2 / 27
    assert d_full < 1e-11 and abs(d_full - info["c_train"]) < 1e-13
    p = O.default_params(multistarts=4, m_init=9, seed=3, dist_tol=1e-11, max_iter=3000)
    gates, info = O.qd_instantiate(3, n, pairs, psi, phi, n_val=9, params=p)
    assert info["reason_name"] in ("SUCCESS", "NOT_GENERALIZED") and info["c_train"] < 1e-11
    assert info["m_final"] == 18
    C = D.circuit_matrix_d(3, n, pairs, gates)
    assert np.linalg.norm(U - C) ** 2 / 27 < 1e-9


# ------------------------------------------------------------- drawn states and targets
def _lapack_q(A_cols):
    """Q of the QR factorisation of the N x M matrix whose columns are the rows of A_cols,
    with diag(R) made real positive (LAPACK Householder, phases fixed after)."""
    q, r = np.linalg.qr(A_cols.T)
    ph = np.diag(r) / np.abs(np.diag(r))
    return (q * ph).T


@pytest.mark.parametrize("d,n,M", [(3, 3, 5), (4, 2, 7), (3, 4, 12), (2, 5, 6)])
def test_qudit_draw_is_qr_of_the_ginibre_stream(d, n, M):
    """Sec. 3 / App. A: the states are the columns of a Haar unitary, here the Q of the
    N x M Ginibre matrix (Philox index j N + i) with positive diag(R): equal to LAPACK's
    QR with its phases fixed; the first rows of a larger draw are the smaller draw (what
    the extension on doubling relies on); d = 2 is the qubit draw."""
    N = d ** n
    A = O.ginibre(N, M, 11, O.ROLE_TRAIN, 0)
    st = O.qd_draw_states(d, n, M, 11, O.ROLE_TRAIN, 0)
    assert np.allclose(st, _lapack_q(A), atol=1e-12)
    assert np.allclose(st.conj() @ st.T, np.eye(M), atol=1e-13)
    big = O.qd_draw_states(d, n, M + 3, 11, O.ROLE_TRAIN, 0)
    assert np.array_equal(big[:M], st)
    other = O.qd_draw_states(d, n, M, 11, O.ROLE_VAL, 1)
    assert np.max(np.abs(other - st)) > 0.1
    if d == 2:
        assert np.array_equal(st, O.draw_states(n, M, 11, O.ROLE_TRAIN, 0))


def _qudit_problem(d, n, pairs, seed):
    g = np.random.default_rng(seed)
    tg = np.stack([I.haar_unitary(d * d, g) for _ in pairs])
    return tg, D.circuit_matrix_d(d, n, pairs, tg)


def test_qudit_dense_and_circuit_targets_agree_and_double():
    """A target circuit and its dense unitary (built independently by Kronecker
    products) give the same training pairs, hence the same run: same reason, start,
    sweeps and doublings, costs to rounding. (M d^(n-2) >= d^2 from the first sweep, so
    every environment has full rank and each update is unique: with fewer samples the
    polar factor's completion follows rounding.) The doubling record shows the Sec. 3
    double-and-restart on drawn states: the new training set is the larger draw (old
    states kept, new ones orthonormal to them), phi = U psi on it, every gate kept."""
    d, n = 3, 3
    pairs = [(0, 1), (1, 2), (0, 1), (1, 2)]
    tg, U = _qudit_problem(d, n, pairs, 30)
    p = O.default_params(multistarts=2, m_init=3, seed=9, dist_tol=1e-10, max_iter=300, min_iter=3)
    ga, ia = O.qd_instantiate_target(d, n, pairs, U=U, params=p, doubling_capacity=4)
    gb, ib = O.qd_instantiate_target(d, n, pairs, target_pairs=pairs, target_gates=tg, params=p)
    for k in ("reason_name", "best_start", "sweeps", "restarts", "m_final"):
        assert ia[k] == ib[k], (k, ia[k], ib[k])
    assert ia["reason_name"] == "SUCCESS"
    assert abs(ia["c_train"] - ib["c_train"]) <= 1e-8 * ib["c_train"] + 1e-18
    assert ia["restarts"] >= 1, ia
    rec = ia["trace"]["doublings"][0]
    m_old, m_new = rec["m_old"], rec["m_new"]
    assert m_new == 2 * m_old
    draw = O.qd_draw_states(d, n, m_new, 9, O.ROLE_TRAIN, 0)
    assert np.allclose(rec["psi"], draw, atol=1e-14)
    assert np.allclose(rec["phi"], rec["psi"] @ U.T, atol=1e-12)
    assert np.array_equal(rec["gates_before"], rec["gates_after"])


@pytest.mark.parametrize("d,n,pairs", [(3, 3, [(0, 1), (1, 2), (0, 1)]), (4, 2, [(0, 1)]),
                                       (4, 3, [(0, 1), (1, 2)])])
def test_qudit_reachable_target_recovered_from_drawn_states(d, n, pairs):
    """A target built from the template is recovered: SUCCESS, and the returned gates
    reproduce the target unitary (full distance, Eq. 1, from Kronecker products)."""
    tg, U = _qudit_problem(d, n, pairs, 40 + d + n)
    p = O.default_params(multistarts=4, m_init=d * d, seed=4, dist_tol=1e-11, max_iter=3000)
    gates, info = O.qd_instantiate_target(d, n, pairs, target_pairs=pairs, target_gates=tg, params=p)
    assert info["reason_name"] == "SUCCESS", info
    C = D.circuit_matrix_d(d, n, pairs, gates)
    assert np.linalg.norm(U - C) ** 2 / d ** n < 1e-8


# ------------------------------------------------------------------ qudit gate kinds
def _csum(d):
    """Constant two-qudit gate |x, y> -> |x, y + x mod d> (local index d x + y)."""
    D = d * d
    U = np.zeros((D, D), dtype=np.complex128)
    for x in range(d):
        for y in range(d):
            U[d * x + (y + x) % d, d * x + y] = 1.0
    return U


def _kind_slots(d, kinds, g):
    D = d * d
    out = []
    for k in kinds:
        if k == O.GATE_1Q:
            out.append(np.kron(I.haar_unitary(d, g), np.eye(d)))
        elif k == O.GATE_FIXED:
            out.append(_csum(d))
        else:
            out.append(I.haar_unitary(D, g))
    return np.stack(out)


def test_d2_kinds_sweep_is_the_qubit_kinds_sweep():
    n = 4
    g = np.random.default_rng(31)
    pairs = [(0, 1), (1, 2), (2, 3), (3, 0), (1, 3), (2, 0)]
    kinds = [O.GATE_1Q, O.GATE_FIXED, O.GATE_2Q, O.GATE_1Q, O.GATE_2Q, O.GATE_FIXED]
    gates = _kind_slots(2, kinds, g)
    psi = I.orthonormal_samples(n, 5, g)
    phi = O.apply_circuit(n, psi, pairs, I.haar_gates(6, g))
    x, cx = O.qd_sweep(2, n, pairs, psi, phi, gates, kinds=kinds)
    y, cy = O.sweep(n, pairs, psi, phi, gates, kinds=kinds)
    assert np.allclose(x, y, atol=1e-12) and abs(cx - cy) < 1e-13


@pytest.mark.parametrize("qa,qb", [(0, 1), (1, 2), (2, 0)])
def test_qutrit_one_qudit_update_is_polar_of_its_contraction(qa, qb):
    """L = 1, one one-qutrit gate on qa (spectator qb): its environment is the contraction
    of phi against psi over every digit but qa (numpy), and the sweep sets the slot to
    polar(G1) (x) I_3 (SciPy), whatever the spectator."""
    n, M = 3, 4
    g = np.random.default_rng(40 + qa)
    psi, phi = _samples(3, n, M, g), _rand_c(g, M, 27)
    a = phi.reshape((M,) + (3,) * n)
    b = psi.reshape((M,) + (3,) * n)
    G1 = np.tensordot(np.moveaxis(a, 1 + qa, 1), np.moveaxis(b, 1 + qa, 1).conj(),
                      axes=([0] + list(range(2, n + 1)), [0] + list(range(2, n + 1))))
    assert np.allclose(O.qd_environment1(3, n, phi, psi, qa), G1, atol=1e-12)
    slot = np.kron(I.haar_unitary(3, g), np.eye(3))
    new, _ = O.qd_sweep(3, n, [(qa, qb)], psi, phi, slot[None], kinds=[O.GATE_1Q])
    v = scipy.linalg.polar(G1, side="right")[0]
    assert np.allclose(new[0], np.kron(v, np.eye(3)), atol=1e-12)


def test_qutrit_kinds_sweep_keeps_forms_and_descends():
    """Constant gates stay as given, one-qudit slots keep the form v (x) I_3 with v unitary,
    and the Eq. 9 cost never rises over the sweeps."""
    n, M = 4, 6
    g = np.random.default_rng(32)
    pairs = [(0, 1), (1, 2), (2, 3), (3, 1), (0, 2), (2, 1), (1, 0)]
    kinds = [O.GATE_1Q, O.GATE_FIXED, O.GATE_2Q, O.GATE_1Q, O.GATE_FIXED, O.GATE_1Q, O.GATE_2Q]
    gates = _kind_slots(3, kinds, g)
    psi = _samples(3, n, M, g)
    phi = O.qd_apply_circuit(3, n, psi, pairs, _kind_slots(3, kinds, g))
    c_prev = np.inf
    for _ in range(6):
        gates, c = O.qd_sweep(3, n, pairs, psi, phi, gates, kinds=kinds)
        assert c <= c_prev + 1e-12
        c_prev = c
        for k, kind in enumerate(kinds):
            if kind == O.GATE_FIXED:
                assert np.array_equal(gates[k], _csum(3))
            elif kind == O.GATE_1Q:
                v = gates[k][::3, ::3]
                assert np.allclose(gates[k], np.kron(v, np.eye(3)), atol=1e-14)
                assert np.allclose(v.conj().T @ v, np.eye(3), atol=1e-12)


def test_qd_haar_gate1_is_a_unitary_slot():
    for s in range(3):
        for k in range(5):
            u = O.qd_haar_gate1(3, 9, s, k)
            v = u[::3, ::3]
            assert np.allclose(u, np.kron(v, np.eye(3)), atol=0)
            assert np.allclose(v.conj().T @ v, np.eye(3), atol=1e-13)


def test_qutrit_kinds_target_recovered():
    """3 qutrits: one-qutrit gates around constant CSUM gates; a target from the same
    template with other one-qutrit gates is recovered from drawn states (SUCCESS, full
    distance from Kronecker products)."""
    n = 3
    pairs = [(0, 1), (1, 2), (0, 1), (1, 0), (2, 1), (0, 1), (1, 2)]
    kinds = [O.GATE_1Q, O.GATE_1Q, O.GATE_FIXED, O.GATE_1Q, O.GATE_1Q, O.GATE_FIXED, O.GATE_1Q]
    g = np.random.default_rng(33)
    tg = _kind_slots(3, kinds, g)
    fixed = np.stack([_csum(3)] * len(pairs))
    U = D.circuit_matrix_d(3, n, pairs, tg)
    p = O.default_params(multistarts=8, m_init=3, seed=5, dist_tol=1e-11, max_iter=2000)
    gates, info = O.qd_instantiate_target(3, n, pairs, target_pairs=pairs, target_gates=tg, params=p,
                                          kinds=kinds, fixed=fixed)
    assert info["reason_name"] == "SUCCESS", info
    for k, kind in enumerate(kinds):
        if kind == O.GATE_FIXED:
            assert np.array_equal(gates[k], _csum(3))
    C = D.circuit_matrix_d(3, n, pairs, gates)
    assert np.linalg.norm(U - C) ** 2 / 27 < 1e-8
