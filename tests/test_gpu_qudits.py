"""GPU parity of the qudit path (Sec. 5: the method on d-level gates) against the FP64
oracle's qudit functions, through the C ABI.

d = 2 must reproduce the qubit path; d = 3 (qutrits) and d = 4 run in lock step with the
oracle (FP64: cost and gates 1e-10 over 10 sweeps; complex64 states teacher-forced,
|dc| <= 1e-6 max(c, c_initial)), follow its control flow on fixed sample sets and on
dense and circuit targets with states drawn on each side, and handle a rank-deficient
environment (several optimal gates: the cost, which depends only on the sum of singular
values, is compared).
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2405_12866_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_12866_amd import qfs as Q  # noqa: E402

DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.complex128)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _samples(d, n, M, g):
    z = g.standard_normal((d ** n, M)) + 1j * g.standard_normal((d ** n, M))
    q, _ = np.linalg.qr(z)
    return np.ascontiguousarray(q.T)


def _problem(d, n, L, M, starts, seed):
    g = np.random.default_rng(seed)
    pairs = I.random_pair_template(n, L, g)
    D = d * d
    tg = np.stack([I.haar_unitary(D, g) for _ in range(L)])
    psi = _samples(d, n, M, g)
    phi = O.qd_apply_circuit(d, n, psi, pairs, tg)
    gates = np.stack([np.stack([I.haar_unitary(D, g) for _ in range(L)]) for _ in range(starts)])
    return pairs, psi, phi, gates, tg


def test_d2_qudit_sweep_equals_qubit_sweep():
    say("qudit d=2 vs qubit sweep")
    pairs, psi, phi, gates, _ = _problem(2, 6, 9, 5, 2, seed=1)
    a, b = dev(gates), dev(gates)
    for _ in range(5):
        ca = Q.qfs_qudit_sweep(2, 6, pairs, dev(psi), dev(phi), a, precision=Q.QFS_PREC_FP64)
        cb = Q.qfs_sweep(6, pairs, dev(psi), dev(phi), b, precision=Q.QFS_PREC_FP64)
        assert np.max(np.abs(ca - cb)) <= 1e-12 * max(np.max(cb), 1e-3)
    assert np.max(np.abs(host(a) - host(b))) < 1e-11


@pytest.mark.parametrize("n,L,M,starts", [(2, 1, 9, 1), (3, 4, 5, 2), (5, 7, 6, 2), (6, 6, 3, 3)])
def test_qutrit_fp64_lock_step(n, L, M, starts):
    say(f"qutrit fp64 lock-step n={n} L={L} M={M} starts={starts}")
    pairs, psi, phi, gates, _ = _problem(3, n, L, M, starts, seed=10 * n + L)
    dg, dpsi, dphi = dev(gates), dev(psi), dev(phi)
    ref = gates.copy()
    for sweep in range(10):
        c = Q.qfs_qudit_sweep(3, n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_FP64)
        for s in range(starts):
            ref[s], cr = O.qd_sweep(3, n, pairs, psi, phi, ref[s])
            assert abs(c[s] - cr) <= 1e-10 * max(cr, 1e-3), (sweep, s, c[s], cr)
        assert np.max(np.abs(host(dg) - ref)) < 1e-10


def test_qutrit_mixed_teacher_forced():
    say("qutrit mixed teacher-forced n=6")
    n, L, M = 6, 8, 16
    pairs, psi, phi, gates, _ = _problem(3, n, L, M, 2, seed=7)
    dpsi, dphi, dg = dev(psi), dev(phi), dev(gates)
    c_init = max(O.qd_sweep(3, n, pairs, psi, phi, gates[0])[1], 1e-3)
    for sweep in range(5):
        start = host(dg).copy()
        c = Q.qfs_qudit_sweep(3, n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_MIXED)
        new = host(dg)
        for s in range(2):
            _, cr = O.qd_sweep(3, n, pairs, psi, phi, start[s])
            assert abs(c[s] - cr) <= 1e-6 * max(cr, c_init), (sweep, s, c[s], cr)
            for u in new[s]:
                assert np.max(np.abs(u.conj().T @ u - np.eye(9))) < 1e-12


def test_qutrit_rank_deficient_environment():
    """n = 2 qutrits, one gate, M = 2: the 9 x 9 environment has rank 2, so the update is
    not unique; the device's gate must be unitary and reach the oracle's cost (set by the
    sum of the singular values alone)."""
    say("qutrit rank-deficient environment")
    pairs, psi, phi, gates, _ = _problem(3, 2, 1, 2, 1, seed=3)
    dg = dev(gates)
    c = Q.qfs_qudit_sweep(3, 2, pairs, dev(psi), dev(phi), dg, precision=Q.QFS_PREC_FP64)
    _, cr = O.qd_sweep(3, 2, pairs, psi, phi, gates[0])
    u = host(dg)[0, 0]
    assert np.max(np.abs(u.conj().T @ u - np.eye(9))) < 1e-12
    assert abs(c[0] - cr) < 1e-12


@pytest.mark.parametrize("m_init,n_val", [(3, 9), (27, 0)])
def test_qutrit_instantiate_follows_oracle(m_init, n_val):
    """FP64, initial gates drawn on each side from the seed: same reason, start, sweeps,
    doublings and final M as the oracle, cost to 1e-9 relative."""
    say(f"qutrit instantiate vs oracle m_init={m_init} n_val={n_val}")
    n = 3
    g = np.random.default_rng(20)
    pairs = [(0, 1), (1, 2), (0, 1)]
    tg = np.stack([I.haar_unitary(9, g) for _ in pairs])
    psi = _samples(3, n, 27, g)
    phi = O.qd_apply_circuit(3, n, psi, pairs, tg)
    p = O.default_params(multistarts=3, m_init=m_init, seed=5, dist_tol=1e-11, max_iter=400)
    g_ref, ref = O.qd_instantiate(3, n, pairs, psi, phi, n_val=n_val, params=p)
    g_gpu, got = Q.qfs_qudit_instantiate(3, n, pairs, dev(psi), dev(phi), n_val=n_val,
                                         params=dict(p, precision=Q.QFS_PREC_FP64))
    for k in ("reason_name", "best_start", "sweeps", "restarts", "m_final"):
        assert got[k] == ref[k], (k, got, ref)
    assert abs(got["c_train"] - ref["c_train"]) <= 1e-9 * max(ref["c_train"], 1e-12) + 1e-20
    assert np.max(np.abs(host(g_gpu) - g_ref)) < 1e-8


def test_qutrit_instantiate_mixed_reaches_target():
    """complex64 states with complex128 refinement, 5 qutrits, 4 gates, training from 9
    samples with doubling against 9 validation samples: success, and the returned gates
    reproduce the target on fresh states (oracle simulation)."""
    say("qutrit instantiate mixed n=5")
    n = 5
    g = np.random.default_rng(21)
    pairs = [(0, 1), (2, 3), (1, 2), (3, 4)]
    tg = np.stack([I.haar_unitary(9, g) for _ in pairs])
    psi = _samples(3, n, 137, g)
    phi = O.qd_apply_circuit(3, n, psi, pairs, tg)
    p = Q.qfs_default_params(multistarts=8, m_init=9, seed=6, dist_tol=1e-9, max_iter=3000)
    gates, info = Q.qfs_qudit_instantiate(3, n, pairs, dev(psi), dev(phi), n_val=9, params=p)
    assert info["reason_name"] == "SUCCESS", info
    fresh = _samples(3, n, 12, np.random.default_rng(22))
    a = O.qd_apply_circuit(3, n, fresh, pairs, host(gates))
    b = O.qd_apply_circuit(3, n, fresh, pairs, tg)
    assert np.sum(np.abs(a - b) ** 2) / 12 < 1e-7


def test_qudit_entries_reject_bad_arguments():
    say("qudit argument checks")
    psi = dev(np.eye(25)[:2])
    with pytest.raises(Q.QfsError) as e:
        Q.qfs_qudit_instantiate(5, 2, [(0, 1)], psi, psi, params=Q.qfs_default_params())
    assert e.value.code == Q.QFS_EUNSUPPORTED
    psi = dev(np.eye(9)[:2])
    with pytest.raises(Q.QfsError) as e:
        Q.qfs_qudit_instantiate(3, 2, [(0, 0)], psi, psi, params=Q.qfs_default_params())
    assert e.value.code == Q.QFS_EINVAL


@pytest.mark.parametrize("n,L,M,starts", [(2, 1, 17, 1), (2, 3, 16, 2), (3, 4, 7, 2), (4, 5, 3, 3)])
def test_d4_fp64_lock_step(n, L, M, starts):
    """d = 4: 16 x 16 gates (environment rows two per block, the 16 x 16 Jacobi polar).
    M 4^(n-2) >= 16, so every environment has full rank and the updated gates are unique."""
    say(f"d=4 fp64 lock-step n={n} L={L} M={M} starts={starts}")
    pairs, psi, phi, gates, _ = _problem(4, n, L, M, starts, seed=100 + 10 * n + L)
    dg, dpsi, dphi = dev(gates), dev(psi), dev(phi)
    ref = gates.copy()
    for sweep in range(10):
        c = Q.qfs_qudit_sweep(4, n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_FP64)
        for s in range(starts):
            ref[s], cr = O.qd_sweep(4, n, pairs, psi, phi, ref[s])
            assert abs(c[s] - cr) <= 1e-10 * max(cr, 1e-3), (sweep, s, c[s], cr)
        assert np.max(np.abs(host(dg) - ref)) < 1e-10


def test_d4_rank_deficient_environment():
    """n = 2 ququarts, M = 5: each 16 x 16 environment has rank 5, so the polar factor is
    not unique; the gates must stay unitary and each sweep's cost must match the oracle's
    from the same gates (it depends only on the singular values)."""
    say("d=4 rank-deficient environment")
    pairs, psi, phi, gates, _ = _problem(4, 2, 3, 5, 2, seed=130)
    dg, dpsi, dphi = dev(gates), dev(psi), dev(phi)
    for sweep in range(4):
        start = host(dg).copy()
        c = Q.qfs_qudit_sweep(4, 2, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_FP64)
        for s in range(2):
            _, cr = O.qd_sweep(4, 2, pairs, psi, phi, start[s])
            assert abs(c[s] - cr) <= 1e-10 * max(cr, 1e-3), (sweep, s, c[s], cr)
            for u in host(dg)[s]:
                assert np.max(np.abs(u.conj().T @ u - np.eye(16))) < 1e-12


def test_d4_mixed_teacher_forced():
    say("d=4 mixed teacher-forced n=4")
    n, L, M = 4, 6, 12
    pairs, psi, phi, gates, _ = _problem(4, n, L, M, 2, seed=71)
    dpsi, dphi, dg = dev(psi), dev(phi), dev(gates)
    c_init = max(O.qd_sweep(4, n, pairs, psi, phi, gates[0])[1], 1e-3)
    for sweep in range(4):
        start = host(dg).copy()
        c = Q.qfs_qudit_sweep(4, n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_MIXED)
        new = host(dg)
        for s in range(2):
            _, cr = O.qd_sweep(4, n, pairs, psi, phi, start[s])
            assert abs(c[s] - cr) <= 1e-6 * max(cr, c_init), (sweep, s, c[s], cr)
            for u in new[s]:
                assert np.max(np.abs(u.conj().T @ u - np.eye(16))) < 1e-12


def test_d4_instantiate_follows_oracle():
    """FP64 on a fixed set of 3 ququarts (N = 64): same reason, start, sweeps, doublings,
    final M and cost as the oracle."""
    say("d=4 instantiate vs oracle n=3")
    n = 3
    g = np.random.default_rng(23)
    pairs = [(0, 1), (1, 2)]
    tg = np.stack([I.haar_unitary(16, g) for _ in pairs])
    psi = _samples(4, n, 64, g)
    phi = O.qd_apply_circuit(4, n, psi, pairs, tg)
    p = O.default_params(multistarts=2, m_init=4, seed=8, dist_tol=1e-11, max_iter=400)
    g_ref, ref = O.qd_instantiate(4, n, pairs, psi, phi, n_val=16, params=p)
    g_gpu, got = Q.qfs_qudit_instantiate(4, n, pairs, dev(psi), dev(phi), n_val=16,
                                         params=dict(p, precision=Q.QFS_PREC_FP64))
    for k in ("reason_name", "best_start", "sweeps", "restarts", "m_final"):
        assert got[k] == ref[k], (k, got, ref)
    assert abs(got["c_train"] - ref["c_train"]) <= 1e-9 * max(ref["c_train"], 1e-12) + 1e-20
    assert np.max(np.abs(host(g_gpu) - g_ref)) < 1e-8


def _target_case(d, n, pairs, seed):
    g = np.random.default_rng(seed)
    tg = np.stack([I.haar_unitary(d * d, g) for _ in pairs])
    return tg


@pytest.mark.parametrize("d,n,pairs,form,m_init,starts", [
    (3, 3, [(0, 1), (1, 2), (0, 1), (1, 2)], "dense", 3, 2),
    (3, 3, [(0, 1), (1, 2), (0, 1), (1, 2)], "circuit", 3, 2),
    (3, 4, [(0, 1), (2, 3), (1, 2), (0, 1)], "circuit", 2, 2),
    (4, 3, [(0, 1), (1, 2)], "circuit", 4, 1),
])
def test_qudit_target_instantiate_follows_oracle(d, n, pairs, form, m_init, starts):
    """States drawn on each side (device: Philox + CholeskyQR2; oracle: Philox +
    Gram-Schmidt), targets formed on each side, FP64: same reason, start, sweeps,
    doublings and final M, cost and gates to rounding. Every environment has full rank
    (M d^(n-2) >= d^2), so each update is unique. (The d = 4 case runs one start: there
    every start reaches the exact target, cost ~1e-30, so the pick among starts that
    succeed in the same sweep is decided by rounding.)"""
    say(f"qudit target instantiate d={d} n={n} {form} m_init={m_init} starts={starts}")
    tg = _target_case(d, n, pairs, 50 + d + n)
    p = O.default_params(multistarts=starts, m_init=m_init, seed=9, dist_tol=1e-10, max_iter=300, min_iter=3)
    if form == "dense":
        # row c of the circuit applied to the basis rows is column c of its unitary
        U = O.qd_apply_circuit(d, n, np.eye(d ** n, dtype=np.complex128), pairs, tg).T.copy()
        g_ref, ref = O.qd_instantiate_target(d, n, pairs, U=U, params=p)
        g_gpu, got = Q.qfs_qudit_instantiate_target(d, n, pairs, U=dev(U),
                                                    params=dict(p, precision=Q.QFS_PREC_FP64))
    else:
        g_ref, ref = O.qd_instantiate_target(d, n, pairs, target_pairs=pairs, target_gates=tg, params=p)
        g_gpu, got = Q.qfs_qudit_instantiate_target(d, n, pairs, target_pairs=pairs, target_gates=dev(tg),
                                                    params=dict(p, precision=Q.QFS_PREC_FP64))
    say(f"  oracle {ref['reason_name']} sweeps={ref['sweeps']} restarts={ref['restarts']} "
        f"c={ref['c_train']:.3e}; device {got['reason_name']} sweeps={got['sweeps']} c={got['c_train']:.3e}")
    for k in ("reason_name", "best_start", "sweeps", "restarts", "m_final"):
        assert got[k] == ref[k], (k, got, ref)
    assert ref["restarts"] >= 1
    assert abs(got["c_train"] - ref["c_train"]) <= 1e-8 * ref["c_train"] + 1e-18
    assert abs(got["c_val"] - ref["c_val"]) <= 1e-8 * ref["c_val"] + 1e-18
    assert np.max(np.abs(host(g_gpu) - g_ref)) < 1e-7


def test_qutrit_circuit_target_mixed_reaches_target():
    """complex64 states with complex128 refinement, 5 qutrits, drawn states with doubling:
    success, and the returned gates reproduce the target on fresh states."""
    say("qutrit circuit target mixed n=5")
    n = 5
    pairs = [(0, 1), (2, 3), (1, 2), (3, 4)]
    tg = _target_case(3, n, pairs, 61)
    p = Q.qfs_default_params(multistarts=8, m_init=3, seed=6, dist_tol=1e-9, max_iter=3000)
    gates, info = Q.qfs_qudit_instantiate_target(3, n, pairs, target_pairs=pairs, target_gates=dev(tg),
                                                 params=p)
    say(f"  {info['reason_name']} m_final={info['m_final']} restarts={info['restarts']} refined={info['refined']}")
    assert info["reason_name"] == "SUCCESS", info
    fresh = _samples(3, n, 12, np.random.default_rng(62))
    a = O.qd_apply_circuit(3, n, fresh, pairs, host(gates))
    b = O.qd_apply_circuit(3, n, fresh, pairs, tg)
    assert np.sum(np.abs(a - b) ** 2) / 12 < 1e-7


def test_qudit_target_samples_form_forwards():
    """The SAMPLES form of the target entry is qfs_qudit_instantiate."""
    say("qudit target samples form")
    n = 3
    g = np.random.default_rng(24)
    pairs = [(0, 1), (1, 2)]
    tg = np.stack([I.haar_unitary(9, g) for _ in pairs])
    psi = _samples(3, n, 27, g)
    phi = O.qd_apply_circuit(3, n, psi, pairs, tg)
    p = Q.qfs_default_params(multistarts=2, m_init=9, seed=3, dist_tol=1e-11, max_iter=200,
                             precision=Q.QFS_PREC_FP64)
    ga, ia = Q.qfs_qudit_instantiate(3, n, pairs, dev(psi), dev(phi), n_val=0, params=p)
    gb, ib = Q.qfs_qudit_instantiate_target(3, n, pairs, psi=dev(psi), phi=dev(phi), n_val=0, params=p)
    for k in ("reason_name", "best_start", "sweeps", "restarts", "m_final", "c_train"):
        assert ia[k] == ib[k], k
    assert torch.equal(ga, gb)


# ------------------------------------------------------------------ qudit gate kinds
def _csum(d):
    D = d * d
    U = np.zeros((D, D), dtype=np.complex128)
    for x in range(d):
        for y in range(d):
            U[d * x + (y + x) % d, d * x + y] = 1.0
    return U


def _kind_slots(d, kinds, g):
    out = []
    for k in kinds:
        if k == Q.QFS_GATE_1Q:
            out.append(np.kron(I.haar_unitary(d, g), np.eye(d)))
        elif k == Q.QFS_GATE_FIXED:
            out.append(_csum(d))
        else:
            out.append(I.haar_unitary(d * d, g))
    return np.stack(out)


KIND_PAIRS = [(0, 1), (1, 2), (2, 0), (1, 0), (0, 2), (2, 1), (1, 2)]
KINDS = [1, 2, 0, 1, 2, 1, 0]  # QFS_GATE_1Q, QFS_GATE_FIXED, QFS_GATE_2Q, ...


def test_d2_qudit_kinds_sweep_equals_qubit_kinds_sweep():
    say("qudit d=2 kinds vs qubit kinds sweep")
    g = np.random.default_rng(81)
    n, M = 4, 6
    pairs = [(0, 1), (1, 2), (2, 3), (3, 0), (1, 3), (2, 0)]
    kinds = [1, 2, 0, 1, 0, 2]
    gates = np.stack([_kind_slots(2, kinds, g) for _ in range(2)])
    psi = _samples(2, n, M, g)
    phi = O.apply_circuit(n, psi, pairs, I.haar_gates(6, g))
    a, b = dev(gates), dev(gates)
    for _ in range(4):
        ca = Q.qfs_qudit_sweep(2, n, pairs, dev(psi), dev(phi), a, precision=Q.QFS_PREC_FP64, kinds=kinds)
        cb = Q.qfs_sweep(n, pairs, dev(psi), dev(phi), b, precision=Q.QFS_PREC_FP64, kinds=kinds)
        assert np.max(np.abs(np.asarray(ca) - np.asarray(cb))) <= 1e-12 * max(np.max(cb), 1e-3)
    assert np.max(np.abs(host(a) - host(b))) < 1e-11


@pytest.mark.parametrize("d,n,M,starts", [(3, 3, 4, 2), (3, 5, 3, 2), (4, 3, 4, 1)])
def test_qudit_kinds_fp64_lock_step(d, n, M, starts):
    """One-qudit, constant and two-qudit gates: FP64 lock step with the oracle for 10 sweeps
    (cost and gates 1e-10); constant slots stay bitwise as given, one-qudit slots keep
    the form v (x) I_d."""
    say(f"qudit kinds lock-step d={d} n={n} M={M}")
    g = np.random.default_rng(90 + 10 * d + n)
    pairs = KIND_PAIRS
    gates = np.stack([_kind_slots(d, KINDS, g) for _ in range(starts)])
    psi = _samples(d, n, M, g)
    phi = O.qd_apply_circuit(d, n, psi, pairs, _kind_slots(d, KINDS, g))
    dg, dpsi, dphi = dev(gates), dev(psi), dev(phi)
    ref = gates.copy()
    for sweep in range(10):
        c = Q.qfs_qudit_sweep(d, n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_FP64, kinds=KINDS)
        for s in range(starts):
            ref[s], cr = O.qd_sweep(d, n, pairs, psi, phi, ref[s], kinds=KINDS)
            assert abs(c[s] - cr) <= 1e-10 * max(cr, 1e-3), (sweep, s, c[s], cr)
        got = host(dg)
        assert np.max(np.abs(got - ref)) < 1e-10
    for s in range(starts):
        for k, kind in enumerate(KINDS):
            if kind == Q.QFS_GATE_FIXED:
                assert np.array_equal(got[s, k], _csum(d))
            elif kind == Q.QFS_GATE_1Q:
                v = got[s, k][::d, ::d]
                assert np.array_equal(got[s, k], np.kron(v, np.eye(d)))


def test_qutrit_kinds_mixed_teacher_forced():
    say("qutrit kinds mixed teacher-forced n=5")
    n, M = 5, 8
    g = np.random.default_rng(95)
    pairs = KIND_PAIRS + [(3, 4), (4, 2)]
    kinds = KINDS + [Q.QFS_GATE_2Q, Q.QFS_GATE_1Q]
    gates = np.stack([_kind_slots(3, kinds, g) for _ in range(2)])
    psi = _samples(3, n, M, g)
    phi = O.qd_apply_circuit(3, n, psi, pairs, _kind_slots(3, kinds, g))
    dpsi, dphi, dg = dev(psi), dev(phi), dev(gates)
    c_init = max(O.qd_sweep(3, n, pairs, psi, phi, gates[0], kinds=kinds)[1], 1e-3)
    for sweep in range(4):
        start = host(dg).copy()
        c = Q.qfs_qudit_sweep(3, n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_MIXED, kinds=kinds)
        for s in range(2):
            _, cr = O.qd_sweep(3, n, pairs, psi, phi, start[s], kinds=kinds)
            assert abs(c[s] - cr) <= 1e-6 * max(cr, c_init), (sweep, s, c[s], cr)


def test_qutrit_kinds_instantiate_follows_oracle():
    """Initial gates drawn on each side (one-qutrit Haar slots, CSUM constants), states
    drawn on each side, a circuit target from the same template: same reason, sweeps,
    doublings and final M as the oracle, cost to rounding; the constants kept. One start:
    the target is exactly reachable, so starts that succeed in the same sweep all end at
    the rounding floor (~1e-30) and the pick among them is decided by rounding."""
    say("qutrit kinds instantiate vs oracle")
    n = 3
    g = np.random.default_rng(96)
    tg = _kind_slots(3, KINDS, g)
    fixed = np.stack([_csum(3)] * len(KINDS))
    p = O.default_params(multistarts=1, m_init=3, seed=12, dist_tol=1e-10, max_iter=400, min_iter=3)
    g_ref, ref = O.qd_instantiate_target(3, n, KIND_PAIRS, target_pairs=KIND_PAIRS, target_gates=tg,
                                         params=p, kinds=KINDS, fixed=fixed)
    g_gpu, got = Q.qfs_qudit_instantiate_target(3, n, KIND_PAIRS, target_pairs=KIND_PAIRS,
                                                target_gates=dev(tg), params=dict(p, precision=Q.QFS_PREC_FP64),
                                                kinds=KINDS, fixed_gates=dev(fixed))
    say(f"  oracle {ref['reason_name']} start={ref['best_start']} sweeps={ref['sweeps']} "
        f"restarts={ref['restarts']} c={ref['c_train']:.3e}; device {got['reason_name']} "
        f"start={got['best_start']} sweeps={got['sweeps']} c={got['c_train']:.3e}")
    for k in ("reason_name", "best_start", "sweeps", "restarts", "m_final"):
        assert got[k] == ref[k], (k, got, ref)
    assert abs(got["c_train"] - ref["c_train"]) <= 1e-8 * ref["c_train"] + 1e-18
    out = host(g_gpu)
    assert np.max(np.abs(out - g_ref)) < 1e-7
    for k, kind in enumerate(KINDS):
        if kind == Q.QFS_GATE_FIXED:
            assert np.array_equal(out[k], _csum(3))


def test_qudit_kinds_rejected_when_malformed():
    say("qudit kinds argument checks")
    psi = dev(np.eye(27)[:3])
    with pytest.raises(Q.QfsError) as e:  # constant gates without their matrices
        Q.qfs_qudit_instantiate(3, 3, KIND_PAIRS, psi, psi, params=Q.qfs_default_params(), kinds=KINDS)
    assert e.value.code == Q.QFS_EINVAL
    with pytest.raises(Q.QfsError) as e:
        Q.qfs_qudit_instantiate(3, 3, [(0, 1)], psi, psi, params=Q.qfs_default_params(), kinds=[7])
    assert e.value.code == Q.QFS_EINVAL


def test_qutrit_starts_split_under_a_memory_budget():
    """App. A: when the starts do not fit the device budget they run as two halves, each
    with its own control loop, and the better result is returned. A budget that holds two
    of four starts gives two groups; each group follows the oracle run of its own starts
    (starts 2, 3 through their Haar draws as initial gates)."""
    say("qutrit multistart split under a budget")
    n = 3
    g = np.random.default_rng(97)
    pairs = [(0, 1), (1, 2), (0, 1)]
    tg = np.stack([I.haar_unitary(9, g) for _ in pairs])
    psi = _samples(3, n, 27, g)
    phi = O.qd_apply_circuit(3, n, psi, pairs, tg)
    p = O.default_params(multistarts=4, m_init=3, seed=7, dist_tol=1e-11, max_iter=300)
    g_gpu, got = Q.qfs_qudit_instantiate(3, n, pairs, dev(psi), dev(phi), n_val=9,
                                         params=dict(p, precision=Q.QFS_PREC_FP64, device_mem_budget=800_000))
    assert got["start_groups"] == 2, got
    halves = []
    for s0 in (0, 2):
        gi = np.stack([np.stack([O.qd_haar_gate(3, 7, s, k) for k in range(len(pairs))]) for s in (s0, s0 + 1)])
        gr, ir = O.qd_instantiate(3, n, pairs, psi, phi, n_val=9, params=dict(p, multistarts=2), gates_in=gi)
        ir["best_start"] += s0
        halves.append((gr, ir))
    succ = [h[1]["reason_name"] == "SUCCESS" for h in halves]
    pick = 1 if (succ[1] and not succ[0]) or (succ[0] == succ[1] and halves[1][1]["c_train"] < halves[0][1]["c_train"]) else 0
    g_ref, ref = halves[pick]
    say(f"  halves {[h[1]['reason_name'] for h in halves]}; device {got['reason_name']} start={got['best_start']}")
    for k in ("reason_name", "best_start", "sweeps", "restarts", "m_final"):
        assert got[k] == ref[k], (k, got, ref)
    assert abs(got["c_train"] - ref["c_train"]) <= 1e-9 * max(ref["c_train"], 1e-12) + 1e-20
    assert np.max(np.abs(host(g_gpu) - g_ref)) < 1e-8
    # without the budget all four starts run as one group
    _, one = Q.qfs_qudit_instantiate(3, n, pairs, dev(psi), dev(phi), n_val=9,
                                     params=dict(p, precision=Q.QFS_PREC_FP64))
    assert one["start_groups"] == 1


def test_qudit_batch_equals_one_at_a_time():
    """The batched qudit entry runs problems side by side on streams of their own; each
    problem's result equals that of the single entry with the same params (the same
    kernels on the same starts): circuit targets with drawn states, a fixed sample set,
    and a gate-kinds template."""
    say("qudit batch vs single entries")
    g = np.random.default_rng(98)
    probs = []
    for n, L, seed in ((3, 3, 1), (4, 4, 2), (3, 5, 3), (5, 4, 4)):
        pairs = I.random_pair_template(n, L, np.random.default_rng(seed))
        tg = np.stack([I.haar_unitary(9, g) for _ in pairs])
        probs.append(dict(n=n, pairs=pairs, target_pairs=pairs, target_gates=dev(tg)))
    psi = _samples(3, 3, 27, g)
    tg = np.stack([I.haar_unitary(9, g) for _ in range(3)])
    phi = O.qd_apply_circuit(3, 3, psi, [(0, 1), (1, 2), (0, 2)], tg)
    probs.append(dict(n=3, pairs=[(0, 1), (1, 2), (0, 2)], psi=dev(psi), phi=dev(phi), n_val=9))
    fixed = np.stack([_csum(3)] * len(KINDS))
    probs.append(dict(n=3, pairs=KIND_PAIRS, kinds=KINDS, fixed_gates=dev(fixed), target_pairs=KIND_PAIRS,
                      target_gates=dev(_kind_slots(3, KINDS, g))))
    p = Q.qfs_default_params(multistarts=4, m_init=3, seed=17, dist_tol=1e-10, max_iter=300,
                             precision=Q.QFS_PREC_FP64)
    gb, rb = Q.qfs_qudit_instantiate_batch(3, probs, p)
    for i, pr in enumerate(probs):
        tkeys = {k: pr[k] for k in ("target_pairs", "target_gates", "psi", "phi", "n_val") if k in pr}
        gs, rs = Q.qfs_qudit_instantiate_target(3, pr["n"], pr["pairs"], params=p, kinds=pr.get("kinds"),
                                                fixed_gates=pr.get("fixed_gates"), **tkeys)
        say(f"  problem {i}: {rs['reason_name']} sweeps={rs['sweeps']} batch {rb[i]['reason_name']} "
            f"sweeps={rb[i]['sweeps']}")
        for k in ("reason_name", "best_start", "sweeps", "restarts", "m_final"):
            assert rb[i][k] == rs[k], (i, k, rb[i], rs)
        assert abs(rb[i]["c_train"] - rs["c_train"]) <= 1e-12 * max(rs["c_train"], 1e-12) + 1e-24
        assert np.max(np.abs(host(gb[i]) - host(gs))) < 1e-12
