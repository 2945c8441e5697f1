"""GPU parity of the qudit path (Sec. 5: the method on d-level gates) against the FP64
oracle's qudit functions, through the C ABI.

d = 2 must reproduce the qubit path; d = 3 (qutrits) runs in lock step with the oracle
(FP64: cost and gates 1e-10 over 10 sweeps; complex64 states teacher-forced,
|dc| <= 1e-6 max(c, c_initial)), follows its control flow, and handles a rank-deficient
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
    psi = dev(np.eye(16)[:2])
    with pytest.raises(Q.QfsError) as e:
        Q.qfs_qudit_instantiate(4, 2, [(0, 1)], psi, psi, params=Q.qfs_default_params())
    assert e.value.code == Q.QFS_EUNSUPPORTED
    psi = dev(np.eye(9)[:2])
    with pytest.raises(Q.QfsError) as e:
        Q.qfs_qudit_instantiate(3, 2, [(0, 0)], psi, psi, params=Q.qfs_default_params())
    assert e.value.code == Q.QFS_EINVAL
