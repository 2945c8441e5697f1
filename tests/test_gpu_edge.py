"""GPU edge cases against the FP64 oracle: a single training state, the full basis,
repeated and reversed gate pairs, a fixed sample set without a validation part, a
one-sweep budget, the smallest problem in the batched engine, and host-forced stops
(time budget). Every case runs the HIP path through the C ABI.
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
    return t.detach().cpu().numpy()


def _lockstep(n, pairs, M, starts, seed, sweeps=10):
    g = np.random.default_rng(seed)
    tg = I.haar_gates(len(pairs), g)
    psi = I.orthonormal_samples(n, M, g)
    phi = O.apply_circuit(n, psi, pairs, tg)
    gates = np.stack([I.haar_gates(len(pairs), g) for _ in range(starts)])
    dg, dpsi, dphi = dev(gates), dev(psi), dev(phi)
    ref = gates.copy()
    for sweep in range(sweeps):
        c_gpu = Q.qfs_sweep(n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_FP64)
        for s in range(starts):
            ref[s], c_ref = O.sweep(n, pairs, psi, phi, ref[s])
            assert abs(c_gpu[s] - c_ref) <= 1e-10 * max(c_ref, 1e-3), (sweep, s, c_gpu[s], c_ref)
    assert np.max(np.abs(host(dg) - ref)) < 1e-10


def test_single_training_state():
    say("lock step with M = 1")
    _lockstep(4, I.random_pair_template(4, 5, np.random.default_rng(1)), 1, 2, seed=11)


def test_repeated_and_reversed_pairs():
    say("lock step with a repeated pair and its reversal")
    pairs = [(0, 1), (0, 1), (1, 0), (2, 1), (1, 2), (1, 2)]
    _lockstep(3, pairs, 3, 2, seed=12)


def test_full_basis_cost_is_the_full_distance():
    """M = 2^n: the training cost is the full distance (Eq. 1 over 2^n), success needs
    no validation (the basis is complete), and the returned gates reproduce the target."""
    say("full basis instantiation, 3 qubits")
    pairs = [(0, 1), (1, 2), (0, 2)]
    tg = I.haar_gates(3, np.random.default_rng(13))
    p = Q.qfs_default_params(m_init=8, multistarts=4, seed=5, dist_tol=1e-11, max_iter=500,
                             precision=Q.QFS_PREC_FP64)
    g, info = Q.qfs_instantiate(3, pairs, target_pairs=pairs, target_gates=dev(tg), params=p)
    assert info["reason_name"] == "SUCCESS" and info["m_final"] == 8 and info["restarts"] == 0
    basis = np.eye(8, dtype=np.complex128)
    d = O.state_distance(3, O.apply_circuit(3, basis, pairs, host(g)), O.apply_circuit(3, basis, pairs, tg))
    assert abs(d - info["c_train"]) <= 1e-12 + 1e-6 * d
    assert d < 1e-11


def test_samples_without_validation_follow_oracle():
    """A fixed sample set with n_val = 0: no validation cost, the success test is the
    training cost alone; the GPU control flow follows the oracle's."""
    say("samples target, no validation rows")
    n = 4
    g = np.random.default_rng(14)
    pairs = I.random_pair_template(n, 4, g)
    tg = I.haar_gates(4, g)
    psi = I.orthonormal_samples(n, 6, g)
    phi = O.apply_circuit(n, psi, pairs, tg)
    kw = dict(multistarts=3, seed=8, max_iter=300, dist_tol=1e-10, diff_tol_r=1e-6)
    g_ref, ref = O.instantiate(n, pairs, psi=psi, phi=phi, n_val=0, params=O.default_params(**kw))
    g_gpu, got = Q.qfs_instantiate(n, pairs, psi=dev(psi), phi=dev(phi), n_val=0,
                                   params=Q.qfs_default_params(precision=Q.QFS_PREC_FP64, **kw))
    assert got["reason_name"] == ref["reason_name"]
    assert got["sweeps"] == ref["sweeps"] and got["best_start"] == ref["best_start"]
    assert abs(got["c_train"] - ref["c_train"]) <= 1e-9 * max(ref["c_train"], 1e-12) + 1e-18


def test_one_sweep_budget():
    say("max_iter = 1")
    pairs = [(0, 1), (1, 2)]
    tg = I.haar_gates(2, np.random.default_rng(15))
    kw = dict(multistarts=2, seed=9, max_iter=1, m_init=4)
    _, ref = O.instantiate(3, pairs, target_pairs=pairs, target_gates=tg, params=O.default_params(**kw))
    _, got = Q.qfs_instantiate(3, pairs, target_pairs=pairs, target_gates=dev(tg),
                               params=Q.qfs_default_params(precision=Q.QFS_PREC_FP64, **kw))
    assert ref["sweeps"] == got["sweeps"] == 1
    assert got["reason_name"] == ref["reason_name"]
    assert abs(got["c_train"] - ref["c_train"]) <= 1e-10 * max(ref["c_train"], 1e-12)


def test_batched_smallest_problem_is_exact_after_one_sweep():
    """n = 2, one gate, full basis: the environment is U itself, so one sweep returns U
    (the special case pinned on the oracle); the batched engine stops at sweep 1."""
    say("batched n = 2, L = 1")
    U = I.haar_unitary(4, np.random.default_rng(16))
    params = Q.qfs_default_params(multistarts=2, seed=1, m_init=4, precision=Q.QFS_PREC_FP64,
                                  batch_sweeps=1, dist_tol=1e-12)
    gates, infos = Q.qfs_instantiate_batch([dict(n=2, pairs=[(0, 1)], U=dev(U))], params)
    assert infos[0]["reason_name"] == "SUCCESS" and infos[0]["sweeps"] == 1
    assert np.max(np.abs(host(gates[0])[0] - U)) < 1e-12


def test_time_budget_stops_with_timeout():
    """A budget already spent stops every start after its first sweep with TIMEOUT (the
    stop is taken on the host; every kernel ends normally)."""
    say("time budget")
    n = 6
    g = np.random.default_rng(17)
    pairs = I.random_pair_template(n, 12, g)
    tg = dev(I.haar_gates(12, g))
    p = Q.qfs_default_params(multistarts=4, seed=2, max_iter=100000, time_budget_s=1e-9,
                             dist_tol=1e-14)
    _, info = Q.qfs_instantiate(n, pairs, target_pairs=pairs, target_gates=tg, params=p)
    assert info["reason_name"] == "TIMEOUT" and info["sweeps"] >= 1
    _, infos = Q.qfs_instantiate_batch([dict(n=n, pairs=pairs, target_pairs=pairs, target_gates=tg)], p)
    assert infos[0]["reason_name"] == "TIMEOUT"
