"""GPU parity of the full-unitary QFactor mode (params full_unitary = 1, Sec. 2.1): the
training set is the complete computational basis, so the sweep is QFactor's and c_train
is the full distance ||U - C||_F^2 / 2^n. Compared with the oracle run on the same basis
as a fixed sample set (the oracle's full-basis sweep is pinned to the dense full-unitary
QFactor sweep of the brute-force checker).
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


def _oracle_qfactor(n, pairs, U, p, kinds=None, fixed=None):
    N = 1 << n
    basis = np.eye(N, dtype=np.complex128)
    return O.instantiate(n, pairs, psi=basis, phi=basis @ U.T, n_val=0,
                         params=dict(p, m_init=N), kinds=kinds, fixed=fixed)


@pytest.mark.parametrize("n,L,seed", [(3, 4, 1), (4, 6, 2)])
def test_full_unitary_fp64_matches_oracle(n, L, seed):
    """Dense target, FP64: same start, reason, sweeps as the oracle on the basis, cost to
    1e-9 relative, gates to 1e-8; M reported as 2^n, no doubling."""
    say(f"full-unitary fp64 n={n} L={L}")
    g = np.random.default_rng(seed)
    pairs = I.random_pair_template(n, L, g)
    U = I.circuit_unitary_columns(n, pairs, I.haar_gates(L, g), np.eye(1 << n)).T
    p = O.default_params(dist_tol=1e-11, multistarts=4, seed=seed, max_iter=1500, diff_tol_r=1e-7)
    g_ref, ref = _oracle_qfactor(n, pairs, U, p)
    g_gpu, got = Q.qfs_instantiate(n, pairs, U=dev(U), params=dict(p, precision=Q.QFS_PREC_FP64,
                                                                   full_unitary=1))
    assert got["reason_name"] == ref["reason_name"]
    assert got["best_start"] == ref["best_start"] and got["sweeps"] == ref["sweeps"]
    assert got["m_final"] == 1 << n and got["restarts"] == 0
    assert abs(got["c_train"] - ref["c_train"]) <= 1e-9 * max(ref["c_train"], 1e-12) + 1e-20
    assert np.max(np.abs(host(g_gpu) - g_ref)) < 1e-8


def test_full_unitary_cost_is_full_distance():
    """c_train of the full-unitary mode is ||U - C||_F^2 / 2^n of the returned gates (Eq. 1
    over 2^n), here after a budget of 3 sweeps (MAX_ITER)."""
    say("full-unitary cost = full distance")
    n, L = 5, 8
    g = np.random.default_rng(3)
    pairs = I.random_pair_template(n, L, g)
    U = I.haar_unitary(1 << n, g)
    p = Q.qfs_default_params(multistarts=2, seed=4, max_iter=3, precision=Q.QFS_PREC_FP64, full_unitary=1)
    gates, info = Q.qfs_instantiate(n, pairs, U=dev(U), params=p)
    assert info["reason_name"] == "MAX_ITER" and info["sweeps"] == 3
    C = I.circuit_unitary_columns(n, pairs, host(gates), np.eye(1 << n)).T
    d_full = np.linalg.norm(U - C) ** 2 / (1 << n)
    assert abs(info["c_train"] - d_full) < 1e-12


def test_full_unitary_u3_cnot_mixed():
    """The U3 + CNOT template of 6 qubits in the full-unitary mode with complex64 states and
    complex128 refinement: success with the full distance <= 1e-8 and constants kept."""
    say("full-unitary mixed 6q U3+CNOT")
    n = 6
    w = I.workload_u3_cnot(n, 3)
    p = Q.qfs_default_params(multistarts=8, seed=5, max_iter=3000, dist_tol=1e-9, full_unitary=1)
    gates, info = Q.qfs_instantiate(n, w["pairs"], target_pairs=w["target_pairs"],
                                    target_gates=dev(w["target_gates"]), params=p, kinds=w["kinds"],
                                    fixed_gates=dev(w["fixed"]))
    assert info["reason_name"] == "SUCCESS", info
    G = host(gates)
    fx = w["kinds"] == I.GATE_FIXED
    assert np.array_equal(G[fx], w["fixed"][fx])
    basis = np.eye(1 << n)
    d = O.state_distance(n, O.apply_circuit(n, basis, w["pairs"], G),
                         O.apply_circuit(n, basis, w["target_pairs"], w["target_gates"]))
    assert d <= 1e-8


def test_full_unitary_rejects_sample_targets():
    say("full-unitary with a sample target")
    psi = dev(np.eye(4)[:2])
    with pytest.raises(Q.QfsError) as e:
        Q.qfs_instantiate(2, [(0, 1)], psi=psi, phi=psi, params=Q.qfs_default_params(full_unitary=1))
    assert e.value.code == Q.QFS_EINVAL
