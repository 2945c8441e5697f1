"""The 3-qubit workload on the device against the FP64 oracle (MI355X only).

Workload: 3 qubits, the linear template (0,1),(1,2) repeated three times (L = 6), the
target the same template with Haar 4x4 gates, M = 4 Haar training states, complex128,
sweeps until c_train < 1e-10 or 200 sweeps. Four states fix U only on a
four-dimensional subspace, so with doubling on the generalisation test fails and M
doubles once to 8 = 2^n (Sec. 3: doubling stops at 2^n).

Checked here: lock-step sweeps at M = 4 (free-running for 20 sweeps, then every sweep
teacher-forced from the device's gates up to the stop), the oracle's control flow with
doubling (same start, reason, sweeps, the doubling event, M = 8), and recovery of the
target by 16 starts to d_full < 1e-10 from the dense 8 x 8 products.
"""
import sys

import numpy as np
import pytest

import oracle as O
from brute import dense as D
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


def test_c1_lockstep_sweeps_to_the_stop():
    """1 start, M = 4, FP64 states: free-running lock step for the first 20 sweeps (cost
    1e-10 relative, gates 1e-10), then each further sweep teacher-forced from the
    device's gates (cost 1e-10 relative plus 1e-18 absolute, gates 1e-10) until
    c_train < 1e-10 or 200 sweeps."""
    w = I.workload_3q()
    pairs = w["pairs"]
    psi = O.draw_states(3, 4, seed=0x5A17 + 1)
    phi = O.apply_circuit(3, psi, pairs, w["target_gates"])
    g0 = np.stack([O.haar_gate(0x5A17 + 1, 0, k) for k in range(len(pairs))])
    dpsi, dphi = dev(psi), dev(phi)
    dg = dev(g0[None])
    ref = g0.copy()
    sweeps, c = 0, np.inf
    for t in range(200):
        start = host(dg)[0]
        c_dev = Q.qfs_sweep(3, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_FP64)[0]
        got = host(dg)[0]
        if t < 20:
            ref, c_ref = O.sweep(3, pairs, psi, phi, ref)
            assert abs(c_dev - c_ref) <= 1e-10 * max(c_ref, 1e-12), (t, c_dev, c_ref)
            assert np.max(np.abs(got - ref)) < 1e-10, t
        else:
            g_tf, c_tf = O.sweep(3, pairs, psi, phi, start)
            # near the solution the difference form loses relative accuracy: |a - psi|
            # is about sqrt(c) with an FP64 rounding of about 1e-15, so |dc| is about
            # 2 sqrt(c) 1e-15 (2e-20 at c = 1e-10); 1e-18 absolute covers it 50-fold
            assert abs(c_dev - c_tf) <= 1e-10 * c_tf + 1e-18, (t, c_dev, c_tf)
            assert np.max(np.abs(got - g_tf)) < 1e-10, t
        sweeps, c = t + 1, c_dev
        if c < 1e-10:
            break
    say(f"  c_train {c:.3e} after {sweeps} sweeps")
    assert c < 1e-10 or sweeps == 200


def test_c1_control_flow_with_the_doubling():
    """Doubling on (m_init = 4): the device run follows the oracle's run with the same
    seed: same returned start, reason, sweep count and doublings; M ends at 8 = 2^n;
    costs 1e-9 relative (absolute 1e-20 at exact solutions)."""
    w = I.workload_3q()
    kw = dict(dist_tol=1e-10, multistarts=1, seed=0x5A17 + 1, max_iter=200, m_init=4)
    g, got = Q.qfs_instantiate(3, w["pairs"], target_pairs=w["target_pairs"],
                               target_gates=dev(w["target_gates"]),
                               params=Q.qfs_default_params(precision=Q.QFS_PREC_FP64, **kw))
    g_ref, ref = O.instantiate(3, w["pairs"], target_pairs=w["target_pairs"],
                               target_gates=w["target_gates"], params=O.default_params(**kw),
                               trace_capacity=1000, doubling_capacity=4)
    say(f"  device {got['reason_name']} after {got['sweeps']} sweeps, {got['restarts']} doublings, "
        f"M={got['m_final']}; oracle {ref['reason_name']} / {ref['sweeps']} / {ref['restarts']} / "
        f"{ref['m_final']}")
    assert ref["restarts"] == 1 and ref["m_final"] == 8
    dbl = ref["trace"]["doublings"][0]
    assert (dbl["m_old"], dbl["m_new"]) == (4, 8)
    for key in ("reason", "sweeps", "restarts", "m_final", "best_start", "m_total"):
        assert got[key] == ref[key], (key, got[key], ref[key])
    for key in ("c_train", "c_val"):
        assert abs(got[key] - ref[key]) <= 1e-9 * ref[key] + 1e-20, (key, got[key], ref[key])
    # the doubling happened at the oracle's sweep: the last sweep at M = 4 is the
    # first one allowed to test for overtraining
    tr = ref["trace"]
    at4 = tr["sweep"][tr["m"] == 4]
    assert at4.max() >= 6


def test_c1_recovery_with_16_starts():
    """Pin P12 on the device: the target built from the template is recovered by the
    best of 16 starts, d_full from the dense 8 x 8 products below 1e-10 (doubling on,
    FP64 and MIXED with complex128 refinement)."""
    w = I.workload_3q()
    U = D.circuit_matrix(3, w["target_pairs"], w["target_gates"])
    for prec in (Q.QFS_PREC_FP64, Q.QFS_PREC_MIXED):
        # the last decades of this template converge slowly (the oracle's best start
        # needs about 3900 sweeps), so the plateau test is loosened to 1e-7
        p = Q.qfs_default_params(dist_tol=1e-10, multistarts=16, seed=0x5A17 + 1, max_iter=10000,
                                 m_init=4, diff_tol_r=1e-7, precision=prec)
        g, info = Q.qfs_instantiate(3, w["pairs"], target_pairs=w["target_pairs"],
                                    target_gates=dev(w["target_gates"]), params=p)
        C = D.circuit_matrix(3, w["pairs"], host(g))
        d = D.full_distance(U, C)
        say(f"  precision {prec}: {info['reason_name']} after {info['sweeps']} sweeps, "
            f"M={info['m_final']}, d_full {d:.2e}")
        assert info["reason_name"] == "SUCCESS"
        assert d < 1e-10
