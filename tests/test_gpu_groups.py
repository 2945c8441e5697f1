"""GPU parity of the grouped backward pass (consecutive gates whose qubits fit in four
share one pass; every environment of the group is derived from one 16 x 16 second-moment
matrix reduced on the matrix cores) against the FP64 CPU oracle, which updates one gate at
a time (Sec. 3; Fig. env_calc_tensor). MI355X only; calls go through the C ABI.

Tolerances as in test_gpu_parity: complex128 states agree with the oracle to 1e-10 over 20
lock-step sweeps (costs and gates); complex64 states are compared teacher-forced to
1e-6 * max(c, c_initial).
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2405_12866_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts only under -m gpu
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


def _groups(pairs):
    """Group boundaries as the library plans them: from the last gate down, each group as
    long as its qubits fit in four (used here only to describe the cases)."""
    out, k = [], len(pairs) - 1
    while k >= 0:
        qs, hi = set(), k
        while k >= 0 and hi - k < 16 and len(qs | set(pairs[k])) <= 4:
            qs |= set(pairs[k])
            k -= 1
        out.append((hi, k + 1, len(qs)))
    return out


def _problem(n, pairs, M, starts, seed):
    g = np.random.default_rng(seed)
    tg = I.haar_gates(len(pairs), g)
    psi = I.orthonormal_samples(n, M, g)
    phi = O.apply_circuit(n, psi, pairs, tg)
    gates = np.stack([I.haar_gates(len(pairs), g) for _ in range(starts)])
    return psi, phi, gates


def _templates():
    g = np.random.default_rng(2024)
    cases = []
    # random pairs: groups whose unions hold 2, 3 and 4 qubits, ragged sample chunks
    for n, L, M, starts in [(4, 7, 5, 2), (5, 11, 9, 2), (6, 13, 3, 1), (8, 17, 16, 2), (10, 9, 6, 2)]:
        cases.append((f"random n={n} L={L}", n, [tuple(p) for p in I.random_pair_template(n, L, g)], M, starts))
    # brickwork (the 12-qubit workload's shape, smaller) and gates on the lowest amplitude bits
    cases.append(("brickwork n=7 depth 4", 7, [tuple(p) for p in I.brickwork_template(7, 4)], 12, 2))
    cases.append(("low bits n=9", 9, [(8, 7), (7, 6), (8, 6), (5, 8), (6, 7), (2, 8), (7, 8), (8, 7)], 5, 2))
    # one gate, and every gate on the same two qubits (one group of 16 gates, then the rest)
    cases.append(("single gate n=5", 5, [(1, 3)], 4, 1))
    cases.append(("same pair x18 n=4", 4, [(2, 0)] * 9 + [(0, 2)] * 9, 6, 1))
    return cases


CASES = _templates()


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
@pytest.mark.parametrize("mode", [Q.QFS_BWD_GROUPED, Q.QFS_BWD_PER_GATE], ids=["grouped", "per_gate"])
def test_fp64_lock_step_both_modes(case, mode):
    """20 complex128 sweeps in lock step with the oracle, grouped and per-gate passes."""
    name, n, pairs, M, starts = CASES[case]
    say(f"groups fp64 lock-step {name} M={M} starts={starts} mode={mode} groups={_groups(pairs)}")
    psi, phi, gates = _problem(n, pairs, M, starts, seed=case + 11)
    dg, dpsi, dphi = dev(gates), dev(psi), dev(phi)
    ref = gates.copy()
    for sweep in range(20):
        c_gpu = Q.qfs_sweep(n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_FP64, backward=mode)
        for s in range(starts):
            ref[s], c_ref = O.sweep(n, pairs, psi, phi, ref[s])
            assert abs(c_gpu[s] - c_ref) <= 1e-10 * max(c_ref, 1e-3), (sweep, s, c_gpu[s], c_ref)
        assert np.max(np.abs(host(dg) - ref)) < 1e-10, sweep


@pytest.mark.parametrize("case", [1, 3, 5, 6])
def test_mixed_teacher_forced_grouped(case):
    """complex64 states (FP32 matrix-core products, FP64 sums): each sweep starts from the
    device's FP64 gates on both sides; |dc| <= 1e-6 max(c, c_initial), gates unitary."""
    name, n, pairs, M, starts = CASES[case]
    say(f"groups mixed teacher-forced {name}")
    psi, phi, gates = _problem(n, pairs, M, starts, seed=case + 50)
    dg, dpsi, dphi = dev(gates), dev(psi), dev(phi)
    c_init = max(O.sweep(n, pairs, psi, phi, gates[0].copy())[1], 1e-3)
    for sweep in range(6):
        start = host(dg).copy()
        c_gpu = Q.qfs_sweep(n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_MIXED)
        new = host(dg)
        for s in range(starts):
            _, c_ref = O.sweep(n, pairs, psi, phi, start[s].copy())
            assert abs(c_gpu[s] - c_ref) <= 1e-6 * max(c_ref, c_init), (sweep, s, c_gpu[s], c_ref)
            for u in new[s]:
                assert np.max(np.abs(u.conj().T @ u - np.eye(4))) < 1e-12


def test_u3_cnot_lock_step_grouped():
    """U3 + CNOT template (one-qubit slots and constant CNOTs in the groups): 20 complex128
    sweeps in lock step; constant gates stay bit-identical."""
    n, M, starts = 6, 8, 2
    pairs, kinds, fixed = I.u3_cnot_template(n, 3)
    say(f"groups u3+cnot fp64 lock-step n={n} L={len(pairs)} groups={_groups([tuple(p) for p in pairs])}")
    g = np.random.default_rng(5)
    tg = I.kinds_target_gates(kinds, fixed, g)
    psi = I.orthonormal_samples(n, M, g)
    phi = O.apply_circuit(n, psi, pairs, tg)
    gates = np.stack([O.initial_gates(9, s, kinds, fixed) for s in range(starts)])
    dg, dpsi, dphi = dev(gates), dev(psi), dev(phi)
    ref = gates.copy()
    fx = kinds == I.GATE_FIXED
    for sweep in range(20):
        c_gpu = Q.qfs_sweep(n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_FP64, kinds=kinds)
        for s in range(starts):
            ref[s], c_ref = O.sweep(n, pairs, psi, phi, ref[s], kinds=kinds)
            assert abs(c_gpu[s] - c_ref) <= 1e-10 * max(c_ref, 1e-3), (sweep, s, c_gpu[s], c_ref)
        got = host(dg)
        assert np.max(np.abs(got - ref)) < 1e-10
        assert np.array_equal(got[:, fx], gates[:, fx])


def test_grouped_is_deterministic():
    """Fixed-order sums: two identical sweeps give bitwise identical gates and costs."""
    n, pairs = 8, [tuple(p) for p in I.brickwork_template(8, 4)]
    say("groups determinism")
    psi, phi, gates = _problem(n, pairs, 32, 3, seed=3)
    dpsi, dphi = dev(psi), dev(phi)
    outs = []
    for _ in range(2):
        dg = dev(gates)
        c = Q.qfs_sweep(n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_MIXED)
        outs.append((host(dg), np.asarray(c)))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_instantiate_grouped_matches_per_gate_control_flow():
    """The control loop on top of either pass (FP64, doubling from M = 2, 4 starts) ends with
    the oracle's start, reason and sweep count."""
    n = 4
    pairs = [(0, 1), (2, 3), (1, 2), (0, 3), (1, 3), (0, 2)]
    g = np.random.default_rng(8)
    tg = I.haar_gates(len(pairs), g)
    say("groups instantiate control flow")
    op = O.default_params(dist_tol=1e-10, multistarts=4, seed=21, max_iter=400)
    _, ref = O.instantiate(n, pairs, target_pairs=pairs, target_gates=tg, params=op)
    for mode in (Q.QFS_BWD_GROUPED, Q.QFS_BWD_PER_GATE):
        p = Q.qfs_default_params(dist_tol=1e-10, multistarts=4, seed=21, max_iter=400,
                                 precision=Q.QFS_PREC_FP64, backward_mode=mode)
        _, info = Q.qfs_instantiate(n, pairs, target_pairs=pairs, target_gates=dev(tg), params=p)
        assert (info["reason_name"], info["sweeps"], info["best_start"], info["m_final"]) == \
            (ref["reason_name"], ref["sweeps"], ref["best_start"], ref["m_final"]), (mode, info, ref)
        assert abs(info["c_train"] - ref["c_train"]) <= 1e-9 * max(ref["c_train"], 1e-6)
