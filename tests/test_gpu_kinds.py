"""GPU parity for templates with variable one-qubit gates and constant gates (U3 + CNOT
style circuits, Sec. 4): the HIP path through the C ABI against the FP64 oracle.

A one-qubit gate's slot is v (x) I_2 on (qubit, spectator); the device reduces the 4x4
environment on that pair and takes its trace over the spectator, the oracle contracts
the 2x2 environment directly. Constant gates are only applied. Tolerances as in the
two-qubit parity tests: FP64 lock step 1e-10 over 20 sweeps; complex64 states
teacher-forced, |dc| <= 1e-6 max(c, c_initial).
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


def _mixed_problem(n, L, M, starts, seed, ends_fixed=False):
    g = np.random.default_rng(seed)
    pairs = I.random_pair_template(n, L, g)
    kinds = g.integers(0, 3, size=L).astype(np.int32)
    kinds[: min(3, L)] = [1, 2, 0][: min(3, L)]
    g.shuffle(kinds)
    if ends_fixed:
        kinds[0] = kinds[-1] = I.GATE_FIXED
    fixed = np.stack([I.haar_unitary(4, g) for _ in range(L)])
    tg = I.kinds_target_gates(kinds, fixed, g)
    psi = I.orthonormal_samples(n, M, g)
    phi = O.apply_circuit(n, psi, pairs, tg)
    gates = np.stack([O.initial_gates(seed, s, kinds, fixed) for s in range(starts)])
    return pairs, kinds, psi, phi, gates


@pytest.mark.parametrize("n,L,M,starts,ends_fixed", [(2, 3, 4, 1, False), (4, 9, 3, 2, True),
                                                     (7, 14, 6, 2, False), (9, 16, 5, 2, True),
                                                     (10, 12, 3, 1, False)])
def test_fp64_lock_step_with_kinds(n, L, M, starts, ends_fixed):
    """20 FP64 sweeps in lock step: costs and gates within 1e-10; constant gates stay
    bit-identical and one-qubit slots keep the v (x) I_2 form on the device."""
    say(f"kinds fp64 lock-step n={n} L={L} M={M} starts={starts} ends_fixed={ends_fixed}")
    pairs, kinds, psi, phi, gates = _mixed_problem(n, L, M, starts, seed=n + L, ends_fixed=ends_fixed)
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
        for k in np.flatnonzero(kinds == I.GATE_1Q):
            v = got[:, k, 0::2, 0::2]
            assert np.max(np.abs(got[:, k] - np.stack([np.kron(x, np.eye(2)) for x in v]))) < 1e-15


def _folding_template():
    """n = 5: constant gates whose backward step folds into the next one (the gate after
    them on the same two qubits, in the same or the opposite order), and constant gates
    that cannot fold (different qubits after them, a constant gate before them, the last
    gate, the first gate)."""
    pairs = [(0, 1), (1, 2), (1, 2), (3, 4), (2, 3), (3, 2), (0, 4), (0, 1), (1, 0), (2, 4),
             (2, 4), (4, 1), (3, 1), (3, 0)]
    kinds = [I.GATE_FIXED, I.GATE_2Q, I.GATE_FIXED, I.GATE_2Q, I.GATE_FIXED, I.GATE_1Q,
             I.GATE_2Q, I.GATE_FIXED, I.GATE_2Q, I.GATE_FIXED, I.GATE_FIXED, I.GATE_1Q,
             I.GATE_2Q, I.GATE_FIXED]
    return np.asarray(pairs, dtype=np.int32), np.asarray(kinds, dtype=np.int32)


@pytest.mark.parametrize("precision", [Q.QFS_PREC_FP64, Q.QFS_PREC_MIXED])
def test_folded_constant_steps_follow_oracle(precision):
    """The backward step of a constant gate is folded into the next step when the gate
    after it acts on the same two qubits (the device applies u_k^dag u_{k+1}^dag in one
    pass, the oracle one gate at a time). FP64: 20 sweeps in lock step to 1e-10;
    complex64 states: teacher-forced to 1e-6 max(c, c_initial)."""
    say(f"folded constant steps, precision={precision}")
    n, M, starts = 5, 7, 2
    pairs, kinds = _folding_template()
    L = len(pairs)
    g = np.random.default_rng(77)
    fixed = np.stack([I.haar_unitary(4, g) for _ in range(L)])
    tg = I.kinds_target_gates(kinds, fixed, g)
    psi = I.orthonormal_samples(n, M, g)
    phi = O.apply_circuit(n, psi, pairs, tg)
    gates = np.stack([O.initial_gates(5, s, kinds, fixed) for s in range(starts)])
    dg, dpsi, dphi = dev(gates), dev(psi), dev(phi)
    ref = gates.copy()
    c_init = max(O.sweep(n, pairs, psi, phi, gates[0].copy(), kinds=kinds)[1], 1e-3)
    for sweep in range(20 if precision == Q.QFS_PREC_FP64 else 6):
        start = host(dg).copy()
        c_gpu = Q.qfs_sweep(n, pairs, dpsi, dphi, dg, precision=precision, kinds=kinds)
        for s in range(starts):
            if precision == Q.QFS_PREC_FP64:
                ref[s], c_ref = O.sweep(n, pairs, psi, phi, ref[s], kinds=kinds)
                assert abs(c_gpu[s] - c_ref) <= 1e-10 * max(c_ref, 1e-3), (sweep, s, c_gpu[s], c_ref)
            else:
                _, c_ref = O.sweep(n, pairs, psi, phi, start[s].copy(), kinds=kinds)
                assert abs(c_gpu[s] - c_ref) <= 1e-6 * max(c_ref, c_init), (sweep, s, c_gpu[s], c_ref)
        if precision == Q.QFS_PREC_FP64:
            assert np.max(np.abs(host(dg) - ref)) < 1e-10


def test_mixed_u3_cnot_teacher_forced():
    """complex64 states on an 8-qubit U3 + CNOT template (4 sublayers, 14 CNOTs and 36
    one-qubit gates): each sweep from the device's own FP64 gates on both sides."""
    say("kinds mixed teacher-forced 8q U3+CNOT")
    w = I.workload_u3_cnot(8, 4)
    n, pairs, kinds = 8, w["pairs"], w["kinds"]
    g = np.random.default_rng(80)
    psi = I.orthonormal_samples(n, 32, g)
    phi = O.apply_circuit(n, psi, pairs, w["target_gates"])
    gates = np.stack([O.initial_gates(81, s, kinds, w["fixed"]) for s in range(2)])
    dpsi, dphi, dg = dev(psi), dev(phi), dev(gates)
    c_init = max(O.sweep(n, pairs, psi, phi, gates[0], kinds=kinds)[1], 1e-3)
    for sweep in range(6):
        start = host(dg).copy()
        c_gpu = Q.qfs_sweep(n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_MIXED, kinds=kinds)
        new = host(dg)
        for s in range(2):
            _, c_ref = O.sweep(n, pairs, psi, phi, start[s], kinds=kinds)
            assert abs(c_gpu[s] - c_ref) <= 1e-6 * max(c_ref, c_init), (sweep, s, c_gpu[s], c_ref)
            for u in new[s]:
                assert np.max(np.abs(u.conj().T @ u - np.eye(4))) < 1e-12


CNOT_A = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=np.complex128)
CNOT_B = np.array([[1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0], [0, 1, 0, 0]], dtype=np.complex128)
SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)


def test_mixed_constant_gate_forms_teacher_forced():
    """complex64 states on a random-pair template whose constant gates are CNOTs with the
    control on either qubit of the pair (applied as amplitude exchanges in the grouped
    forward pass), SWAPs and Haar 4x4 gates (applied as dense products), among one- and
    two-qubit variable gates: each sweep teacher-forced against the oracle."""
    say("kinds mixed teacher-forced: CNOT forms")
    n, L, M, starts = 8, 40, 32, 2
    g = np.random.default_rng(90)
    pairs = I.random_pair_template(n, L, g)
    kinds = np.array([I.GATE_FIXED, I.GATE_1Q, I.GATE_2Q, I.GATE_1Q] * (L // 4), dtype=np.int32)
    forms = [CNOT_A, CNOT_B, SWAP, None]
    fixed = np.stack([forms[(k // 4) % 4] if forms[(k // 4) % 4] is not None else I.haar_unitary(4, g)
                      for k in range(L)])
    tg = I.kinds_target_gates(kinds, fixed, g)
    psi = I.orthonormal_samples(n, M, g)
    phi = O.apply_circuit(n, psi, pairs, tg)
    gates = np.stack([O.initial_gates(91, s, kinds, fixed) for s in range(starts)])
    dpsi, dphi, dg = dev(psi), dev(phi), dev(gates)
    c_init = max(O.sweep(n, pairs, psi, phi, gates[0], kinds=kinds)[1], 1e-3)
    for sweep in range(6):
        start = host(dg).copy()
        c_gpu = Q.qfs_sweep(n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_MIXED, kinds=kinds)
        new = host(dg)
        for s in range(starts):
            _, c_ref = O.sweep(n, pairs, psi, phi, start[s], kinds=kinds)
            assert abs(c_gpu[s] - c_ref) <= 1e-6 * max(c_ref, c_init), (sweep, s, c_gpu[s], c_ref)
            for k in range(L):
                if kinds[k] == I.GATE_FIXED:
                    assert np.array_equal(new[s][k], fixed[k]), (sweep, s, k)


def test_instantiate_u3_cnot_fp64_matches_oracle_control_flow():
    """Initial one-qubit gates drawn on the device as on the oracle (Haar 2x2 from the same
    counter stream), then the same control flow: reason, start, sweeps, doublings, cost."""
    say("kinds instantiate fp64 vs oracle (3q U3+CNOT)")
    w = I.workload_u3_cnot(3, 2, seed_base=0x5A17 + 63)
    p = O.default_params(dist_tol=1e-11, multistarts=4, seed=6, max_iter=2000, diff_tol_r=1e-7)
    g_ref, ref = O.instantiate(3, w["pairs"], target_pairs=w["target_pairs"],
                               target_gates=w["target_gates"], params=p, kinds=w["kinds"],
                               fixed=w["fixed"])
    qp = dict(p, precision=Q.QFS_PREC_FP64)
    g_gpu, got = Q.qfs_instantiate(3, w["pairs"], target_pairs=w["target_pairs"],
                                   target_gates=dev(w["target_gates"]), params=qp, kinds=w["kinds"],
                                   fixed_gates=dev(w["fixed"]))
    assert got["reason_name"] == ref["reason_name"] == "SUCCESS"
    assert got["best_start"] == ref["best_start"] and got["sweeps"] == ref["sweeps"]
    assert got["m_final"] == ref["m_final"] and got["restarts"] == ref["restarts"]
    assert abs(got["c_train"] - ref["c_train"]) < 1e-9 * max(ref["c_train"], 1e-12) + 1e-20
    assert np.max(np.abs(host(g_gpu) - g_ref)) < 1e-8


def test_instantiate_u3_cnot_mixed_reaches_distance():
    """MIXED precision on a 7-qubit U3 + CNOT template: success, refinement, constant
    gates returned unchanged, and d_full <= 1e-8 by the oracle's simulation."""
    say("kinds instantiate mixed 7q U3+CNOT")
    n = 7
    w = I.workload_u3_cnot(n, 3)
    qp = Q.qfs_default_params(dist_tol=1e-9, multistarts=8, seed=4, max_iter=4000, m_init=4,
                              diff_tol_r=1e-7)
    g_gpu, info = Q.qfs_instantiate(n, w["pairs"], target_pairs=w["target_pairs"],
                                    target_gates=dev(w["target_gates"]), params=qp, kinds=w["kinds"],
                                    fixed_gates=dev(w["fixed"]))
    assert info["reason_name"] == "SUCCESS", info
    gates = host(g_gpu)
    fx = w["kinds"] == I.GATE_FIXED
    assert np.array_equal(gates[fx], w["fixed"][fx])
    psi = O.draw_states(n, 1 << n, seed=556)
    d_full = O.state_distance(n, O.apply_circuit(n, psi, w["pairs"], gates),
                              O.apply_circuit(n, psi, w["target_pairs"], w["target_gates"]))
    assert d_full <= 1e-8


def test_gates_in_and_fixed_gates_validated():
    say("kinds input validation")
    pairs = [(0, 1), (1, 0)]
    kinds = [I.GATE_1Q, I.GATE_FIXED]
    U = dev(np.eye(4))
    p = Q.qfs_default_params(multistarts=1)
    good_fixed = dev(np.stack([np.eye(4), I.CNOT]))
    not_kron = dev(np.stack([I.haar_unitary(4, np.random.default_rng(1)), np.eye(4)])[None])
    with pytest.raises(Q.QfsError) as e:
        Q.qfs_instantiate(2, pairs, U=U, params=p, kinds=kinds, fixed_gates=good_fixed, gates_in=not_kron)
    assert e.value.code == Q.QFS_EINVAL and "v (x) I_2" in str(e.value)
    bad_fixed = dev(np.stack([np.eye(4), 2 * np.eye(4)]))
    with pytest.raises(Q.QfsError) as e:
        Q.qfs_instantiate(2, pairs, U=U, params=p, kinds=kinds, fixed_gates=bad_fixed)
    assert e.value.code == Q.QFS_EINVAL and "fixed_gates" in str(e.value)


def test_all_constant_template_keeps_gates():
    """A template without variable gates: a sweep changes nothing and returns the cost of
    the constant circuit."""
    say("kinds all constant")
    n = 4
    g = np.random.default_rng(3)
    pairs = I.random_pair_template(n, 5, g)
    kinds = np.full(5, I.GATE_FIXED, dtype=np.int32)
    gates = np.stack([I.haar_gates(5, g)])
    psi = I.orthonormal_samples(n, 4, g)
    phi = O.apply_circuit(n, psi, pairs, I.haar_gates(5, g))
    dg = dev(gates)
    c = Q.qfs_sweep(n, pairs, dev(psi), dev(phi), dg, precision=Q.QFS_PREC_FP64, kinds=kinds)
    assert np.array_equal(host(dg), gates)
    ref = O.state_distance(n, O.apply_circuit(n, psi, pairs, gates[0]), phi)
    assert abs(c[0] - ref) < 1e-12


def test_full_size_u3_cnot_sweep_sampled_start():
    """12-qubit U3 + CNOT template (8 sublayers: 44 CNOTs, 100 one-qubit gates) at M = 256
    with 16 starts, complex64 states: one device sweep; one start re-run by the oracle from
    the same gates (teacher forced); every slot unitary; constant gates unchanged; and a
    second sweep lowers no start's cost."""
    n, M, S = 12, 256, 16
    w = I.workload_u3_cnot(n, 8)
    pairs, kinds = w["pairs"], w["kinds"]
    g = np.random.default_rng(1213)
    say("full size U3+CNOT: drawing 12q states")
    psi = I.orthonormal_samples(n, M, g)
    phi = O.apply_circuit(n, psi, pairs, w["target_gates"])
    gates = np.stack([O.initial_gates(1214, s, kinds, w["fixed"]) for s in range(S)])
    dpsi, dphi, dg = dev(psi), dev(phi), dev(gates)
    say("full size U3+CNOT: GPU sweep (16 starts, MIXED)")
    c_gpu = Q.qfs_sweep(n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_MIXED, kinds=kinds)
    new = host(dg)
    fx = kinds == I.GATE_FIXED
    assert np.array_equal(new[:, fx], gates[:, fx])
    for s in range(S):
        for u in new[s]:
            assert np.max(np.abs(u.conj().T @ u - np.eye(4))) < 1e-12
    s = 5
    say(f"full size U3+CNOT: oracle sweep of start {s}")
    c0 = O.state_distance(n, O.apply_circuit(n, psi, pairs, gates[s]), phi)
    _, c_ref = O.sweep(n, pairs, psi, phi, gates[s], kinds=kinds)
    assert abs(c_gpu[s] - c_ref) <= 1e-6 * max(c_ref, c0), (s, c_gpu[s], c_ref)
    say("full size U3+CNOT: second sweep")
    c2 = Q.qfs_sweep(n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_MIXED, kinds=kinds)
    assert np.all(c2 <= c_gpu + 1e-6 * np.maximum(c_gpu, 1e-3))


# ------------------------------------------------------------------ batched engine
def _kind_problems(count, seed):
    """U3 + CNOT templates and random mixed-kind templates of 3-6 qubits."""
    g = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = 3 + i % 4
        if i % 2 == 0:
            w = I.workload_u3_cnot(n, 1 + i % 3, seed_base=0x5A17 + 80 + i)
            out.append((n, w["pairs"], w["kinds"], w["fixed"], w["target_gates"]))
        else:
            L = 4 + i % 5
            pairs = I.random_pair_template(n, L, g)
            kinds = g.integers(0, 3, size=L).astype(np.int32)
            kinds[0] = I.GATE_1Q
            fixed = np.stack([I.haar_unitary(4, g) for _ in range(L)])
            out.append((n, pairs, kinds, fixed, I.kinds_target_gates(kinds, fixed, g)))
    return out


def test_batched_kinds_one_sweep_per_launch_follows_oracle():
    """FP64 states, one sweep per launch: every problem follows the oracle's control flow
    (its own seed params.seed + p, initial one-qubit gates drawn as on the oracle)."""
    say("kinds batched K=1 vs oracle")
    probs = _kind_problems(6, 90)
    bp = Q.qfs_default_params(dist_tol=1e-10, multistarts=3, seed=50, max_iter=400,
                              precision=Q.QFS_PREC_FP64, batch_sweeps=1)
    dprobs = [dict(n=n, pairs=pr, kinds=k, fixed_gates=dev(f), target_pairs=pr, target_gates=dev(tg))
              for n, pr, k, f, tg in probs]
    gates, infos = Q.qfs_instantiate_batch(dprobs, bp)
    for i, (n, pr, k, f, tg) in enumerate(probs):
        op = O.default_params(dist_tol=1e-10, multistarts=3, seed=50 + i, max_iter=400)
        g_ref, ref = O.instantiate(n, pr, target_pairs=pr, target_gates=tg, params=op, kinds=k, fixed=f)
        got = infos[i]
        assert (got["reason_name"], got["sweeps"], got["restarts"], got["m_final"]) == \
            (ref["reason_name"], ref["sweeps"], ref["restarts"], ref["m_final"]), (i, got, ref)
        if ref["c_train"] > 1e-20:
            # a unique best start: same start, cost and gates
            assert got["best_start"] == ref["best_start"], (i, got, ref)
            assert abs(got["c_train"] - ref["c_train"]) <= 1e-9 * max(ref["c_train"], 1e-12) + 1e-20
            assert np.max(np.abs(host(gates[i]) - g_ref)) < 1e-8
        else:
            # several starts solved the problem exactly in the same sweep and rounding
            # noise orders them: the returned start must be one of them, its gates a
            # solution
            G = host(gates[i])
            basis = np.eye(1 << n)
            d = O.state_distance(n, O.apply_circuit(n, basis, pr, G), O.apply_circuit(n, basis, pr, tg))
            assert got["c_train"] < 1e-20 and d < 1e-20, (i, got["c_train"], d)


def test_batched_kinds_mixed_successes_are_solutions():
    """complex64 states, automatic sweeps per launch, 40 problems: every reported success
    is a real solution (full distance by the oracle's simulation <= 1e-8 at dist_tol 1e-9),
    constant gates returned unchanged."""
    say("kinds batched MIXED successes")
    probs = _kind_problems(40, 91)
    bp = Q.qfs_default_params(dist_tol=1e-9, multistarts=8, seed=60, max_iter=3000)
    dprobs = [dict(n=n, pairs=pr, kinds=k, fixed_gates=dev(f), target_pairs=pr, target_gates=dev(tg))
              for n, pr, k, f, tg in probs]
    gates, infos = Q.qfs_instantiate_batch(dprobs, bp)
    ok = 0
    for i, (n, pr, k, f, tg) in enumerate(probs):
        G = host(gates[i])
        fx = k == I.GATE_FIXED
        assert np.array_equal(G[fx], f[fx])
        if infos[i]["reason_name"] != "SUCCESS":
            continue
        ok += 1
        basis = np.eye(1 << n)
        d = O.state_distance(n, O.apply_circuit(n, basis, pr, G), O.apply_circuit(n, basis, pr, tg))
        assert d <= 1e-8, (i, d)
    say(f"  {ok}/40 succeeded")
    assert ok >= 20
