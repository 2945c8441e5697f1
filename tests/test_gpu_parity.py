"""GPU parity: the HIP path, called through the C ABI, against the FP64 CPU oracle on
identical seeded inputs (MI355X only).

Tolerances: complex128 (FP64) paths agree with the oracle to rounding, 1e-12 relative
on single steps and 1e-10 over 20 lock-step sweeps. The complex64 (MIXED) sweep is
compared teacher-forced (both sides start each sweep from the same FP64 gates): its
cost must agree to 1e-6 * max(c, c_initial), the bound a complex64 state propagation
allows (see the design notes).
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


def relerr(a, b):
    return np.max(np.abs(a - b)) / max(1e-300, np.max(np.abs(b)))


# ------------------------------------------------------------------ single steps
@pytest.mark.parametrize("n,M", [(2, 1), (3, 5), (6, 8), (9, 3)])
def test_draw_states_match_oracle(n, M):
    say(f"draw_states n={n} M={M}")
    got = host(Q.qfs_draw_states(n, M, seed=1234, role=1, stream=0, device=DEV))
    ref = O.draw_states(n, M, seed=1234)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_haar_gates_match_oracle():
    say("haar_gates")
    got = host(Q.qfs_haar_gates(99, 3, 7, device=DEV))
    for s in range(3):
        for k in range(7):
            assert np.max(np.abs(got[s, k] - O.haar_gate(99, s, k))) < 1e-13


@pytest.mark.parametrize("n,M", [(2, 2), (3, 5), (5, 7), (8, 4)])
def test_apply_gates_match_oracle(n, M):
    say(f"apply_gates n={n} M={M}")
    g = np.random.default_rng(n * 7 + M)
    pairs = [(a, b) for a in range(n) for b in range(n) if a != b]
    gates = I.haar_gates(len(pairs), g)
    st = I.orthonormal_samples(n, M, g) if M <= (1 << n) else None
    for dag in (False, True):
        got = host(Q.qfs_apply_gates(n, dev(st), pairs, dev(gates), dagger=dag))
        ref = st.copy()
        seq = range(len(pairs) - 1, -1, -1) if dag else range(len(pairs))
        for k in seq:
            ref = O.apply_gate(n, ref, pairs[k][0], pairs[k][1], gates[k], dagger=dag)
        assert relerr(got, ref) < 1e-13


def test_dense_apply_matches_oracle():
    say("dense_apply n=6 M=9")
    g = np.random.default_rng(3)
    U = I.haar_unitary(64, g)
    psi = I.orthonormal_samples(6, 9, g)
    got = host(Q.qfs_dense_apply(6, dev(U), dev(psi)))
    assert relerr(got, O.dense_apply(6, U, psi)) < 1e-13


@pytest.mark.parametrize("n,M", [(2, 3), (5, 3), (7, 6), (10, 2)])
def test_environment_matches_oracle_all_pairs(n, M):
    say(f"environment n={n} M={M}")
    g = np.random.default_rng(10 * n + M)
    a = g.standard_normal((M, 1 << n)) + 1j * g.standard_normal((M, 1 << n))
    b = g.standard_normal((M, 1 << n)) + 1j * g.standard_normal((M, 1 << n))
    da, db = dev(a), dev(b)
    for qa in range(n):
        for qb in range(n):
            if qa == qb:
                continue
            got = host(Q.qfs_environment(n, da, db, qa, qb))
            assert relerr(got, O.environment(n, a, b, qa, qb)) < 1e-12


def test_polar_update_matches_oracle():
    say("polar_update")
    g = np.random.default_rng(5)
    G = [g.standard_normal((4, 4)) + 1j * g.standard_normal((4, 4)) for _ in range(64)]
    G += [np.zeros((4, 4), complex), np.eye(4, dtype=complex), np.diag([3, 3, 1, 0]).astype(complex),
          np.outer(g.standard_normal(4), g.standard_normal(4)).astype(complex)]
    G = np.stack(G)
    got = host(Q.qfs_polar_update(dev(G)))
    for i in range(len(G)):
        u = got[i]
        assert np.max(np.abs(u.conj().T @ u - np.eye(4))) < 1e-13
        s = np.linalg.svd(G[i], compute_uv=False)
        f = np.real(np.sum(G[i].conj() * u))
        assert abs(f - s.sum()) < 1e-12 * max(1.0, s.sum())
        if i < 64:  # full rank: the polar factor is unique
            assert np.max(np.abs(u - O.update_gate(G[i]))) < 1e-12
    # beta = 1 keeps the gate (App. A)
    u0 = np.stack([I.haar_unitary(4, g) for _ in range(4)])
    got = host(Q.qfs_polar_update(dev(G[:4]), beta=1.0, u=dev(u0)))
    assert np.max(np.abs(got - u0)) < 1e-13


def test_state_distance_matches_oracle():
    say("state_distance")
    g = np.random.default_rng(6)
    x = g.standard_normal((5, 128)) + 1j * g.standard_normal((5, 128))
    y = g.standard_normal((5, 128)) + 1j * g.standard_normal((5, 128))
    assert abs(Q.qfs_state_distance(7, dev(x), dev(y)) - O.state_distance(7, x, y)) < 1e-12


# ------------------------------------------------------------------ sweeps
def _lowbit_template(n, L, g):
    """Random pairs, two thirds of them inside the last three qubits (the lowest
    amplitude bits), so consecutive backward steps mix low and high bit positions."""
    pairs = []
    for k in range(L):
        if k % 3 != 2:
            a, b = g.choice(np.arange(n - 3, n), 2, replace=False)
        else:
            a, b = g.choice(n, 2, replace=False)
        pairs.append((int(a), int(b)))
    return np.asarray(pairs, dtype=np.int32)


def _sweep_problem(n, L, M, starts, seed, brick=False, lowbit=False):
    g = np.random.default_rng(seed)
    if lowbit:
        pairs = _lowbit_template(n, L, g)
    else:
        pairs = I.brickwork_template(n, L) if brick else I.random_pair_template(n, L, g)
    tg = I.haar_gates(len(pairs), g)
    psi = I.orthonormal_samples(n, M, g)
    phi = O.apply_circuit(n, psi, pairs, tg)
    gates = np.stack([I.haar_gates(len(pairs), g) for _ in range(starts)])
    return pairs, psi, phi, gates


@pytest.mark.parametrize("n,L,M,starts,lowbit", [(2, 1, 4, 1, False), (3, 6, 3, 2, False),
                                                 (5, 9, 5, 3, False), (8, 12, 16, 2, False),
                                                 (10, 15, 6, 2, True), (9, 12, 3, 3, True)])
def test_fp64_sweeps_lock_step(n, L, M, starts, lowbit):
    """20 sweeps in lock step: per-sweep costs within 1e-10 relative, gates 1e-10. The
    low-bit templates drive the LDS-staged backward step (gates on the lowest amplitude
    bits) interleaved with the plain one, and ragged sample chunks."""
    say(f"fp64 lock-step n={n} L={L} M={M} starts={starts} lowbit={lowbit}")
    pairs, psi, phi, gates = _sweep_problem(n, L, M, starts, seed=n + L, lowbit=lowbit)
    dg = dev(gates)
    dpsi, dphi = dev(psi), dev(phi)
    ref = gates.copy()
    for sweep in range(20):
        c_gpu = Q.qfs_sweep(n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_FP64)
        for s in range(starts):
            ref[s], c_ref = O.sweep(n, pairs, psi, phi, ref[s])
            assert abs(c_gpu[s] - c_ref) <= 1e-10 * max(c_ref, 1e-3), (sweep, s, c_gpu[s], c_ref)
        assert np.max(np.abs(host(dg) - ref)) < 1e-10


@pytest.mark.parametrize("n,L,M", [(6, 10, 8), (8, 21, 32), (11, 12, 24)])
def test_mixed_sweep_teacher_forced(n, L, M):
    """complex64 states, FP64 update/cost: each sweep starts from the GPU's own FP64
    gates on both sides; |c_gpu - c_oracle| <= 1e-6 * max(c, c_initial). The 11-qubit
    case uses a low-bit template (LDS-staged backward steps)."""
    say(f"mixed teacher-forced n={n} L={L} M={M}")
    pairs, psi, phi, gates = _sweep_problem(n, L // 2 * 2 if n == 8 else L, M, 2, seed=77,
                                            brick=(n == 8), lowbit=(n == 11))
    if n == 8:
        pairs = I.brickwork_template(8, 6)
        g = np.random.default_rng(78)
        tg = I.haar_gates(len(pairs), g)
        phi = O.apply_circuit(n, psi, pairs, tg)
        gates = np.stack([I.haar_gates(len(pairs), g) for _ in range(2)])
    dpsi, dphi = dev(psi), dev(phi)
    c_init = max(O.sweep(n, pairs, psi, phi, gates[0])[1], 1e-3)
    dg = dev(gates)
    for sweep in range(8):
        start_gates = host(dg).copy()
        c_gpu = Q.qfs_sweep(n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_MIXED)
        new = host(dg)
        for s in range(2):
            u_ref, c_ref = O.sweep(n, pairs, psi, phi, start_gates[s])
            assert abs(c_gpu[s] - c_ref) <= 1e-6 * max(c_ref, c_init), (sweep, s, c_gpu[s], c_ref)
            for u in new[s]:
                assert np.max(np.abs(u.conj().T @ u - np.eye(4))) < 1e-12


# ------------------------------------------------------------------ full instantiation
def test_instantiate_fp64_matches_oracle_control_flow():
    """Same seed, same readings: the GPU control loop follows the oracle's trajectory
    (doubling from M = 2, multistarts) and ends with the same start, reason, sweeps and
    cost."""
    say("instantiate fp64 vs oracle (3 qubits, 4 gates)")
    pairs = [(0, 1), (1, 2), (0, 1), (1, 2)]
    tg = I.haar_gates(4, np.random.default_rng(5))
    p = O.default_params(dist_tol=1e-11, multistarts=4, seed=3, max_iter=400, diff_tol_r=1e-7)
    g_ref, info_ref = O.instantiate(3, pairs, target_pairs=pairs, target_gates=tg, params=p)
    qp = dict(p)
    qp["precision"] = Q.QFS_PREC_FP64
    g_gpu, info = Q.qfs_instantiate(3, pairs, target_pairs=pairs, target_gates=dev(tg), params=qp)
    assert info["reason_name"] == info_ref["reason_name"] == "SUCCESS"
    assert info["best_start"] == info_ref["best_start"]
    assert info["sweeps"] == info_ref["sweeps"]
    assert info["m_final"] == info_ref["m_final"] and info["restarts"] == info_ref["restarts"]
    assert abs(info["c_train"] - info_ref["c_train"]) < 1e-9 * max(info_ref["c_train"], 1e-12) + 1e-20
    assert np.max(np.abs(host(g_gpu) - g_ref)) < 1e-8


def test_instantiate_samples_minimal_entry():
    say("instantiate_samples (minimal entry)")
    pairs = [(0, 1), (1, 2), (0, 2)]
    g = np.random.default_rng(8)
    tg = I.haar_gates(3, g)
    psi = I.orthonormal_samples(3, 8, g)
    phi = O.apply_circuit(3, psi, pairs, tg)
    gates, cost = Q.qfs_instantiate_samples(3, pairs, dev(psi), dev(phi), 8, 1e-12)
    assert cost < 1e-12
    C_psi = O.apply_circuit(3, psi, pairs, host(gates))
    assert O.state_distance(3, C_psi, phi) < 1e-11


def test_instantiate_mixed_reaches_distance_after_refinement():
    """MIXED precision: complex64 sweeps, then complex128 refinement below 1e-5; the
    returned gates reach d_full <= 1e-8, checked by the oracle's own dense product."""
    say("instantiate mixed 6 qubits")
    n = 6
    pairs = I.brickwork_template(n, 4)
    tg = I.haar_gates(len(pairs), np.random.default_rng(11))
    qp = Q.qfs_default_params(dist_tol=1e-9, multistarts=8, seed=4, max_iter=3000, m_init=4,
                              diff_tol_r=1e-7)
    g_gpu, info = Q.qfs_instantiate(n, pairs, target_pairs=pairs, target_gates=dev(tg), params=qp)
    assert info["reason_name"] == "SUCCESS", info
    assert info["refined"] == 1
    gates = host(g_gpu)
    psi = O.draw_states(n, 1 << n, seed=555)
    d_full = O.state_distance(n, O.apply_circuit(n, psi, pairs, gates), O.apply_circuit(n, psi, pairs, tg))
    assert d_full <= 1e-8


def test_memory_split_matches_unsplit_run():
    """App. A out-of-memory recovery: a device-memory budget too small for all starts
    runs them as halves; with a fixed training set (no doubling) the starts are
    independent, so the result equals the unsplit run."""
    say("memory split")
    pairs = I.brickwork_template(5, 4)
    tg = I.haar_gates(len(pairs), np.random.default_rng(12))
    base = Q.qfs_default_params(dist_tol=1e-30, multistarts=8, seed=9, max_iter=12, m_init=8,
                                fixed_m=1, precision=Q.QFS_PREC_FP64, diff_tol_r=0.0,
                                plateau_window=100)
    g1, i1 = Q.qfs_instantiate(5, pairs, target_pairs=pairs, target_gates=dev(tg), params=base)
    # the largest budget (in steps of 0.8 from 4 MB) under which the starts no longer fit
    # together: the run splits them and must still succeed
    g2 = i2 = None
    budget = 4_000_000.0
    while budget > 20_000 and g2 is None:
        try:
            g, i = Q.qfs_instantiate(5, pairs, target_pairs=pairs, target_gates=dev(tg),
                                     params=dict(base, device_mem_budget=int(budget)))
            if i["start_groups"] > 1:
                g2, i2 = g, i
        except Q.QfsError as e:
            assert e.code == Q.QFS_ENOMEM
            break
        budget *= 0.8
    say(f"memory split at a budget of {int(budget)} bytes")
    assert g2 is not None, "no budget split the starts"
    assert i1["start_groups"] == 1 and i2["start_groups"] > 1
    assert i2["best_start"] == i1["best_start"] and abs(i2["c_train"] - i1["c_train"]) < 1e-14
    assert np.max(np.abs(host(g1) - host(g2))) < 1e-14


def test_invalid_gates_in_rejected():
    say("gates_in validation")
    pairs = [(0, 1)]
    bad = dev(np.ones((1, 1, 4, 4)))
    with pytest.raises(Q.QfsError) as e:
        Q.qfs_instantiate(2, pairs, U=dev(np.eye(4)), params=Q.qfs_default_params(multistarts=1),
                          gates_in=bad)
    assert e.value.code == Q.QFS_EINVAL


# ------------------------------------------------------------------ full-size workload
def test_full_size_sweep_sampled_starts():
    """The 12-qubit workload at its full size and in the bench's configuration (44
    brickwork gates, M = 256, 16 starts, complex64 states): one sweep of all starts on
    the device; two sampled starts re-run by the oracle from the same gates (teacher
    forced, |dc| <= 1e-6 max(c, c_init)); every updated gate unitary to 1e-12; and the
    cost can only fall (block-coordinate ascent, Sec. 3) for every start."""
    n, M, S = 12, 256, 16
    w = I.workload_12q()
    pairs = w["pairs"]
    g = np.random.default_rng(1212)
    say("full size: drawing 12q states")
    psi = I.orthonormal_samples(n, M, g)
    phi = O.apply_circuit(n, psi, pairs, w["target_gates"])
    gates = np.stack([I.haar_gates(len(pairs), g) for _ in range(S)])
    dpsi, dphi, dg = dev(psi), dev(phi), dev(gates)
    say("full size: GPU sweep (16 starts, MIXED)")
    c_gpu = Q.qfs_sweep(n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_MIXED)
    new = host(dg)
    for s in range(S):
        for u in new[s]:
            assert np.max(np.abs(u.conj().T @ u - np.eye(4))) < 1e-12
    for s in (0, 11):
        say(f"full size: oracle sweep of start {s}")
        c0 = O.state_distance(n, O.apply_circuit(n, psi, pairs, gates[s]), phi)
        _, c_ref = O.sweep(n, pairs, psi, phi, gates[s])
        assert abs(c_gpu[s] - c_ref) <= 1e-6 * max(c_ref, c0), (s, c_gpu[s], c_ref)
        assert c_gpu[s] <= c0 + 1e-6 * c0
    say("full size: second sweep must not increase any start's cost")
    c2 = Q.qfs_sweep(n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_MIXED)
    assert np.all(c2 <= c_gpu + 1e-6 * np.maximum(c_gpu, 1e-3))


def test_full_size_teacher_forced_all_starts():
    """The parity contract at the bench's full size (12-qubit brickwork, 44 gates,
    M = 256, 16 starts, complex64 states with FP64 environment sums, polar update and
    cost): the bench's inputs (training states and initial gates drawn from its seed,
    U psi of its target) and five sweeps of all 16 starts on the device, each one
    teacher-forced: the oracle re-runs every start's sweep in FP64 from the device's
    FP64 gates before that sweep, and |dc| <= 1e-6 max(c, c_init) for every start and
    sweep. (qfs_sweep runs the sweep kernels of the bench's qfs_instantiate call.)"""
    from concurrent.futures import ThreadPoolExecutor
    import os
    n, M, S, seed = 12, 256, 16, 0x5A17 + 3
    w = I.workload_12q()
    pairs = w["pairs"]
    say("full size teacher-forced: drawing the bench's states and initial gates (oracle)")
    psi = O.draw_states(n, M, seed=seed)
    phi = O.apply_circuit(n, psi, pairs, w["target_gates"])
    gates = np.stack([np.stack([O.haar_gate(seed, s, k) for k in range(len(pairs))]) for s in range(S)])
    dpsi, dphi, dg = dev(psi), dev(phi), dev(gates)
    workers = max(1, min(16, os.cpu_count() or 1))
    pool = ThreadPoolExecutor(max_workers=workers)
    c_init = np.array(list(pool.map(
        lambda s: O.state_distance(n, O.apply_circuit(n, psi, pairs, gates[s]), phi), range(S))))
    for t in range(5):
        before = host(dg)
        say(f"full size teacher-forced: device sweep {t + 1} (16 starts)")
        c_dev = Q.qfs_sweep(n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_MIXED)
        say(f"full size teacher-forced: oracle sweep {t + 1} of 16 starts on {workers} threads")
        c_ref = np.array(list(pool.map(lambda s: O.sweep(n, pairs, psi, phi, before[s])[1], range(S))))
        bound = 1e-6 * np.maximum(c_ref, c_init)
        ratio = np.abs(c_dev - c_ref) / bound
        say(f"  sweep {t + 1}: c in [{c_ref.min():.6f}, {c_ref.max():.6f}], max |dc| "
            f"{np.max(np.abs(c_dev - c_ref)):.2e}, max |dc| / bound {ratio.max():.3f}")
        assert np.all(ratio <= 1.0), (t, ratio)
    pool.shutdown()


@pytest.mark.parametrize("precision", [Q.QFS_PREC_FP64, Q.QFS_PREC_MIXED])
def test_full_size_instantiate_in_bench_configuration(precision):
    """The timed call of the benchmark, shortened to two sweeps: 12-qubit brickwork (44
    gates), M = 256 fixed, 16 starts, the two streams of the backward pass, sample sets and
    initial gates drawn on the device; the oracle runs the same call in FP64 from its own
    draws (same seed). FP64 states: parity, the same best start, c_train and c_val to
    1e-10 relative. complex64 states (the bench's precision): not the parity contract
    (that is checked teacher-forced above) but a bound on how far two free-running
    sweeps drift apart: 1e-4 relative. Far from the solution (c near 2, so f = M (1 - c/2)
    is about 5 while the environment sums terms of total size about M = 256) the FP32
    rounding of the partial sums is amplified about 50-fold, and the two sweeps compound
    it. The best start must agree when the runner-up is not within that tolerance."""
    say(f"full size: qfs_instantiate in the bench configuration (2 sweeps), precision={precision}")
    w = I.workload_12q()
    kw = dict(multistarts=16, m_init=256, fixed_m=1, seed=0x5A17 + 3, max_iter=2, diff_tol_r=0.0,
              plateau_window=1 << 30)
    _, got = Q.qfs_instantiate(12, w["pairs"], target_pairs=w["pairs"], target_gates=dev(w["target_gates"]),
                               params=Q.qfs_default_params(precision=precision, **kw))
    say("full size: oracle of the same call")
    _, ref = O.instantiate(12, w["pairs"], target_pairs=w["pairs"], target_gates=w["target_gates"],
                           params=O.default_params(**kw), trace_capacity=64)
    assert got["reason_name"] == ref["reason_name"] == "MAX_ITER" and got["sweeps"] == 2
    assert got["m_final"] == 256 and got["start_sweeps"] == 32
    tol = 1e-10 if precision == Q.QFS_PREC_FP64 else 1e-4
    tr = ref["trace"]
    last = np.sort(tr["c_train"][tr["sweep"] == 2])
    assert abs(got["c_train"] - ref["c_train"]) <= tol * ref["c_train"], (got["c_train"], ref["c_train"])
    if last[1] - last[0] > 2 * tol * last[0]:
        assert got["best_start"] == ref["best_start"]
        assert abs(got["c_val"] - ref["c_val"]) <= tol * ref["c_val"], (got["c_val"], ref["c_val"])


@pytest.mark.parametrize("precision", [Q.QFS_PREC_FP64, Q.QFS_PREC_MIXED])
def test_backward_split_deterministic_when_starts_stop_unevenly(precision):
    """The backward pass runs the two halves of the running starts on two streams. Once
    starts stop at different sweeps the halves differ in size (and in blocks per start),
    which must not let their environment partials meet: repeated calls of a 12-qubit U3 +
    CNOT instantiation (16 starts, M = 32, starts stopping one by one) agree bit for bit."""
    say(f"split backward determinism, precision={precision}")
    w = I.workload_u3_cnot(12, 4, seed_base=0x5A17 + 9)
    tg, fx = dev(w["target_gates"]), dev(w["fixed"])
    outs = []
    for _ in range(3):
        p = Q.qfs_default_params(seed=23, m_init=32, precision=precision)
        g, r = Q.qfs_instantiate(12, w["pairs"], target_pairs=w["pairs"], target_gates=tg, params=p,
                                 kinds=w["kinds"], fixed_gates=fx)
        outs.append((host(g), r["reason_name"], r["sweeps"], r["best_start"], r["c_train"], r["start_sweeps"]))
    for o in outs[1:]:
        assert o[1:] == outs[0][1:], (o[1:], outs[0][1:])
        assert np.array_equal(o[0], outs[0][0])
    # starts did stop unevenly: fewer start-sweeps than 16 x the returned start's sweeps
    assert outs[0][5] < 16 * outs[0][2]


# ------------------------------------------------------------------ graph replay
@pytest.mark.parametrize("precision", [Q.QFS_PREC_FP64, Q.QFS_PREC_MIXED])
def test_graph_replay_matches_eager(precision):
    """Each sweep replayed from a captured HIP graph (params.graphs = 1) gives bit-identical
    results to launching every kernel: many replays with host decisions and copies in
    between, re-captures after starts stop, after doublings and after the switch to
    complex128 refinement."""
    say(f"graph replay vs eager, precision={precision}")
    n = 6
    g = np.random.default_rng(61)
    pairs = I.random_pair_template(n, 8, g)
    tg = dev(I.haar_gates(len(pairs), g))
    base = dict(multistarts=6, seed=9, max_iter=400, dist_tol=1e-10, precision=precision)
    g_on, r_on = Q.qfs_instantiate(n, pairs, target_pairs=pairs, target_gates=tg,
                                   params=Q.qfs_default_params(graphs=1, **base))
    g_off, r_off = Q.qfs_instantiate(n, pairs, target_pairs=pairs, target_gates=tg,
                                     params=Q.qfs_default_params(graphs=0, **base))
    for key in ("reason", "sweeps", "restarts", "best_start", "m_final", "start_sweeps", "refined"):
        assert r_on[key] == r_off[key], (key, r_on[key], r_off[key])
    assert r_on["c_train"] == r_off["c_train"] and r_on["c_val"] == r_off["c_val"]
    assert np.array_equal(host(g_on), host(g_off))
    say(f"  {r_on['reason_name']} after {r_on['sweeps']} sweeps, {r_on['restarts']} doublings")
