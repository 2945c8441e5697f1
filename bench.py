#!/usr/bin/env python3
"""Benchmark of the QFactor-Sample hot path on one MI355X.

Workload (default): 12-qubit brickwork of depth 8 (44 general two-qubit gates), target
= the same template with Haar-random gates, M = 256 fixed training states (doubling
off), 16 lock-step random starts, complex64 states with FP64 environment sums, polar
updates and costs (MIXED precision), validation cost every sweep.

One step = one sweep of every start through the whole per-sweep path: forward B
list and validation forward pass, right-to-left environment + FP64 polar update +
backward propagation, Eq. 9 cost, and the control decision on the host. The timed
region is one qfs_instantiate call with max_iter = steps (it also draws the sample
states and forms U psi on the device, once). value = start-sweeps per second.

Prints one JSON line. The dominant kernel's roofline comes from a second call of the
same workload in which the library records hipEvents around every launch on the
call's stream (kept out of the headline timing).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "instantiation sweeps/s + time-to-dist 1e-8 (12q, HBM GB/s); batched vs plain"
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_bwd_group_12q_M256_S16_pmc.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2405_12866_amd", "csrc", "group.hip")


def measured_traffic():
    """HBM bytes per k_bwd_group launch from the committed PMC summary, when it was taken
    on the current kernel source (sha256 of group.hip recorded there); else None."""
    import hashlib
    try:
        with open(PMC_SUMMARY) as f:
            text = f.read()
        with open(KERNEL_SOURCE, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != sha:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None
HBM_PEAK_GBPS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--m", type=int, default=256)
    ap.add_argument("--starts", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ttd", action="store_true", help="skip the time-to-distance runs")
    ap.add_argument("--timing", type=int, default=1)
    ap.add_argument("--repeats", type=int, default=10,
                    help="further calls of the headline workload for the median and IQR")
    ap.add_argument("--graphs", type=int, default=0, help="replay sweeps from HIP graphs (params.graphs)")
    ap.add_argument("--bwd-split", type=int, default=1,
                    help="0: run the backward pass of all starts on one stream in every call (the "
                         "instrumented call always does), so every step launch covers all starts, "
                         "as needed to compare a profiler's per-launch averages with the roofline")
    ap.add_argument("--batched", type=int, default=4096,
                    help="problems in the batched workload (0 skips it)")
    ap.add_argument("--batched-u3cx", type=int, default=4096,
                    help="U3 + CNOT problems in a second batched workload (0 skips it)")
    ap.add_argument("--plain-sample", type=int, default=128,
                    help="problems of the batched workload also run one by one")
    ap.add_argument("--learned", type=int, default=1024,
                    help="held-out problems for the learned-M comparison (0 skips it)")
    ap.add_argument("--u3cx", type=int, default=1,
                    help="1: also time the 12-qubit U3 + CNOT template (one-qubit variable gates "
                         "around constant CNOTs); 0 skips it")
    ap.add_argument("--qf", type=str, default="6,8,10,12",
                    help="qubit counts of U3 + CNOT problems run with full-unitary QFactor and "
                         "with QFactor-Sample (time to solution); empty skips it")
    ap.add_argument("--qudits", type=int, default=1,
                    help="1: time qutrit sweeps and QFactor vs QFactor-Sample on qutrits; 0 skips it")
    ap.add_argument("--shares", type=str, default="2,4,8",
                    help="GPU counts G: time the 12-qubit workload at M / G samples, one GPU's "
                         "share of a sample-sharded run (empty skips it)")
    ap.add_argument("--sec8d", type=int, default=1,
                    help="measurement rows C1, C2, C3 (every M, 1 and 16 starts) and errors against the oracle")
    ap.add_argument("--learned-large", type=int, default=0,
                    help="10-14 qubit random-pair problems (30-120 gates) for the learned-M "
                         "comparison through qfs_instantiate (0 skips it)")
    return ap.parse_args()


def host_cpu():
    """nproc, the cores this process may use, and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "usable": usable, "model": model}


def cpu_baseline(w, M, starts, min_seconds=8.0, max_rounds=30):
    """The FP64 oracle on the host cores, twice: on one thread (one start) and on every
    core the process may use (one start per thread, as many starts as threads; the
    thread count is capped by OMP_NUM_THREADS, the host share given to one GPU). Each
    measurement runs rounds of one sweep plus the validation forward pass of each start,
    each start continuing from its updated gates, until at least `min_seconds` (a bounded
    sample of the workload). The all-core figure is the reported value."""
    cpu = host_cpu()
    allc = max(1, min(cpu["usable"], int(os.environ.get("OMP_NUM_THREADS", str(cpu["usable"])))))
    one = _oracle_rounds(w, M, 1, min_seconds, max_rounds)
    many = _oracle_rounds(w, M, allc, min_seconds, max_rounds)
    out = dict(many)
    out["one_thread"] = {"value": one["value"], "sample": one["sample"]}
    out["all_cores"] = {"value": many["value"], "threads": allc, "sample": many["sample"]}
    out["host"] = cpu
    return out


def _oracle_rounds(w, M, cores, min_seconds, max_rounds):
    import concurrent.futures as cf

    import numpy as np

    import oracle as O
    from paper_2405_12866_amd import inputs as I

    g = np.random.default_rng(1)
    n, pairs = w["n"], w["pairs"]
    psi = I.orthonormal_samples(n, M, g)
    phi = O.apply_circuit(n, psi, pairs, w["target_gates"])
    psiv = I.orthonormal_samples(n, M, g)
    phiv = O.apply_circuit(n, psiv, pairs, w["target_gates"])
    gates = [I.haar_gates(len(pairs), g) for _ in range(cores)]

    def one(s):
        gates[s], c = O.sweep(n, pairs, psi, phi, gates[s])
        cv = O.state_distance(n, O.apply_circuit(n, psiv, pairs, gates[s]), phiv)
        return c, cv

    rounds = 0
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        while rounds < max_rounds and (rounds == 0 or time.perf_counter() - t0 < min_seconds):
            list(ex.map(one, range(cores)))
            rounds += 1
    dt = time.perf_counter() - t0
    return {"value": rounds * cores / dt, "unit": "start-sweeps/s", "cores": cores, "kind": "oracle",
            "sample": f"{rounds} rounds of 1 sweep + validation forward pass of each of {cores} "
                      f"starts (one thread each), 12 qubits, {len(pairs)} gates, M={M}, complex128; "
                      f"{dt:.1f} s"}


def u3_cnot(dev, M, S, steps, warmup, timing):
    """The 12-qubit U3 + CNOT template (8 brickwork sublayers: 44 constant CNOTs and 100
    variable one-qubit gates, 144 gates), Haar one-qubit target gates, M fixed, S lock-step
    starts, MIXED precision: start-sweeps/s and the per-kernel classes; plus the
    time-to-distance 1e-8 of the 8-qubit U3 + CNOT template (4 sublayers) with App. A
    defaults (M from 2, doubling, 16 starts)."""
    import torch

    from paper_2405_12866_amd import inputs as I
    from paper_2405_12866_amd import qfs as Q

    w = I.workload_u3_cnot(12, 8)
    n, pairs, kinds = 12, w["pairs"], w["kinds"]
    tg = torch.as_tensor(w["target_gates"]).to(dev)
    fx = torch.as_tensor(w["fixed"]).to(dev)
    base = Q.qfs_default_params(multistarts=S, m_init=M, fixed_m=1, seed=0x5A17 + 8,
                                precision=Q.QFS_PREC_MIXED, diff_tol_r=0.0, plateau_window=1 << 30)
    kw = dict(target_pairs=pairs, target_gates=tg, kinds=kinds, fixed_gates=fx)
    Q.qfs_instantiate(n, pairs, params=dict(base, max_iter=max(1, warmup)), **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = Q.qfs_instantiate(n, pairs, params=dict(base, max_iter=steps), **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    L, nvar = len(pairs), int((kinds != I.GATE_FIXED).sum())
    S_amp = M * (1 << n)
    # algorithmic bytes per start-sweep: the B list entries before variable gates written
    # and read once, plus phi, complex64
    alg = 16.0 * S_amp * nvar + 8.0 * S_amp
    out = {"workload": f"12q U3+CNOT, 8 sublayers ({L} gates: {nvar} variable one-qubit, "
                       f"{L - nvar} constant CNOT), M={M} fixed, {S} lock-step starts, MIXED",
           "start_sweeps_per_s": round(info["start_sweeps"] / dt, 2),
           "ms_per_step": round(1e3 * dt / steps, 4),
           "sweep_algorithmic_GBps": round(alg * info["start_sweeps"] / dt / 1e9, 1)}
    if timing:
        _, ti = Q.qfs_instantiate(n, pairs, params=dict(base, max_iter=steps, timing=1), **kw)
        kl, ks, kb = ti["kernel_launches"], ti["kernel_seconds"], ti["kernel_bytes"]
        out["kernel_classes"] = {
            name: {"launches": kl[i], "seconds": round(ks[i], 5),
                   "GBps": round(kb[i] / ks[i] / 1e9, 1) if ks[i] > 0 and kb[i] > 0 else None,
                   "avg_us": round(1e6 * ks[i] / kl[i], 2) if kl[i] else None}
            for i, name in enumerate(["bwd_step", "forward", "distance", "env_finalize_polar"])}
    w8 = I.workload_u3_cnot(8, 4)
    p = Q.qfs_default_params(multistarts=16, seed=9, max_iter=3000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, r = Q.qfs_instantiate(8, w8["pairs"], target_pairs=w8["pairs"],
                             target_gates=torch.as_tensor(w8["target_gates"]).to(dev), params=p,
                             kinds=w8["kinds"], fixed_gates=torch.as_tensor(w8["fixed"]).to(dev))
    torch.cuda.synchronize()
    out["time_to_distance_8q"] = {"seconds": round(time.perf_counter() - t0, 4), "reason": r["reason_name"],
                                  "m_final": r["m_final"], "sweeps": r["sweeps"], "c_train": r["c_train"],
                                  "start_sweeps": r["start_sweeps"]}
    return out


def qf_vs_qfs(dev, sizes):
    """Time to solution of full-unitary QFactor (params full_unitary: the complete basis,
    M = 2^n) against QFactor-Sample (M from 2, doubling on the validation cost) on the same
    MI355X and kernels: U3 + CNOT templates with 4 sublayers, Haar one-qubit target gates,
    App. A defaults (16 starts, dist_tol 1e-8), MIXED precision, same seed; the sample
    method both from M = 2 (App. A) and from M = 32. For the sample method the full
    distance of the returned gates is measured on the device."""
    import numpy as np
    import torch

    from paper_2405_12866_amd import inputs as I
    from paper_2405_12866_amd import qfs as Q

    rows = []
    for n in sizes:
        w = I.workload_u3_cnot(n, 4, seed_base=0x5A17 + 9)
        tg = torch.as_tensor(w["target_gates"]).to(dev)
        fx = torch.as_tensor(w["fixed"]).to(dev)
        kw = dict(target_pairs=w["pairs"], target_gates=tg, kinds=w["kinds"], fixed_gates=fx)
        row = {"n": n, "gates": len(w["pairs"])}
        for name, full, m0 in (("qfs", 0, 2), ("qfs_m32", 0, 32), ("qf", 1, 2)):
            p = Q.qfs_default_params(seed=11 + n, full_unitary=full, m_init=min(m0, 1 << n),
                                     time_budget_s=120.0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g, r = Q.qfs_instantiate(n, w["pairs"], params=p, **kw)
            torch.cuda.synchronize()
            row[name] = {"seconds": round(time.perf_counter() - t0, 4), "reason": r["reason_name"],
                         "sweeps": r["sweeps"], "m_final": r["m_final"], "c_train": r["c_train"],
                         "start_sweeps": r["start_sweeps"]}
            if not full:
                N = 1 << n
                basis = torch.eye(N, dtype=torch.complex128, device=dev)
                got = Q.qfs_apply_gates(n, basis.clone(), w["pairs"], g)
                want = Q.qfs_apply_gates(n, basis.clone(), w["pairs"], tg)
                row[name]["d_full"] = Q.qfs_state_distance(n, got, want)
        row["speedup"] = round(row["qf"]["seconds"] / row["qfs"]["seconds"], 2)
        row["speedup_m32"] = round(row["qf"]["seconds"] / row["qfs_m32"]["seconds"], 2)
        rows.append(row)
    out = {"problems": rows}
    for key, name in (("speedup", "qfs"), ("speedup_m32", "qfs_m32")):
        ok = [r[key] for r in rows if r["qf"]["reason"] == r[name]["reason"] == "SUCCESS"]
        out[f"mean_{key}_both_succeeded"] = round(float(np.mean(ok)), 2) if ok else None
    return out


def qudits_leg(dev, steps):
    """Qutrits (d = 3, Sec. 5). (a) Sweeps: 7 qutrits (2187 amplitudes), brickwork of 4
    sublayers (12 two-qutrit gates, 9 x 9), Haar target gates, M = 64 fixed samples, 16
    lock-step starts, MIXED: start-sweeps/s and algorithmic GB/s (each call also converts
    the sets to the internal layout). (b) Time to solution of full-unitary QFactor (the
    complete basis as the sample set, M = 3^n, no validation set) against the sample method
    (M from 9, doubling up to 144 against 9 validation samples) on 6 and 7 qutrits
    (brickwork, 4 sublayers), 16 starts, App. A rules, MIXED, same seed. (c) Sweeps of 5
    ququarts (d = 4, 16 x 16 gates), as (a). (d) Gate kinds: time to 1e-8 of a 6-qutrit
    template of one-qutrit gates around constant CSUM gates, states drawn on the device.
    (e) 64 qutrit problems through the batched entry against one at a time."""
    import numpy as np
    import torch

    from paper_2405_12866_amd import inputs as I
    from paper_2405_12866_amd import qfs as Q

    out = {}
    g = I.rng(I.derive_seed(0x5A17 + 11))
    n, M, S = 7, 64, 16
    pairs = I.qudit_brickwork(n, 4)
    L = len(pairs)
    tg = np.stack([I.haar_unitary(9, g) for _ in range(L)])
    N = 3 ** n
    psi = I.orthonormal_states(N, M, g)
    phi = I.qudit_circuit_apply(3, n, psi, pairs, tg)
    dpsi, dphi = torch.as_tensor(psi).to(dev), torch.as_tensor(phi).to(dev)
    base = Q.qfs_default_params(multistarts=S, m_init=M, fixed_m=1, seed=0x5A17 + 11, diff_tol_r=0.0,
                                plateau_window=1 << 30)
    Q.qfs_qudit_instantiate(3, n, pairs, dpsi, dphi, params=dict(base, max_iter=2))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, r = Q.qfs_qudit_instantiate(3, n, pairs, dpsi, dphi, params=dict(base, max_iter=steps))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    S_amp = M * N
    alg = 16.0 * S_amp * L + 8.0 * S_amp
    out["sweeps_7qutrits"] = {"workload": f"7 qutrits, {L} two-qutrit gates, M={M} fixed, {S} lock-step starts, "
                                          f"MIXED, one qfs_qudit_instantiate call of {steps} sweeps",
                              "start_sweeps_per_s": round(r["start_sweeps"] / dt, 1),
                              "ms_per_step": round(1e3 * dt / steps, 3),
                              "sweep_algorithmic_GBps": round(alg * r["start_sweeps"] / dt / 1e9, 1)}
    rows = []
    for n in (6, 7):
        N = 3 ** n
        pairs = I.qudit_brickwork(n, 4)
        tg = np.stack([I.haar_unitary(9, g) for _ in pairs])
        basis = np.eye(N, dtype=np.complex128)
        samples = I.orthonormal_states(N, 9 + 144, g)
        row = {"n": n, "gates": len(pairs)}
        for name, ps, m0, nv in (("qf", basis, N, 0), ("qfs", samples, 9, 9)):
            ph = I.qudit_circuit_apply(3, n, ps, pairs, tg)
            p = Q.qfs_default_params(seed=31 + n, m_init=m0, time_budget_s=120.0)
            dps, dph = torch.as_tensor(ps).to(dev), torch.as_tensor(ph).to(dev)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, r = Q.qfs_qudit_instantiate(3, n, pairs, dps, dph, n_val=nv, params=p)
            torch.cuda.synchronize()
            row[name] = {"seconds": round(time.perf_counter() - t1, 4), "reason": r["reason_name"],
                         "m_final": r["m_final"], "sweeps": r["sweeps"], "c_train": r["c_train"],
                         "c_val": r["c_val"]}
        row["speedup"] = round(row["qf"]["seconds"] / row["qfs"]["seconds"], 2)
        rows.append(row)
    out["qf_vs_qfs_qutrits"] = rows
    # (c) d = 4: 5 ququarts (1024 amplitudes), the same brickwork, M = 64, 16 starts
    n, d, M = 5, 4, 64
    pairs = I.qudit_brickwork(n, 4)
    L = len(pairs)
    tg = np.stack([I.haar_unitary(16, g) for _ in range(L)])
    N = d ** n
    psi = I.orthonormal_states(N, M, g)
    phi = I.qudit_circuit_apply(d, n, psi, pairs, tg)
    dpsi, dphi = torch.as_tensor(psi).to(dev), torch.as_tensor(phi).to(dev)
    Q.qfs_qudit_instantiate(d, n, pairs, dpsi, dphi, params=dict(base, max_iter=2))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, r = Q.qfs_qudit_instantiate(d, n, pairs, dpsi, dphi, params=dict(base, max_iter=steps))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    S_amp = M * N
    alg = 16.0 * S_amp * L + 8.0 * S_amp
    out["sweeps_5ququarts"] = {"workload": f"5 ququarts (d = 4), {L} two-ququart gates (16 x 16), M={M} fixed, "
                                           f"{S} lock-step starts, MIXED, one qfs_qudit_instantiate call of {steps} sweeps",
                               "start_sweeps_per_s": round(r["start_sweeps"] / dt, 1),
                               "ms_per_step": round(1e3 * dt / steps, 3),
                               "sweep_algorithmic_GBps": round(alg * r["start_sweeps"] / dt / 1e9, 1)}
    # (d) gate kinds: 6 qutrits, one-qutrit gates around constant CSUM gates (a qutrit
    # counterpart of the U3 + CNOT partitions), time to 1e-8 from drawn states against a
    # target from the same template
    n = 6
    pairs, kinds = [], []
    for layer in range(4):
        for a in range(layer % 2, n - 1, 2):
            pairs += [(a, a + 1), (a + 1, a), (a, a + 1)]
            kinds += [Q.QFS_GATE_1Q, Q.QFS_GATE_1Q, Q.QFS_GATE_FIXED]
    csum = np.zeros((9, 9), dtype=np.complex128)
    for x in range(3):
        for y in range(3):
            csum[3 * x + (y + x) % 3, 3 * x + y] = 1.0
    slots = []
    for k in kinds:
        slots.append(csum if k == Q.QFS_GATE_FIXED else np.kron(I.haar_unitary(3, g), np.eye(3)))
    tg = np.stack(slots)
    fixed = torch.as_tensor(np.stack([csum] * len(kinds))).to(dev)
    p = Q.qfs_default_params(seed=41, m_init=9, time_budget_s=60.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, r = Q.qfs_qudit_instantiate_target(3, n, pairs, target_pairs=pairs, target_gates=torch.as_tensor(tg).to(dev),
                                          params=p, kinds=kinds, fixed_gates=fixed)
    torch.cuda.synchronize()
    out["kinds_6qutrits_csum"] = {"workload": f"6 qutrits, {len(kinds)} gates ({kinds.count(Q.QFS_GATE_1Q)} one-qutrit, "
                                              f"{kinds.count(Q.QFS_GATE_FIXED)} constant CSUM), target from the same "
                                              "template, states drawn on the device, 16 starts, MIXED, App. A rules",
                                  "seconds": round(time.perf_counter() - t0, 4), "reason": r["reason_name"],
                                  "m_final": r["m_final"], "sweeps": r["sweeps"], "c_train": r["c_train"],
                                  "c_val": r["c_val"]}
    # (e) problems side by side: 64 qutrit problems (4-6 qutrits, 4-10 random-pair gates,
    # targets from their templates, states drawn on the device), 16 starts each, MIXED,
    # App. A rules from M = 9: the batched entry against the same problems one at a time
    rng = np.random.default_rng(0x5A17 + 12)
    bprobs = []
    for i in range(64):
        nq = int(rng.integers(4, 7))
        prs = I.random_pair_template(nq, int(rng.integers(4, 11)), rng)
        tgb = torch.as_tensor(np.stack([I.haar_unitary(9, rng) for _ in prs])).to(dev)
        bprobs.append(dict(n=nq, pairs=prs, target_pairs=prs, target_gates=tgb))
    pb = Q.qfs_default_params(seed=43, m_init=9, time_budget_s=30.0)
    Q.qfs_qudit_instantiate_batch(3, bprobs[:4], pb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rb = Q.qfs_qudit_instantiate_batch(3, bprobs, pb)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    ok_one = 0
    for pr in bprobs:
        _, r1 = Q.qfs_qudit_instantiate_target(3, pr["n"], pr["pairs"], target_pairs=pr["target_pairs"],
                                               target_gates=pr["target_gates"], params=pb)
        ok_one += r1["reason_name"] == "SUCCESS"
    torch.cuda.synchronize()
    t_one = time.perf_counter() - t0
    out["batched_qutrits"] = {"workload": "64 qutrit problems (4-6 qutrits, 4-10 random-pair two-qutrit gates, "
                                          "targets from the templates, states drawn on the device), 16 starts, "
                                          "MIXED, App. A rules from M = 9",
                              "batched_s": round(t_batch, 3), "one_at_a_time_s": round(t_one, 3),
                              "successes": sum(r["reason_name"] == "SUCCESS" for r in rb),
                              "successes_one_at_a_time": ok_one, "speedup": round(t_one / t_batch, 2)}
    return out


def shard_shares(dev, M, S, steps, counts):
    """One GPU's share of a run that shards the M training states over G GPUs (each GPU
    holds M / G samples with their B lists; one 256-byte reduction of the partial
    environment per gate would join them): the 12-qubit workload at M / G fixed samples,
    16 lock-step starts, MIXED, timed as the main leg. The exchange itself is not run."""
    import torch

    from paper_2405_12866_amd import inputs as I
    from paper_2405_12866_amd import qfs as Q

    w = I.workload_12q()
    tg = torch.as_tensor(w["target_gates"]).to(dev)
    out = {}
    for G in counts:
        m = max(1, M // G)
        base = Q.qfs_default_params(multistarts=S, m_init=m, fixed_m=1, seed=0x5A17 + 3,
                                    diff_tol_r=0.0, plateau_window=1 << 30)
        Q.qfs_instantiate(12, w["pairs"], target_pairs=w["pairs"], target_gates=tg, params=dict(base, max_iter=2))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, r = Q.qfs_instantiate(12, w["pairs"], target_pairs=w["pairs"], target_gates=tg,
                                 params=dict(base, max_iter=steps))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[f"G{G}_M{m}"] = {"ms_per_sweep": round(1e3 * dt / steps, 3),
                            "start_sweeps_per_s": round(r["start_sweeps"] / dt, 1)}
    return out


def time_to_distance(dev, graphs=0):
    """Time-to-distance 1e-8 (App. A defaults, MIXED with FP64 refinement) on the
    8-qubit brickwork (21 gates, M = 32, one start: the plain single-problem case)
    and with 16 starts, and on the 12-qubit U3 + CNOT template (78 gates)."""
    import torch

    from paper_2405_12866_amd import inputs as I
    from paper_2405_12866_amd import qfs as Q

    w = I.workload_8q()
    tg = torch.as_tensor(w["target_gates"]).to(dev)
    out = {}
    for starts in (1, 16):
        p = Q.qfs_default_params(multistarts=starts, m_init=32, fixed_m=1, seed=7, max_iter=3000,
                                 graphs=graphs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = Q.qfs_instantiate(8, w["pairs"], target_pairs=w["pairs"], target_gates=tg, params=p)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[f"8q_M32_starts{starts}"] = {
            "seconds": round(dt, 4), "reason": info["reason_name"], "sweeps": info["sweeps"],
            "c_train": info["c_train"], "start_sweeps": info["start_sweeps"],
            "start_sweeps_per_s": round(info["start_sweeps"] / dt, 1)}
    # 12 qubits: the U3 + CNOT template of 4 sublayers (78 gates), which the method solves
    # from random starts; 16 starts, App. A rules from M = 32 (doubling on the validation
    # cost), MIXED; the full distance of the result is measured on the device
    w12 = I.workload_u3_cnot(12, 4, seed_base=0x5A17 + 9)
    tg12 = torch.as_tensor(w12["target_gates"]).to(dev)
    fx12 = torch.as_tensor(w12["fixed"]).to(dev)
    p = Q.qfs_default_params(seed=23, m_init=32, graphs=graphs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g12, info = Q.qfs_instantiate(12, w12["pairs"], target_pairs=w12["pairs"], target_gates=tg12, params=p,
                                  kinds=w12["kinds"], fixed_gates=fx12)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    basis = torch.eye(1 << 12, dtype=torch.complex128, device=dev)
    d_full = Q.qfs_state_distance(12, Q.qfs_apply_gates(12, basis.clone(), w12["pairs"], g12),
                                  Q.qfs_apply_gates(12, basis.clone(), w12["pairs"], tg12))
    out["12q_u3cx_78gates_M0_32_starts16"] = {
        "seconds": round(dt, 4), "reason": info["reason_name"], "sweeps": info["sweeps"],
        "m_final": info["m_final"], "c_train": info["c_train"], "d_full": d_full,
        "start_sweeps": info["start_sweeps"]}
    return out


def _sweep_bytes(n, M, L, b=8):
    """Algorithmic bytes of one sweep of one start: every B_k written once and read once,
    the running state on chip, U psi read once: 2 b S L + b S with S = M 2^n."""
    S = M * (1 << n)
    return 2.0 * b * S * L + b * S


def _timed_call(Q, torch, n, pairs, tg, params):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g, info = Q.qfs_instantiate(n, pairs, target_pairs=pairs, target_gates=tg, params=params)
    torch.cuda.synchronize()
    return g, info, time.perf_counter() - t0


def _teacher_forced(Q, torch, dev, n, pairs, tg_host, M, starts, sweeps, check_starts, check_sweeps, seed):
    """Error of the device's complex64 sweeps against the FP64 oracle: `sweeps` MIXED sweeps of
    `starts` starts from Haar gates on fixed sample sets; before each sweep in check_sweeps the
    oracle runs one sweep of each start in check_starts from the device's FP64 gates (both sides
    from the same gates), and |c_gpu - c_oracle| / max(c_oracle, c_initial) is recorded."""
    import concurrent.futures as cf

    import numpy as np

    import oracle as O
    from paper_2405_12866_amd import inputs as I

    g = np.random.default_rng(seed)
    psi = I.orthonormal_samples(n, M, g)
    phi = O.apply_circuit(n, psi, pairs, tg_host)
    gates = np.stack([I.haar_gates(len(pairs), g) for _ in range(starts)])
    dpsi = torch.as_tensor(psi).to(dev)
    dphi = torch.as_tensor(phi).to(dev)
    dg = torch.as_tensor(gates).to(dev)
    worst, c_init, rows = 0.0, None, []
    with cf.ThreadPoolExecutor(max_workers=len(check_starts)) as ex:
        for sw in range(sweeps):
            start = None
            if sw in check_sweeps:
                torch.cuda.synchronize()
                start = dg.cpu().numpy().copy()
            c_gpu = Q.qfs_sweep(n, pairs, dpsi, dphi, dg, precision=Q.QFS_PREC_MIXED)
            if start is None:
                continue
            refs = list(ex.map(lambda s: O.sweep(n, pairs, psi, phi, start[s].copy())[1], check_starts))
            if c_init is None:
                c_init = max(refs)
            for s, c_ref in zip(check_starts, refs):
                e = abs(c_gpu[s] - c_ref) / max(c_ref, c_init)
                worst = max(worst, e)
                rows.append({"sweep": sw, "start": s, "c_gpu": c_gpu[s], "c_oracle": c_ref, "rel_err": e})
    return {"worst_rel_err": worst, "contract": 1e-6, "checks": rows,
            "what": f"{n} qubits, {len(pairs)} gates, M={M}, {starts} starts, complex64 sweeps (qfs_sweep) "
                    f"checked teacher-forced against the FP64 oracle at sweeps {list(check_sweeps)} for "
                    f"starts {list(check_starts)}"}


def sec8d(dev, ttd_max_iter=400):
    """Measurement rows: C1 against the oracle, C2's serial chain, C3 at every M with 1 and 16
    starts (throughput and time to distance), and the teacher-forced error of complex64 sweeps
    against the FP64 oracle at the C2 and full C3 sizes."""
    import numpy as np
    import torch

    import oracle as O
    from paper_2405_12866_amd import inputs as I
    from paper_2405_12866_amd import qfs as Q

    out = {}
    # C1: 3 qubits, (0,1),(1,2) x 3, M = 4 with doubling, complex128, to 1e-10 or 200 sweeps
    w = I.workload_3q()
    tg = torch.as_tensor(w["target_gates"]).to(dev)
    c1 = {}
    for starts in (1, 16):
        kw = dict(dist_tol=1e-10, multistarts=starts, seed=0x5A17 + 1, max_iter=200, m_init=4)
        g, info, dt = _timed_call(Q, torch, 3, w["pairs"], tg, Q.qfs_default_params(precision=Q.QFS_PREC_FP64, **kw))
        t0 = time.perf_counter()
        g_ref, ref = O.instantiate(3, w["pairs"], target_pairs=w["pairs"], target_gates=w["target_gates"],
                                   params=O.default_params(**kw))
        dt_o = time.perf_counter() - t0
        same = all(info[k] == ref[k] for k in ("reason_name", "sweeps", "best_start", "restarts", "m_final"))
        c1[f"starts{starts}"] = {
            "gpu_s": round(dt, 4), "oracle_s_one_thread": round(dt_o, 4), "reason": info["reason_name"],
            "sweeps": info["sweeps"], "doublings": info["restarts"], "m_final": info["m_final"],
            "c_train": info["c_train"],
            "vs_oracle": {"same_start_reason_sweeps_doublings": bool(same),
                          "c_train_abs_err": abs(info["c_train"] - ref["c_train"]),
                          "gates_max_abs_err": float(np.max(np.abs(g.cpu().numpy() - g_ref)))}}
    out["C1_3q_L6_M4_c128"] = c1
    # C2: 8 qubits, 21 gates, M = 32, one start (plain): the serial chain per gate step
    w8 = I.workload_8q()
    tg8 = torch.as_tensor(w8["target_gates"]).to(dev)
    L8 = len(w8["pairs"])
    base = dict(multistarts=1, m_init=32, fixed_m=1, seed=5, precision=Q.QFS_PREC_MIXED, diff_tol_r=0.0,
                plateau_window=1 << 30, dist_tol=0.0)
    _timed_call(Q, torch, 8, w8["pairs"], tg8, Q.qfs_default_params(max_iter=5, **base))
    _, info, dt = _timed_call(Q, torch, 8, w8["pairs"], tg8, Q.qfs_default_params(max_iter=200, **base))
    sw = info["start_sweeps"]
    out["C2_8q_L21_M32_1start"] = {
        "sweeps": sw, "wall_us_per_sweep": round(1e6 * dt / sw, 2),
        "device_us_per_sweep": round(1e6 * info["sweep_seconds"] / sw, 2),
        "device_us_per_gate_step": round(1e6 * info["sweep_seconds"] / sw / L8, 3),
        "algorithmic_GBps": round(_sweep_bytes(8, 32, L8) * sw / dt / 1e9, 2),
        "error_vs_oracle": _teacher_forced(Q, torch, dev, 8, w8["pairs"], w8["target_gates"], 32, 1, 6, [0],
                                           (0, 5), seed=81)}
    # C3: 12 qubits, 44 gates, every M with 1 and 16 starts
    w12 = I.workload_12q()
    tg12 = torch.as_tensor(w12["target_gates"]).to(dev)
    L12 = len(w12["pairs"])
    thr, ttd = [], []
    for M in (8, 16, 32, 64, 128, 256):
        for starts in (1, 16):
            base = dict(multistarts=starts, m_init=M, fixed_m=1, seed=0x5A17 + 3, precision=Q.QFS_PREC_MIXED,
                        diff_tol_r=0.0, plateau_window=1 << 30, dist_tol=0.0)
            _timed_call(Q, torch, 12, w12["pairs"], tg12, Q.qfs_default_params(max_iter=3, **base))
            k = 40 if M * starts <= 512 else 20
            _, info, dt = _timed_call(Q, torch, 12, w12["pairs"], tg12, Q.qfs_default_params(max_iter=k, **base))
            sw = info["start_sweeps"]
            ab = _sweep_bytes(12, M, L12) * sw
            thr.append({"M": M, "starts": starts, "start_sweeps": sw,
                        "start_sweeps_per_s": round(sw / dt, 1),
                        "device_ms_per_sweep": round(1e3 * info["sweep_seconds"] / info["sweeps"], 4),
                        "algorithmic_GBps_wall": round(ab / dt / 1e9, 1),
                        "algorithmic_GBps_device": round(ab / info["sweep_seconds"] / 1e9, 1)})
        p = Q.qfs_default_params(multistarts=16, m_init=M, fixed_m=1, seed=0x5A17 + 3, precision=Q.QFS_PREC_MIXED,
                                 max_iter=ttd_max_iter)
        _, info, dt = _timed_call(Q, torch, 12, w12["pairs"], tg12, p)
        ttd.append({"M": M, "starts": 16, "reason": info["reason_name"],
                    "reached_1e-8": info["reason_name"] == "SUCCESS", "sweeps": info["sweeps"],
                    "c_train": info["c_train"], "c_val": info["c_val"], "seconds": round(dt, 3)})
    out["C3_12q_L44_throughput"] = thr
    out["C3_12q_L44_time_to_distance"] = {
        "rows": ttd,
        "note": ("fixed M, App. A stopping rules (plateau 1e-5 over 5 sweeps), at most "
                 f"{ttd_max_iter} sweeps; this brickwork with Haar-random target gates stalls far above 1e-8 "
                 "(in the oracle as well), so the rows report where it stops")}
    out["C3_12q_M256_error_vs_oracle"] = _teacher_forced(Q, torch, dev, 12, w12["pairs"], w12["target_gates"],
                                                         256, 16, 5, [0, 9], (0, 4), seed=83)
    return out


def batched(dev, count, plain_sample):
    """Batched workload: `count` problems (n ~ U{3..7}, L ~ U{2..20} random pairs, Haar
    target from the template), 16 starts each, M0 = 2^(n-1) with doubling to 2^n,
    App. A stopping rules, MIXED precision, automatic sweeps per launch (8, raised as jobs finish). Compared
    with plain qfs_instantiate calls, one problem at a time, on the first
    `plain_sample` problems (same seeds, same success criterion), extrapolated."""
    import numpy as np
    import torch

    from paper_2405_12866_amd import inputs as I
    from paper_2405_12866_amd import qfs as Q

    probs = I.batched_problems(count)
    dprobs = [dict(n=p["n"], pairs=p["pairs"], target_pairs=p["target_pairs"],
                   target_gates=torch.as_tensor(p["target_gates"]).to(dev)) for p in probs]
    m0 = np.array([1 << (p["n"] - 1) for p in probs], dtype=np.int32)
    params = Q.qfs_default_params(multistarts=16, seed=0x5A17 + 4, batch_sweeps=0,
                                  precision=Q.QFS_PREC_MIXED)
    warm = min(256, count)  # code objects + work-group-size autotuner
    Q.qfs_instantiate_batch_ex(dprobs[:warm], params, m_init=m0[:warm])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, infos = Q.qfs_instantiate_batch_ex(dprobs, params, m_init=m0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ok = sum(r["reason_name"] == "SUCCESS" for r in infos)
    job_sweeps = sum(r["start_sweeps"] for r in infos)
    # algorithmic bytes (2 b S L + b S per job-sweep, b = 8) from the amplitude-gate updates
    # of each problem's sweeps, (M + M_val) 2^n L with M_val = M: the training half
    alg = 0.0
    for p, r in zip(probs, infos):
        train = 0.5 * r["amp_updates"]
        alg += 2.0 * 8 * train + 8.0 * train / len(p["pairs"])
    out = {"problems": count, "starts": 16, "wall_s": round(dt, 3),
           "problems_per_s": round(count / dt, 1), "successes": ok,
           "job_sweeps": job_sweeps, "job_sweeps_per_s": round(job_sweeps / dt, 1),
           "doublings": sum(r["restarts"] for r in infos),
           "device_s": round(infos[0]["sweep_seconds"], 3),
           "algorithmic_GBps": round(alg / dt / 1e9, 1),
           "algorithmic_note": "complex64 bytes for every sweep (the final complex128 sweeps counted at 8 B)"}
    k = min(plain_sample, count)
    if k > 0:
        t_plain, ok_plain, ok_batch = 0.0, 0, 0
        for i in range(k):
            p = dict(params, seed=params["seed"] + i, m_init=int(m0[i]))
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, r = Q.qfs_instantiate(probs[i]["n"], probs[i]["pairs"], target_pairs=probs[i]["pairs"],
                                     target_gates=dprobs[i]["target_gates"], params=p)
            torch.cuda.synchronize()
            t_plain += time.perf_counter() - t1
            ok_plain += r["reason_name"] == "SUCCESS"
            ok_batch += infos[i]["reason_name"] == "SUCCESS"
        est = t_plain / k * count
        out["plain_loop"] = {"sample": k, "sample_s": round(t_plain, 3),
                             "sample_successes": ok_plain, "batched_successes_on_sample": ok_batch,
                             "extrapolated_s": round(est, 2), "batched_speedup": round(est / dt, 1)}
    return out


def batched_u3cx(dev, count, plain_sample):
    """Batched U3 + CNOT workload: `count` problems (n ~ U{3..7}, 1-4 brickwork sublayers
    of CNOT blocks with one-qubit gates, Haar one-qubit targets), 16 starts, M0 =
    2^(n-1), App. A rules, MIXED, automatic sweeps per launch; compared with plain
    qfs_instantiate calls on the first `plain_sample` problems, extrapolated."""
    import numpy as np
    import torch

    from paper_2405_12866_amd import inputs as I
    from paper_2405_12866_amd import qfs as Q

    probs = I.batched_u3_cnot_problems(count)
    dprobs = [dict(n=p["n"], pairs=p["pairs"], kinds=p["kinds"],
                   fixed_gates=torch.as_tensor(p["fixed"]).to(dev), target_pairs=p["target_pairs"],
                   target_gates=torch.as_tensor(p["target_gates"]).to(dev)) for p in probs]
    m0 = np.array([1 << (p["n"] - 1) for p in probs], dtype=np.int32)
    params = Q.qfs_default_params(multistarts=16, seed=0x5A17 + 10, batch_sweeps=0,
                                  precision=Q.QFS_PREC_MIXED)
    warm = min(128, count)
    Q.qfs_instantiate_batch_ex(dprobs[:warm], params, m_init=m0[:warm])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, infos = Q.qfs_instantiate_batch_ex(dprobs, params, m_init=m0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    job_sweeps = sum(r["start_sweeps"] for r in infos)
    out = {"problems": count, "starts": 16, "wall_s": round(dt, 3), "problems_per_s": round(count / dt, 1),
           "successes": sum(r["reason_name"] == "SUCCESS" for r in infos), "job_sweeps": job_sweeps,
           "job_sweeps_per_s": round(job_sweeps / dt, 1)}
    k = min(plain_sample, count)
    if k > 0:
        t_plain, ok_plain = 0.0, 0
        for i in range(k):
            p = dict(params, seed=params["seed"] + i, m_init=int(m0[i]))
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, r = Q.qfs_instantiate(probs[i]["n"], probs[i]["pairs"], target_pairs=probs[i]["pairs"],
                                     target_gates=dprobs[i]["target_gates"], params=p,
                                     kinds=probs[i]["kinds"], fixed_gates=dprobs[i]["fixed_gates"])
            torch.cuda.synchronize()
            t_plain += time.perf_counter() - t1
            ok_plain += r["reason_name"] == "SUCCESS"
        est = t_plain / k * count
        out["plain_loop"] = {"sample": k, "sample_s": round(t_plain, 3), "sample_successes": ok_plain,
                             "batched_successes_on_sample": sum(infos[i]["reason_name"] == "SUCCESS" for i in range(k)),
                             "extrapolated_s": round(est, 2), "batched_speedup": round(est / dt, 1)}
    return out


def learned(dev, count, large):
    """Learned initial M and start pruning against the plain method (M from 2, doubling,
    16 starts, App. A rules, MIXED), both batched, on `count` held-out problems drawn like
    the predictor's training set (new seeds); optionally `large` 10-14 qubit random-pair
    problems through the single-problem entry points. Needs the trained weight file."""
    import torch

    from paper_2405_12866_amd import inputs as I
    from paper_2405_12866_amd import predictor as PR
    from paper_2405_12866_amd import qfs as Q

    if not os.path.exists(PR.DEFAULT_WEIGHTS):
        return {"skipped": f"no weight file {os.path.basename(PR.DEFAULT_WEIGHTS)}"}
    Q.qfs_mlp_load(PR.DEFAULT_WEIGHTS)
    out = {}
    if count > 0:
        probs = PR.training_problems(count, seed_base=0x5A17 + 0x40)  # disjoint from the training streams (+5, +6)
        dprobs = PR.device_problems(probs, dev)
        params = Q.qfs_default_params(multistarts=16, seed=0x5A17 + 6, batch_sweeps=0,
                                      precision=Q.QFS_PREC_MIXED)
        Q.qfs_instantiate_batch(dprobs[:128], params)  # code objects and autotuner
        rows = {}
        for name, fn in (("plain", Q.qfs_instantiate_batch), ("learned", Q.qfs_instantiate_batch_learned)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, infos = fn(dprobs, params)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rows[name] = {"wall_s": round(dt, 3), "successes": sum(r["reason_name"] == "SUCCESS" for r in infos),
                          "start_sweeps": sum(r["start_sweeps"] for r in infos),
                          "amp_updates": sum(r["amp_updates"] for r in infos),
                          "doublings": sum(r["restarts"] for r in infos)}
            if name == "learned":
                rows[name]["fallbacks"] = sum(r["fallback"] for r in infos)
                rows[name]["mean_starts_run"] = round(sum(r["starts_run"] for r in infos) / count, 2)
                rows[name]["mean_m_predicted"] = round(sum(r["m_predicted"] for r in infos) / count, 2)
        rows["problems"] = count
        rows["time_to_solution_speedup"] = round(rows["plain"]["wall_s"] / rows["learned"]["wall_s"], 2)
        rows["work_ratio"] = round(rows["learned"]["amp_updates"] / max(1.0, rows["plain"]["amp_updates"]), 3)
        out["held_out"] = rows
        # one problem at a time (no batch tail): a stratified sample of the same problems,
        # three quarters from the 3-7 qubit part and one quarter from the 8-10 qubit part
        small = count - count // 4
        pick = list(range(min(48, small))) + list(range(small, min(small + 16, count)))
        one = {"plain": {"seconds": 0.0, "successes": 0, "amp_updates": 0.0, "doublings": 0},
               "learned": {"seconds": 0.0, "successes": 0, "amp_updates": 0.0, "doublings": 0, "fallbacks": 0}}
        for name, fn in (("plain", Q.qfs_instantiate), ("learned", Q.qfs_instantiate_learned)):
            for i in pick[:2]:  # code objects
                fn(dprobs[i]["n"], dprobs[i]["pairs"], target_pairs=dprobs[i]["target_pairs"],
                   target_gates=dprobs[i]["target_gates"], params=params)
            for i in pick:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, r = fn(dprobs[i]["n"], dprobs[i]["pairs"], target_pairs=dprobs[i]["target_pairs"],
                          target_gates=dprobs[i]["target_gates"], params=params)
                torch.cuda.synchronize()
                row = one[name]
                row["seconds"] += time.perf_counter() - t0
                row["successes"] += r["reason_name"] == "SUCCESS"
                row["amp_updates"] += r["amp_updates"]
                row["doublings"] += r["restarts"]
                if name == "learned":
                    row["fallbacks"] += r["fallback"]
            one[name]["seconds"] = round(one[name]["seconds"], 3)
        one["problems"] = len(pick)
        one["time_to_solution_speedup"] = round(one["plain"]["seconds"] / max(1e-9, one["learned"]["seconds"]), 2)
        one["work_ratio"] = round(one["learned"]["amp_updates"] / max(1.0, one["plain"]["amp_updates"]), 3)
        out["one_at_a_time"] = one
    if large > 0:
        g = I.rng(I.derive_seed(0x5A17 + 7))
        res = {"plain": [], "learned": []}
        for i in range(large):
            n = int(g.integers(10, 15))
            L = int(g.integers(30, 121))
            pairs = I.random_pair_template(n, L, g)
            tg = torch.as_tensor(I.haar_gates(L, g)).to(dev)
            p = Q.qfs_default_params(multistarts=16, seed=100 + i, max_iter=2000, time_budget_s=20.0)
            for name, fn in (("plain", Q.qfs_instantiate), ("learned", Q.qfs_instantiate_learned)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, r = fn(n, pairs, target_pairs=pairs, target_gates=tg, params=p)
                torch.cuda.synchronize()
                res[name].append({"n": n, "L": L, "s": round(time.perf_counter() - t0, 2),
                                  "reason": r["reason_name"], "c_train": r["c_train"],
                                  "m_final": r["m_final"]})
        out["large"] = res
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library "
              f"has no multi-GPU path; problems and multistarts are independent and one GPU "
              f"runs them all", file=sys.stderr)
        sys.exit(2)
    if not args.bwd_split:
        os.environ["QFS_BWD_SPLIT"] = "0"  # read once by the library when it first runs
    import torch

    from paper_2405_12866_amd import inputs as I
    from paper_2405_12866_amd import qfs as Q

    Q.load()
    dev = "cuda:0"
    w = I.workload_12q()
    n, pairs = w["n"], w["pairs"]
    L = len(pairs)
    M, S = args.m, args.starts
    tg = torch.as_tensor(w["target_gates"]).to(dev)
    base = Q.qfs_default_params(multistarts=S, m_init=M, fixed_m=1, seed=0x5A17 + 3,
                                precision=Q.QFS_PREC_MIXED, diff_tol_r=0.0, plateau_window=1 << 30,
                                graphs=args.graphs)
    # warmup (also loads code objects)
    Q.qfs_instantiate(n, pairs, target_pairs=pairs, target_gates=tg,
                      params=dict(base, max_iter=max(1, args.warmup)))
    torch.cuda.synchronize()
    # timed region: one call, max_iter = steps, no instrumentation
    t0 = time.perf_counter()
    _, info = Q.qfs_instantiate(n, pairs, target_pairs=pairs, target_gates=tg,
                                params=dict(base, max_iter=args.steps))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = info["start_sweeps"] / dt
    N = 1 << n
    S_amp = M * N
    # spread: the same call repeated (whole call on the host clock after a device
    # synchronisation; the sweeps alone by the library's hipEvents)
    rep = None
    if args.repeats > 0:
        import numpy as np
        whole, sweeps_only = [], []
        for _ in range(args.repeats):
            t1 = time.perf_counter()
            _, ri = Q.qfs_instantiate(n, pairs, target_pairs=pairs, target_gates=tg,
                                      params=dict(base, max_iter=args.steps))
            torch.cuda.synchronize()
            whole.append(1e3 * (time.perf_counter() - t1) / args.steps)
            sweeps_only.append(1e3 * ri["sweep_seconds"] / args.steps)
        q = lambda v, f: float(np.percentile(v, f))
        rep = {"calls": args.repeats, "steps_per_call": args.steps,
               "ms_per_step_whole_call": {"median": round(q(whole, 50), 4),
                                          "iqr": [round(q(whole, 25), 4), round(q(whole, 75), 4)]},
               "ms_per_step_sweeps_only": {"median": round(q(sweeps_only, 50), 4),
                                           "iqr": [round(q(sweeps_only, 25), 4), round(q(sweeps_only, 75), 4)]},
               "start_sweeps_per_s_median": round(S * 1e3 / q(whole, 50), 2)}
    # instrumented region (same workload): hipEvents around every kernel launch on the
    # call's stream give the per-kernel durations for the roofline
    roof, classes = None, None
    if args.timing:
        _, tinfo = Q.qfs_instantiate(n, pairs, target_pairs=pairs, target_gates=tg,
                                     params=dict(base, max_iter=args.steps, timing=1))
        kl, ks, kb = tinfo["kernel_launches"], tinfo["kernel_seconds"], tinfo["kernel_bytes"]
        if kl[0] > 0:
            # algorithmic bytes of the backward pass (the method's minimum: every B_k
            # written once by the forward pass and read once here, the running state kept
            # on chip): b S per start for each of the L gates, plus U psi read once per
            # sweep (b = 8, complex64). The grouped passes cover a group of gates per
            # launch, so per launch this is (L + 1) b S per start-sweep over the passes of
            # a sweep. With timing on, every launch covers all running starts (one
            # stream), and the bench disables the plateau stop, so every launch covers all
            # S starts.
            sweeps = tinfo["start_sweeps"] / S
            alg = sweeps * S * (L + 1) * 8.0 * S_amp
            achieved = alg / ks[0] / 1e9
            kernel_moved = kb[0] / ks[0] / 1e9  # what the kernel itself reads and writes
            traffic = measured_traffic()
            roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                    "traffic": traffic,
                    "traffic_source": ("rocprofv3 --pmc FETCH_SIZE + WRITE_SIZE of this kernel, from the "
                                       "committed summary taken on the current kernel source "
                                       "(profiles/k_bwd_group_12q_M256_S16_pmc.md), calibrated on a "
                                       "256 MiB device copy") if traffic else None,
                    "kernel": ("k_bwd_group (one pass per gate group: the previous group's 16x16 "
                               "operator and the group's 16x16 second-moment matrix on the matrix cores)"),
                    "launches_per_sweep": round(kl[0] / sweeps, 2),
                    "avg_launch_us": round(1e6 * ks[0] / kl[0], 2),
                    "algorithmic_bytes_per_launch": alg / kl[0],
                    "kernel_moved_bytes_per_launch": kb[0] / kl[0],
                    "kernel_moved_GBps": round(kernel_moved, 1),
                    "kernel_moved_frac": round(kernel_moved / HBM_PEAK_GBPS, 4)}
        classes = {name: {"launches": kl[i], "seconds": round(ks[i], 5),
                          "GBps": round(kb[i] / ks[i] / 1e9, 1) if ks[i] > 0 and kb[i] > 0 else None,
                          "avg_us": round(1e6 * ks[i] / kl[i], 2) if kl[i] else None}
                   for i, name in enumerate(["bwd_step", "forward", "distance", "env_finalize_polar"])}
    sweep_alg_bytes = 16.0 * S_amp * L + 8.0 * S_amp  # per start-sweep, complex64
    extra = {
        "wall_s": round(dt, 4), "start_sweeps": info["start_sweeps"],
        "device_sweep_s": round(info["sweep_seconds"], 4),
        "sweep_algorithmic_GBps": round(sweep_alg_bytes * info["start_sweeps"] / dt / 1e9, 1),
        "sweep_algorithmic_frac": round(sweep_alg_bytes * info["start_sweeps"] / dt / 1e9 / HBM_PEAK_GBPS, 4),
        "kernel_classes": classes,
        "final_c_train": info["c_train"], "final_c_val": info["c_val"],
        "repeats": rep,
    }
    if args.sec8d:
        extra["measurement_rows"] = sec8d(dev)
    if args.u3cx:
        extra["u3_cnot"] = u3_cnot(dev, M, S, args.steps, args.warmup, args.timing)
    if args.shares:
        extra["shard_shares"] = shard_shares(dev, M, S, args.steps, [int(x) for x in args.shares.split(",") if x])
    if args.qudits:
        extra["qudits"] = qudits_leg(dev, args.steps)
    if args.qf:
        extra["qf_vs_qfs"] = qf_vs_qfs(dev, [int(x) for x in args.qf.split(",") if x])
    if args.batched > 0:
        extra["batched"] = batched(dev, args.batched, args.plain_sample)
    if args.batched_u3cx > 0:
        extra["batched_u3cx"] = batched_u3cx(dev, args.batched_u3cx, args.plain_sample)
    if args.learned > 0 or args.learned_large > 0:
        extra["learned"] = learned(dev, args.learned, args.learned_large)
    if not args.no_ttd:
        extra["time_to_distance"] = time_to_distance(dev, args.graphs)
        extra["time_to_distance"]["12q_note"] = (
            "12q Haar-random brickworks of general two-qubit gates do not reach 1e-8 from random "
            "initial gates (they stall near c_train 1.8, in the oracle as well); the 12-qubit "
            "time-to-distance is reported on the U3 + CNOT template")
    rec = {
        "metric": METRIC, "value": round(value, 2), "unit": "start-sweeps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * dt / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64+f64",
        "data": "synthetic",
        "config": {"workload": f"12q brickwork depth 8 ({L} two-qubit gates), Haar target from the "
                               f"same template, M={M} fixed, {S} lock-step starts, MIXED precision",
                   "n_qubits": n, "gates": L, "M": M, "starts": S, "parallelism": "single GPU"},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w, M, S)
    rec["extra"] = extra
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
