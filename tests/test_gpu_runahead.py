"""The control loop's run-ahead (sweep t + 1 issued before the costs of sweep t are read,
undone from a snapshot of the gates where a start stops or a decision for all starts is
taken) and its parts on their own streams running from one sweep into the next: the
result equals that of the loop that decides after every sweep. MI355X only; calls go
through the C ABI.

The loop that decides after every sweep is the one with kernel timing on (timing = 1: one
stream, no run-ahead); both run the same kernels with the same work split per start, so
their FP64 and complex64 results are bitwise equal.
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


def test_staggered_plateaus_match_oracle():
    """An unreachable target (deeper random template): the 8 starts stop on the plateau
    test at different sweeps while the others go on; the run ends with the oracle's start,
    reason, sweep count, cost and gates (FP64, fixed M = 8 on 5 qubits)."""
    n = 5
    g = np.random.default_rng(31)
    pairs = [tuple(p) for p in I.random_pair_template(n, 6, g)]
    tpairs = [tuple(p) for p in I.random_pair_template(n, 14, g)]
    tg = I.haar_gates(len(tpairs), g)
    kw = dict(dist_tol=1e-10, multistarts=8, seed=19, max_iter=400, diff_tol_r=1e-4, m_init=8, fixed_m=1)
    say(f"run-ahead staggered plateaus n={n} L={len(pairs)}")
    g_ref, ref = O.instantiate(n, pairs, target_pairs=tpairs, target_gates=tg, params=O.default_params(**kw))
    assert ref["reason_name"] != "SUCCESS"
    g_gpu, info = Q.qfs_instantiate(n, pairs, target_pairs=tpairs, target_gates=dev(tg),
                                    params=Q.qfs_default_params(precision=Q.QFS_PREC_FP64, **kw))
    say(f"  device {info['reason_name']} start {info['best_start']} after {info['sweeps']} sweeps; "
        f"oracle {ref['reason_name']} start {ref['best_start']} after {ref['sweeps']}")
    for key in ("reason_name", "best_start", "sweeps", "m_final"):
        assert info[key] == ref[key], (key, info[key], ref[key])
    assert abs(info["c_train"] - ref["c_train"]) <= 1e-9 * ref["c_train"]
    assert np.max(np.abs(host(g_gpu) - g_ref)) < 1e-8


def _run(n, pairs, tpairs, tg, timing, **kw):
    p = Q.qfs_default_params(timing=timing, **kw)
    g, info = Q.qfs_instantiate(n, pairs, target_pairs=tpairs, target_gates=dev(tg), params=p)
    return host(g), info


@pytest.mark.parametrize("precision", [Q.QFS_PREC_MIXED, Q.QFS_PREC_FP64], ids=["mixed", "fp64"])
def test_parts_and_run_ahead_equal_one_sweep_at_a_time(precision):
    """16 starts of 2^18 amplitudes each (two parts on two streams), plateau stops at
    different sweeps: run-ahead with the parts running on equals timing = 1 bit for bit
    (start, reason, sweeps, costs, gates)."""
    n, M = 10, 256
    pairs = [tuple(p) for p in I.brickwork_template(n, 4)]
    g = np.random.default_rng(77)
    tpairs = [tuple(p) for p in I.random_pair_template(n, 40, g)]
    tg = I.haar_gates(len(tpairs), g)
    kw = dict(dist_tol=1e-10, multistarts=16, seed=23, max_iter=60, diff_tol_r=2e-3, m_init=M, fixed_m=1,
              precision=precision)
    say(f"run-ahead vs one sweep at a time n={n} M={M} L={len(pairs)} precision={precision}")
    g0, a = _run(n, pairs, tpairs, tg, 0, **kw)
    g1, b = _run(n, pairs, tpairs, tg, 1, **kw)
    say(f"  {a['reason_name']} start {a['best_start']} after {a['sweeps']} sweeps, "
        f"{a['start_sweeps']} start-sweeps; one at a time: {b['reason_name']} / {b['best_start']} / "
        f"{b['sweeps']} / {b['start_sweeps']}")
    for key in ("reason_name", "best_start", "sweeps", "start_sweeps", "c_train", "c_val", "m_final"):
        assert a[key] == b[key], (key, a[key], b[key])
    assert a["start_sweeps"] < 16 * 60  # some starts stopped before the last sweep
    assert np.array_equal(g0, g1)
