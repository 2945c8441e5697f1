"""Device buffers kept between calls: a call that reuses the buffers of an earlier call
(of the same sizes, holding that call's data) returns exactly what a call on freshly
allocated buffers returns, doublings and the two-stream backward pass included, and
qfs_release_device_cache returns the kept buffers. Every case runs the HIP path through
the C ABI.
"""
import sys

import numpy as np
import pytest

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


def _call(n, sublayers, seed, precision, m_init, iters):
    pairs = I.brickwork_template(n, sublayers)
    tg = I.haar_gates(len(pairs), I.rng(seed))
    p = Q.qfs_default_params(multistarts=4, m_init=m_init, max_iter=iters, seed=seed,
                             precision=precision)
    g, info = Q.qfs_instantiate(n, pairs, target_pairs=pairs, target_gates=dev(tg), params=p)
    torch.cuda.synchronize()
    return g.cpu().numpy(), info


KEYS = ("reason", "m_final", "sweeps", "restarts", "m_total", "start_sweeps", "refined",
        "best_start", "c_train", "c_val")


@pytest.mark.parametrize("precision", [Q.QFS_PREC_MIXED, Q.QFS_PREC_FP64])
def test_reused_buffers_give_identical_results(precision):
    say(f"cache reuse: precision {precision}")
    # m_init 2 on 6 qubits doubles a few times (buffers given back and allocated again
    # inside the call); 8 sweeps at M = 16 on 7 qubits do not
    cases = [(6, 4, 11, 2, 60), (7, 4, 12, 16, 8)]
    fresh = []
    for case in cases:
        Q.qfs_release_device_cache()
        fresh.append(_call(*case[:3], precision, *case[3:]))
    # each case twice more, interleaved, so that every call runs on buffers that the
    # calls before it (other sizes included) have written
    for rep in range(2):
        for case, (g1, i1) in reversed(list(zip(cases, fresh))):
            g2, i2 = _call(*case[:3], precision, *case[3:])
            say(f"  case {case} rep {rep}: {i1['reason_name']} M {i1['m_final']} sweeps {i1['sweeps']}")
            for k in KEYS:
                assert i1[k] == i2[k], (case, rep, k, i1[k], i2[k])
            assert np.array_equal(g1, g2), (case, rep)


def test_release_returns_kept_buffers():
    say("cache release")
    _call(6, 4, 13, Q.QFS_PREC_MIXED, 8, 4)
    freed = Q.qfs_release_device_cache()
    assert freed > 0
    assert Q.qfs_release_device_cache() == 0
    # a call after the release allocates afresh and still works
    g, info = _call(6, 4, 13, Q.QFS_PREC_MIXED, 8, 4)
    assert np.isfinite(info["c_train"]) and info["sweeps"] >= 1


def test_concurrent_calls_match_sequential():
    """Two host threads, each on its own stream, run calls at the same time (the kept
    buffers, the pinned cost buffers and the pool streams are shared): every result
    equals the one-at-a-time result bit for bit."""
    import threading
    say("cache: concurrent calls")
    cases = [(6, 4, 21, Q.QFS_PREC_MIXED, 2, 40), (7, 4, 22, Q.QFS_PREC_MIXED, 16, 10)]
    ref = [_call(*c) for c in cases]
    out = [[None, None], [None, None]]
    errs = []

    def worker(t):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for rep in range(2):
                    out[t][rep] = _call(*cases[t])
        except Exception as e:  # reported below
            errs.append(e)

    th = [threading.Thread(target=worker, args=(t,)) for t in range(2)]
    for x in th:
        x.start()
    for x in th:
        x.join(timeout=100)
    assert not any(x.is_alive() for x in th), "a worker did not finish"
    assert not errs, errs
    for t, c in enumerate(cases):
        g1, i1 = ref[t]
        for rep in range(2):
            g2, i2 = out[t][rep]
            for k in KEYS:
                assert i1[k] == i2[k], (c, rep, k, i1[k], i2[k])
            assert np.array_equal(g1, g2), (c, rep)
