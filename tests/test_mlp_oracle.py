"""Pins of the FP64 network oracle (oracle/mlp_oracle.py) and of the template features
(host code of the library, no device work). CPU only.

The oracle's analytic gradient is pinned by central finite differences of its own loss
(a different computation: no chain rule), its loss by the closed form at zero weights,
and its bfloat16 rounding by torch's CPU float32 -> bfloat16 conversion (round to
nearest, ties to even).
"""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as MO


def _rand_theta(rng, scale=1.0):
    th = np.zeros(MO.NUM_PARAMS)
    o = 0
    for _, shape in MO.SIZES:
        k = int(np.prod(shape))
        fan_in = shape[1] if len(shape) == 2 else 4
        th[o:o + k] = rng.uniform(-1, 1, k) * scale * math.sqrt(6.0 / fan_in)
        o += k
    return th


def _data(rng, B):
    X = rng.uniform(0, 1, (B, MO.F))
    T = np.stack([rng.integers(1, 8, B).astype(float), rng.uniform(0, 1, B)], 1)
    T[::3, 0] = np.nan  # unlabelled rows
    return X, T


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    th = _rand_theta(rng)
    X, T = _data(rng, 7)
    g = MO.gradient(th, X, T)
    # every bias and output weight, plus a random sample of hidden weights
    idx = list(range(128 * 64, 128 * 64 + 128))
    b2 = MO.NUM_PARAMS - 2 - 256 - 128
    idx += list(range(b2, MO.NUM_PARAMS))
    idx += list(rng.choice(128 * 64, 150, replace=False)) + list(rng.choice(np.arange(8320, 8320 + 16384), 150, replace=False))
    h = 1e-6
    worst = 0.0
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (MO.loss(th + e, X, T) - MO.loss(th - e, X, T)) / (2 * h)
        # the finite-difference rounding error is about eps * |loss| / h ~ 1e-9
        worst = max(worst, abs(fd - g[i]) / (1e-8 + 1e-6 * abs(g[i])))
    assert worst < 1.0, worst


def test_gradient_fails_if_a_term_is_dropped():
    """The finite-difference check is sensitive to the regression term alone."""
    rng = np.random.default_rng(1)
    th = _rand_theta(rng)
    X, T = _data(rng, 5)
    T2 = T.copy()
    T2[:, 0] = np.nan
    assert np.max(np.abs(MO.gradient(th, X, T) - MO.gradient(th, X, T2))) > 1e-3


def test_loss_closed_form_at_zero_weights():
    rng = np.random.default_rng(2)
    X, T = _data(rng, 9)
    th = np.zeros(MO.NUM_PARAMS)
    lab = np.isfinite(T[:, 0])
    expect = (0.5 * np.sum(T[lab, 0] ** 2) + 9 * math.log(2.0)) / 9
    assert abs(MO.loss(th, X, T) - expect) < 1e-12
    y, _ = MO.forward(th, X)
    assert np.all(y == 0)


def test_output_bias_gradient_closed_form():
    """With zero weights y = b3, so dL/db3 = mean([lab](b0 - t0)) and mean(sigmoid(b1) - t1)."""
    rng = np.random.default_rng(3)
    X, T = _data(rng, 11)
    th = np.zeros(MO.NUM_PARAMS)
    th[-2], th[-1] = 0.7, -0.4
    g = MO.gradient(th, X, T)
    lab = np.isfinite(T[:, 0])
    assert abs(g[-2] - np.sum(0.7 - T[lab, 0]) / 11) < 1e-14
    assert abs(g[-1] - np.mean(1 / (1 + math.exp(0.4)) - T[:, 1])) < 1e-14


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.standard_normal(5000).astype(np.float32),
                        (rng.standard_normal(1000) * 1e-30).astype(np.float32),
                        np.array([0.0, -0.0, 1.0, np.inf, -np.inf, 3.4e38, -3.4e38], np.float32)])
    # exact ties: mantissa low half = 0x8000 with both parities of the kept bit
    ties = (np.array([0x3F808000, 0x3F818000, 0xBF808000, 0xBF818000], np.uint32)).view(np.float32)
    x = np.concatenate([x, ties])
    ours = MO.bf16_round(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(ours.view(np.uint32), ref.view(np.uint32))


# ------------------------------------------------------------------ template features
def _features(n, pairs):
    from paper_2405_12866_amd import qfs as Q
    return Q.qfs_features(n, pairs)


def test_features_linear_3q():
    f = _features(3, [(0, 1), (1, 2)] * 3)
    assert f[0] == pytest.approx(3 / 16) and f[1] == pytest.approx(6 / 128)
    assert f[2] == pytest.approx(6 / 64)  # every gate shares qubit 1: depth 6
    assert f[3] == pytest.approx(math.log2(1 + 96 / 8))
    assert f[5] == pytest.approx(2 / 6) and f[6] == 1.0 and f[7] == 1.0
    assert f[9] == pytest.approx(1 / 3) and f[10] == 1.0
    hist = np.zeros(16)
    hist[3], hist[6] = 2 / 3, 1 / 3
    assert np.allclose(f[12:28], hist)
    assert f[28] == 1.0 and np.all(f[29:44] == 0)
    layers = np.zeros(16)
    for l in range(1, 7):
        layers[min(15, int((l - 1) * 16 / 6))] += 1 / 6
    assert np.allclose(f[44:60], layers)
    assert f[60] == pytest.approx(0.5) and f[61] == pytest.approx(8 / 96)
    assert f[62] == pytest.approx(1 / 3) and f[63] == 1.0


def test_features_brickwork_and_components():
    from paper_2405_12866_amd import inputs as I
    pairs = I.brickwork_template(8, 6)
    f = _features(8, pairs)
    assert len(pairs) == 21
    assert f[2] == pytest.approx(6 / 64)  # one layer per sublayer
    for lo, hi in ((12, 28), (28, 44), (44, 60)):
        assert f[lo:hi].sum() == pytest.approx(1.0, abs=1e-6)
    g = _features(4, [(0, 1)])
    assert g[9] == pytest.approx(3 / 4)  # components {0,1}, {2}, {3}
    assert g[6] == pytest.approx(0.5)


def test_features_reject_bad_templates():
    from paper_2405_12866_amd import qfs as Q
    with pytest.raises(Q.QfsError):
        _features(3, [(0, 0)])
    with pytest.raises(Q.QfsError):
        _features(3, [(0, 3)])
