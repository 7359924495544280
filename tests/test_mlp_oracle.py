"""Pins of the FP64 surrogate-network reference (oracle/mlp.py): its gradient
against central finite differences, its loss against the definition on a
hand-checkable case, and BF16 rounding against the format's definition."""
import numpy as np
import pytest

from oracle import mlp as M

rng = np.random.default_rng(1706070626)


def _batch(n):
    x = np.stack([rng.uniform(-12, 12, n), rng.uniform(-12, 12, n), rng.uniform(0, 0.998, n),
                  np.radians(rng.uniform(5, 85, n))], axis=1)
    t = np.stack([rng.normal(size=n), rng.normal(size=n), rng.normal(size=n), (rng.random(n) < 0.3) * 1.0], axis=1)
    mask = rng.integers(0, 4, n).astype(np.uint8)
    return x, t, mask


def test_parameter_count():
    assert M.NPARAMS == 199684


@pytest.mark.parametrize("weights", [(1.0, 1.0, 1.0, 1.0), (0.5, 2.0, 16.0, 0.25)])
def test_gradient_matches_central_differences(weights):
    p = M.init_params(3) * 0.5
    x, t, mask = _batch(16)
    _, g = M.loss_and_grad(p, x, t, mask, weights=weights)
    idx = np.concatenate([rng.integers(0, 1280, 6), rng.integers(1280, 198656, 10), rng.integers(198656, M.NPARAMS, 6)])
    for i in idx:
        e = np.zeros_like(p)
        e[i] = 1e-6
        fd = (M.loss_and_grad(p + e, x, t, mask, weights=weights)[0] -
              M.loss_and_grad(p - e, x, t, mask, weights=weights)[0]) / 2e-6
        assert fd == pytest.approx(g[i], rel=1e-4, abs=1e-9), i


def test_loss_definition_on_a_zero_network():
    # all-zero weights: outputs are exactly the output bias; take it zero
    p = np.zeros(M.NPARAMS)
    x, _, _ = _batch(4)
    t = np.array([[1.0, 2.0, 3.0, 1.0], [0.5, 0.0, -1.0, 0.0], [0.0, 0.0, 0.0, 0.0], [1.0, 1.0, 1.0, 1.0]])
    mask = np.array([3, 1, 2, 0], np.uint8)
    loss, _ = M.loss_and_grad(p, x, t, mask)
    want = np.mean([1 + 4 + 9 + np.log(2), 0.25 + 0 + np.log(2), 0 + np.log(2), np.log(2)])
    assert loss == pytest.approx(want, rel=1e-12)
    # each weight scales its own term: (r, phi, g, capture) = (2, 3, 5, 7)
    loss_w, _ = M.loss_and_grad(p, x, t, mask, weights=(2.0, 3.0, 5.0, 7.0))
    want_w = np.mean([2 * 1 + 3 * 4 + 5 * 9 + 7 * np.log(2), 2 * 0.25 + 0 + 7 * np.log(2), 0 + 7 * np.log(2),
                      7 * np.log(2)])
    assert loss_w == pytest.approx(want_w, rel=1e-12)


def test_bf16_rounding():
    # values exactly representable stay; ties round to even; 1 + 2^-8 -> 1
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.140625, 1e-3])
    r = M.round_bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -6 and r[3] == -2.5 and r[4] == 3.140625
    assert abs(r[5] - 1e-3) < 1e-3 * 2 ** -8
