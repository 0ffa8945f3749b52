"""Pins of the learned-threshold network oracle: convolution by brute force,
hand-written gradients against finite differences, bfloat16 rounding, Adam."""
import numpy as np
import pytest

from oracle import lbmz_learned as N


def _conv_loops(x, w, b, stride):
    n, c, h, wd = x.shape
    o = w.shape[0]
    ho, wo = (h - 1) // stride + 1, (wd - 1) // stride + 1
    y = np.zeros((n, o, ho, wo))
    for bi in range(n):
        for oc in range(o):
            for i in range(ho):
                for j in range(wo):
                    acc = b[oc]
                    for ci in range(c):
                        for di in range(3):
                            for dj in range(3):
                                yy, xx = stride * i + di - 1, stride * j + dj - 1
                                if 0 <= yy < h and 0 <= xx < wd:
                                    acc += w[oc, ci, di, dj] * x[bi, ci, yy, xx]
                    y[bi, oc, i, j] = acc
    return y


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_matches_loops(stride):
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 3, 8, 8))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    assert np.allclose(N.conv3x3(x, w, b, stride), _conv_loops(x, w, b, stride), atol=1e-12)


def test_parameter_count():
    # 12 input channels (9 coefficient maps, 3 level-energy maps), 32 hidden
    shapes = N.param_shapes(12)
    assert sum(int(np.prod(s)) for s in shapes.values()) == 32 * 12 * 9 + 32 + 2 * (32 * 32 * 9 + 32) + 33 * 12
    assert sum(int(np.prod(s)) for s in shapes.values()) == 22380


def test_gradients_against_finite_differences():
    rng = np.random.default_rng(1)
    k = 3
    p = N.init_params(k, seed=2)
    for name in p:                       # non-zero biases so every ReLU branch is exercised
        p[name] = p[name] + 0.05 * rng.normal(size=p[name].shape)
    x = rng.normal(size=(3, N.C_IN, 8, 8))
    t = rng.normal(size=(3, k))
    _, grads = N.loss_and_grads(p, x, t)
    h = 1e-6
    for name in p:
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = N.loss_and_grads(p, x, t)
            flat[idx] = old - h
            lm, _ = N.loss_and_grads(p, x, t)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(grads[name].reshape(-1)[idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (name, idx)


def test_bf16_rounding():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5, 3.0e38, 1e-40], dtype=np.float32)
    got = N.bf16_round(x)
    assert got[0] == 1.0
    assert got[1] == 1.0                     # tie -> even mantissa
    assert got[2] == np.float32(1 + 2 ** -6)  # tie -> even mantissa (up)
    assert got[3] == -2.5
    assert np.all((got.view(np.uint32) & 0xFFFF) == 0)
    rng = np.random.default_rng(3)
    y = rng.normal(size=1000).astype(np.float32)
    r = N.bf16_round(y)
    assert np.all(np.abs(r - y) <= 2.0 ** -8 * np.abs(y))   # half an ulp of 8 significant bits


def test_adam_step_by_hand():
    p = {"w": np.array([1.0])}
    m = {"w": np.zeros(1)}
    v = {"w": np.zeros(1)}
    N.adam_step(p, m, v, {"w": np.array([0.5])}, step=1, lr=0.1)
    # first step: m_hat = g, v_hat = g^2, update = lr * g / (|g| + eps)
    assert np.isclose(p["w"][0], 1.0 - 0.1 * 0.5 / (0.5 + 1e-8))


def test_training_reduces_the_loss():
    rng = np.random.default_rng(4)
    k = 2
    x = rng.normal(size=(64, N.C_IN, 8, 8))
    t = np.stack([x.std(axis=(1, 2, 3)), x[:, 0].mean(axis=(1, 2))], axis=1)
    p = N.init_params(k, seed=5)
    m = {n: np.zeros_like(a) for n, a in p.items()}
    v = {n: np.zeros_like(a) for n, a in p.items()}
    l0, _ = N.loss_and_grads(p, x, t)
    for s in range(1, 61):
        _, g = N.loss_and_grads(p, x, t)
        N.adam_step(p, m, v, g, s, lr=3e-3)
    l1, _ = N.loss_and_grads(p, x, t)
    assert l1 < 0.5 * l0


def test_choose_thresholds():
    pred = np.array([[-9.0, -8.0, -7.0], [-6.0, -5.0, -4.0]])
    eps = N.choose_thresholds(pred, [1e-5, 1e-4, 1e-3], np.array([-7.5, -7.5]), fallback=3e-5)
    assert eps[0] == 1e-4 and eps[1] == 3e-5


def test_coefficient_levels_by_definition():
    s, L = 65, 5
    lev = N.coefficient_levels(s, L)
    for y in range(s):
        for x in range(s):
            def dim(i):
                if i % (1 << L) == 0:
                    return L + 1
                k = 0
                while i % 2 == 0:
                    i //= 2
                    k += 1
                return k + 1
            assert lev[y, x] == min(dim(x), dim(y))
    # an 8 x 8 block holds its stride-8 corner plus coefficients of levels 1..3 only
    blk = lev[8:16, 16:24]
    assert blk[0, 0] > 3 and np.all(blk.reshape(-1)[1:] <= 3)


def test_raw_features_by_brute_force():
    rng = np.random.default_rng(7)
    coef = rng.standard_normal((2, 9, 65, 65))
    raw = N.raw_features(coef, 5)
    assert raw.shape == (2, 36, 8, 8)
    lev = N.coefficient_levels(65, 5)
    for b in range(2):
        for f in (0, 4, 8):
            for j in range(8):
                for i in range(8):
                    assert raw[b, f, j, i] == coef[b, f, 8 * j, 8 * i]
                    for lv in (1, 2, 3):
                        e = 0.0
                        for y in range(8 * j, 8 * j + 8):
                            for x in range(8 * i, 8 * i + 8):
                                if lev[y, x] == lv:
                                    e += coef[b, f, y, x] ** 2
                        assert abs(raw[b, 9 + 3 * f + lv - 1, j, i] - e) <= 1e-12 * max(e, 1.0)
    x = N.input_map(raw)
    assert x.shape == (2, 12, 8, 8)
    assert np.allclose(x[:, :9], np.arcsinh(coef[:, :, 0:64:8, 0:64:8] / 1e-4))
    e2 = sum(raw[:, 9 + 3 * f + 1] for f in range(9))
    assert np.allclose(x[:, 10], np.arcsinh(np.sqrt(e2) / 1e-4))
