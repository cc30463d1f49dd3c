"""Pins for the oracle's cost-model network (CPU only)."""
import numpy as np

from oracle import mlp as M
from paper_1407_4859_amd import synth

SIZES = [16, 64, 64, 64, 1]


def _u(seed, n, stream=0):
    return synth.splitmix64(seed, stream, 0, n).astype(np.float64) / 2.0 ** 63 - 1.0


def _data(seed, B=32, d=16):
    x = _u(seed, B * d, 1).reshape(B, d)
    y = _u(seed, B, 2)
    return x, y


def test_gradients_match_central_differences():
    params = M.init_params(SIZES, _u(1, 16 * 64 + 64 * 64 * 2 + 64))
    for i in range(1, len(params), 2):
        params[i] = 0.1 * _u(20 + i, params[i].size)
    x, y = _data(2)
    grads = M.backward(params, x, y)
    h = 1e-6
    for pi, p in enumerate(params):
        flat = p.reshape(-1)
        g = grads[pi].reshape(-1)
        for j in np.linspace(0, flat.size - 1, 7).astype(int):
            old = flat[j]
            flat[j] = old + h
            lp = M.loss(params, x, y)
            flat[j] = old - h
            lm = M.loss(params, x, y)
            flat[j] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(fd)), (pi, j, fd, g[j])


def test_linear_model_trains_to_least_squares():
    x, y = _data(3, B=256)
    params = M.init_params([16, 1], _u(4, 16))
    opt = M.Adam(params, lr=1e-2)
    for _ in range(6000):
        opt.step(params, M.backward(params, x, y))
    A = np.hstack([x, np.ones((len(x), 1))])
    sol = np.linalg.lstsq(A, y, rcond=None)[0]
    assert np.allclose(params[0].reshape(-1), sol[:16], atol=1e-5)
    assert np.allclose(params[1], sol[16:], atol=1e-5)


def test_adam_first_step_is_lr_times_sign():
    p = [np.array([[3.0, -2.0]]), np.array([0.5])]
    g = [np.array([[0.2, -7.0]]), np.array([-1e-3])]
    opt = M.Adam(p, lr=1e-3)
    before = [q.copy() for q in p]
    opt.step(p, g)
    step = np.concatenate([(b - a).reshape(-1) for a, b in zip(p, before)])
    assert np.allclose(step, 1e-3 * np.sign(np.concatenate([q.reshape(-1) for q in g])),
                       rtol=1e-4)


def test_relu_zero_region_has_zero_gradient():
    params = M.init_params([2, 3, 1], _u(5, 9))
    params[0][:] = -1.0
    params[1][:] = -1.0       # every hidden unit dead for positive inputs
    x = np.abs(_data(6, B=8, d=2)[0])
    grads = M.backward(params, x, np.ones(8))
    assert not grads[0].any() and not grads[1].any() and not grads[2].any()
