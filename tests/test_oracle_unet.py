"""Pins of the oracle's correction network (oracle/unet.py) to things other
than itself: brute-force loops for the convolution, adjoint identities for
pooling and upsampling, central finite differences for every backward step
and for the whole network, the closed form of Adam's first step, and the
degree-one homogeneity of the residual-to-correction map."""
import numpy as np
import pytest

from oracle import unet
from paper_1212_1397_amd.workloads import init_net_params

RNG = np.random.default_rng(7)


def conv_brute(x, W, b):
    C, Z, Y, X = x.shape
    out = np.zeros((W.shape[0], Z, Y, X))
    for o in range(W.shape[0]):
        for z in range(Z):
            for y in range(Y):
                for xx in range(X):
                    acc = b[o]
                    for c in range(C):
                        for dz in (-1, 0, 1):
                            for dy in (-1, 0, 1):
                                for dx in (-1, 0, 1):
                                    zz, yy, x2 = z + dz, y + dy, xx + dx
                                    if 0 <= zz < Z and 0 <= yy < Y and 0 <= x2 < X:
                                        acc += W[o, c, dz + 1, dy + 1, dx + 1] * x[c, zz, yy, x2]
                    out[o, z, y, xx] = acc
    return out


def test_conv_matches_brute_force():
    x = RNG.standard_normal((2, 3, 4, 5))
    W = RNG.standard_normal((3, 2, 3, 3, 3))
    b = RNG.standard_normal(3)
    np.testing.assert_allclose(unet.conv(x, W, b), conv_brute(x, W, b), rtol=1e-12, atol=1e-12)


def test_conv_identity_kernel():
    x = RNG.standard_normal((2, 4, 3, 5))
    W = np.zeros((2, 2, 3, 3, 3))
    W[0, 0, 1, 1, 1] = W[1, 1, 1, 1, 1] = 1.0
    np.testing.assert_array_equal(unet.conv(x, W, np.zeros(2)), x)
    # a pure x-shift kernel moves the data by one and pads with zero
    W = np.zeros((1, 1, 3, 3, 3))
    W[0, 0, 1, 1, 2] = 1.0
    y = unet.conv(x[:1], W, np.zeros(1))
    np.testing.assert_array_equal(y[0, :, :, :-1], x[0, :, :, 1:])
    np.testing.assert_array_equal(y[0, :, :, -1], 0.0)


@pytest.mark.parametrize("shape", [(4, 6, 8), (5, 3, 7), (1, 2, 3)])
def test_pool_and_up_adjoints(shape):
    x = RNG.standard_normal((3,) + shape)
    ps = unet.pooled_shape(shape)
    y = RNG.standard_normal((3,) + ps)
    assert np.isclose(np.vdot(unet.pool(x), y), np.vdot(x, unet.pool_backward(y, shape)))
    assert np.isclose(np.vdot(unet.up(y, shape), x), np.vdot(y, unet.up_backward(x, ps)))


def test_pool_up_values():
    x = np.arange(2 * 3 * 3 * 3, dtype=float).reshape(2, 3, 3, 3)
    p = unet.pool(x)
    assert p.shape == (2, 2, 2, 2)
    # the first cell averages a full 2x2x2 block; the last has a single entry (/8)
    assert p[0, 0, 0, 0] == np.mean(x[0, :2, :2, :2])
    assert p[1, 1, 1, 1] == x[1, 2, 2, 2] / 8.0
    u = unet.up(p, (3, 3, 3))
    assert u.shape == (2, 3, 3, 3) and u[0, 2, 1, 0] == p[0, 1, 0, 0]


def _fd(f, arr, idx, eps=1e-6):
    old = arr[idx]
    arr[idx] = old + eps
    fp = f()
    arr[idx] = old - eps
    fm = f()
    arr[idx] = old
    return (fp - fm) / (2 * eps)


def test_conv_backward_finite_differences():
    x = RNG.standard_normal((2, 3, 4, 3))
    W = RNG.standard_normal((3, 2, 3, 3, 3))
    b = RNG.standard_normal(3)
    g = RNG.standard_normal((3, 3, 4, 3))
    f = lambda: float(np.sum(g * unet.conv(x, W, b)))
    dx, dW, db = unet.conv_backward(x, W, g)
    for idx in [(0, 0, 0, 0), (1, 2, 3, 2), (0, 1, 2, 1)]:
        assert np.isclose(dx[idx], _fd(f, x, idx), rtol=1e-7, atol=1e-8)
    for idx in [(0, 0, 1, 1, 1), (2, 1, 0, 2, 1), (1, 0, 2, 2, 2)]:
        assert np.isclose(dW[idx], _fd(f, W, idx), rtol=1e-7, atol=1e-8)
    for i in range(3):
        assert np.isclose(db[i], _fd(f, b, (i,)), rtol=1e-7, atol=1e-8)


def small_problem(shape=(5, 6, 7), seed=3):
    params = init_net_params([(l[0], l[1], l[2]) for l in unet.LAYERS], seed)
    rng = np.random.default_rng(seed)
    r = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    t = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return params, r, t


def test_network_gradients_finite_differences():
    params, r, t = small_problem()
    k, h = 30.0 + 0.3j, 1.0 / 40
    L, grads = unet.loss_and_grads(params, r, k, h, t)
    f = lambda: unet.loss_and_grads(params, r, k, h, t)[0]
    rng = np.random.default_rng(11)
    for name, _, _, _ in unet.LAYERS:
        W, b = params[name]
        idx = tuple(int(rng.integers(0, s)) for s in W.shape)
        fd = _fd(f, W, idx)
        assert np.isclose(grads[name][0][idx], fd, rtol=1e-5, atol=1e-9), (name, idx)
        j = (int(rng.integers(0, b.shape[0])),)
        assert np.isclose(grads[name][1][j], _fd(f, b, j), rtol=1e-5, atol=1e-9), (name, j)


def test_network_input_gradient_finite_differences():
    params, r, _ = small_problem((4, 5, 3))
    x, _ = unet.features(r, 20.0, 0.05)
    g = np.random.default_rng(5).standard_normal((2,) + r.shape)
    y, cache = unet.forward(params, x)
    _, dx = unet.backward(params, cache, g)
    f = lambda: float(np.sum(g * unet.forward(params, x)[0]))
    for idx in [(0, 0, 0, 0), (1, 3, 4, 2), (2, 1, 2, 1), (0, 2, 0, 2)]:
        assert np.isclose(dx[idx], _fd(f, x, idx), rtol=1e-5, atol=1e-9)


def test_correction_is_homogeneous_degree_one():
    params, r, _ = small_problem()
    c1 = unet.correction(params, r, 40.0, 0.02)
    c2 = unet.correction(params, 3.0 * r, 40.0, 0.02)
    np.testing.assert_allclose(c2, 3.0 * c1, rtol=1e-12, atol=1e-14)


def test_adam_first_step_closed_form():
    # with zero moments, the first Adam step is -lr g / (|g| + eps)
    params = {"a": (np.array([[1.0, -2.0]]), np.array([0.5]))}
    grads = {"a": (np.array([[0.3, -4.0]]), np.array([1e-3]))}
    state = {}
    unet.adam_step(params, grads, state, lr=0.1)
    np.testing.assert_allclose(params["a"][0], [[1.0 - 0.1 * 0.3 / (0.3 + 1e-8), -2.0 + 0.1 * 4.0 / (4.0 + 1e-8)]])
    np.testing.assert_allclose(params["a"][1], [0.5 - 0.1 * 1e-3 / (1e-3 + 1e-8)])


def test_operator_loss_gradients_finite_differences():
    """L_A = |A (c - t)|^2 / |A t|^2 with the Dirichlet operator of eq. (scheme)
    (complex symmetric there, so A^H u = conj(A conj(u)) is exact): parameter
    gradients against central differences, and A = I reduces to the plain loss."""
    import oracle
    shape = (5, 6, 7)
    params, r, t = small_problem(shape)
    prob = oracle.Problem(tuple(reversed(shape)), 1.0 / 8, 30.0 + 0.0j, tuple("DDDDDD"))
    A = lambda v: oracle.apply_A(prob, v)
    k, h = prob.k, prob.h
    L, grads = unet.loss_and_grads_op(params, r, k, h, t, A)
    f = lambda: unet.loss_and_grads_op(params, r, k, h, t, A)[0]
    rng = np.random.default_rng(13)
    for name, _, _, _ in unet.LAYERS:
        W, b = params[name]
        idx = tuple(int(rng.integers(0, s)) for s in W.shape)
        assert np.isclose(grads[name][0][idx], _fd(f, W, idx), rtol=1e-5, atol=1e-9), (name, idx)
        j = (int(rng.integers(0, b.shape[0])),)
        assert np.isclose(grads[name][1][j], _fd(f, b, j), rtol=1e-5, atol=1e-9), (name, j)
    L0, g0 = unet.loss_and_grads(params, r, k, h, t)
    L1, g1 = unet.loss_and_grads_op(params, r, k, h, t, lambda v: v)
    assert np.isclose(L0, L1, rtol=1e-14)
    for name in g0:
        np.testing.assert_allclose(g1[name][0], g0[name][0], rtol=1e-12, atol=1e-15)


def test_round_bf16_matches_torch_conversion():
    # torch's float32 -> bfloat16 conversion (round to nearest, ties to even)
    import torch
    rng = np.random.default_rng(3)
    a = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        [0.0, -0.0, 1.0, -2.5, 3.0e38]]).astype(np.float32)
    # exact ties: the dropped 16 bits are 0x8000, with an even and an odd kept part
    ties = (np.array([0x3F800000, 0x3F810000, 0xBF828000 & 0xFFFF0000], dtype=np.uint32) | 0x8000)
    a = np.concatenate([a, ties.view(np.float32)])
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(unet.round_bf16(a), ref)


def test_storage_points_of_the_network():
    # the storage map is applied at the definition's BF16 storage points: the
    # input, the ten hidden outputs and the two pools forward; the output
    # gradient, eleven input gradients, two upsampling gradients and two
    # skip + pooling sums backward
    params, r, t = small_problem((6, 5, 4))
    seen = []

    def record(a):
        seen.append(np.shape(a))
        return a

    L0, g0 = unet.loss_and_grads(params, r, 20.0, 0.05, t)
    L1, g1 = unet.loss_and_grads(params, r, 20.0, 0.05, t, store=record)
    assert L1 == L0 and all(np.array_equal(g0[k][0], g1[k][0]) for k in g0)
    n1, n2, n3 = (6, 5, 4), (3, 3, 2), (2, 2, 1)
    fwd = [(3,) + n1, (16,) + n1, (16,) + n1, (16,) + n2, (32,) + n2, (32,) + n2, (32,) + n3,
           (64,) + n3, (64,) + n3, (32,) + n2, (32,) + n2, (16,) + n1, (16,) + n1]
    bwd = [(2,) + n1, (16,) + n1, (16,) + n1, (48,) + n1, (32,) + n2, (32,) + n2, (96,) + n2,
           (64,) + n3, (64,) + n3, (32,) + n3, (32,) + n2, (32,) + n2, (16,) + n2, (16,) + n1,
           (16,) + n1, (3,) + n1]
    assert seen == fwd + bwd


def test_bf16_storage_stays_close_to_the_exact_network():
    # storing in BF16 (unit roundoff 2^-9) at 13 forward points perturbs the
    # output by at most about sqrt(13) 2^-9 ~ 0.7% (less where the output is
    # dominated by the biases) and the gradients by about twice that (all
    # ReLUs active: positive biases)
    params, r, t = small_problem((8, 7, 6))
    params = {k: (0.3 * W, np.ones_like(b)) for k, (W, b) in params.items()}
    c0 = unet.correction(params, r, 20.0, 0.05)
    c1 = unet.correction(params, r, 20.0, 0.05, store=unet.round_bf16)
    assert 0.0 < np.linalg.norm(c1 - c0) / np.linalg.norm(c0) < 2e-2
    _, g0 = unet.loss_and_grads(params, r, 20.0, 0.05, t)
    _, g1 = unet.loss_and_grads(params, r, 20.0, 0.05, t, store=unet.round_bf16)
    for k in g0:
        e = np.linalg.norm(g1[k][0] - g0[k][0]) / np.linalg.norm(g0[k][0])
        assert 1e-5 < e < 4e-2, (k, e)
