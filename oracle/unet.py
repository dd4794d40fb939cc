"""Correction network of the learned preconditioner, in FP64.

TEST INFRASTRUCTURE ONLY: part of the FP64 CPU oracle.  Parity target for
the GPU network (forward pass, and the weight and input gradients of its
training step).

The network is not in the paper; it is the learned correction to the
preconditioner A_p^{-1} of eq. (3DAP) (Section 3.3) used inside flexible
GMRES.  Definition (the one the GPU path implements):

* Arrays are channels-first, (C, n'z, n'y, n'x), like the oracle's unknown
  vectors with a leading channel axis.
* conv(x; W, b): zero-padded 3x3x3 cross-correlation,
    out[o, p] = b[o] + sum_{c, t} W[o, c, t] x[c, p + t],  t in {-1,0,1}^3,
  with W of shape (Cout, Cin, 3, 3, 3) indexed (dz, dy, dx).
* pool: 2x2x2 average, output extent ceil(n/2) per axis; entries past the
  input's end count as zero (the divisor is always 8).
* up: nearest-neighbour upsampling to a given extent, out[p] = in[p // 2].
* Three levels, channels 16 / 32 / 64; ReLU after every convolution but the
  last; skip connections by channel concatenation ([upsampled, skip]):
      s1 = R(e1b(R(e1a(x))))                 3 -> 16 -> 16
      s2 = R(e2b(R(e2a(pool s1))))          16 -> 32 -> 32
      b3 = R(b3b(R(b3a(pool s2))))          32 -> 64 -> 64
      d2 = R(d2b(R(d2a([up b3, s2]))))      96 -> 32 -> 32
      d1 = R(d1b(R(d1a([up d2, s1]))))      48 -> 16 -> 16
      y  = out(d1)                          16 -> 2
* Features of a residual r: s = sqrt(mean |r|^2); x = [Re r / s, Im r / s,
  Re(k) h]; the correction is c = s (y_0 + i y_1).  (The scaling makes the
  map r -> c positively homogeneous of degree one.)
* Loss of a training pair (r, target t): L = sum |c - t|^2 / sum |t|^2.
* Operator-weighted loss with a linear operator A (the h^2-scaled operator of
  eq. (scheme) on the pair's grid): L_A = sum |A (c - t)|^2 / sum |A t|^2, the
  quantity a correction must lower to pass the solver's judge (t = e - A_p^{-1} r
  gives A t = r - A A_p^{-1} r).  Its gradient uses A^H u = conj(A conj(u)),
  exact when A is complex symmetric (Dirichlet faces); with Neumann or
  Sommerfeld faces A is not symmetric in its closure rows and this is the
  training gradient by definition (the GPU computes the same).

* Storage precision.  The device stores activations and gradients in BF16
  (the network's definition: BF16 activations, FP32 accumulation); the
  functions below take an optional `store` map applied exactly where a value
  is stored: the input features, every hidden layer's output after its ReLU,
  the pooled values (forward); the output gradient, every convolution's input
  gradient, the upsampling gradient and the sum of a skip gradient with the
  pooling gradient (backward).  The final layer's output stays unrounded.
  store=None is the exact FP64 network; store=round_bf16 takes every ReLU
  decision on the values the device holds (both sides then decide in the
  kernel's precision), so the two differ only by accumulation order.

Gradients are written out by hand (the adjoint of each step in reverse
order); the tests pin them to central finite differences.
"""
from __future__ import annotations

import numpy as np

# (name, Cin, Cout, relu)
LAYERS = [
    ("e1a", 3, 16, True), ("e1b", 16, 16, True),
    ("e2a", 16, 32, True), ("e2b", 32, 32, True),
    ("b3a", 32, 64, True), ("b3b", 64, 64, True),
    ("d2a", 96, 32, True), ("d2b", 32, 32, True),
    ("d1a", 48, 16, True), ("d1b", 16, 16, True),
    ("out", 16, 2, False),
]


def _taps():
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                yield dz, dy, dx


def conv(x, W, b):
    """Zero-padded 3x3x3 cross-correlation with bias."""
    C, Z, Y, X = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1)))
    out = np.empty((W.shape[0], Z, Y, X))
    out[...] = b[:, None, None, None]
    for dz, dy, dx in _taps():
        # out[o, p] += sum_c W[o, c, t] x[c, p + t]  (contraction over the channel axis)
        out += np.tensordot(W[:, :, dz, dy, dx], xp[:, dz:dz + Z, dy:dy + Y, dx:dx + X], axes=(1, 0))
    return out


def conv_backward(x, W, dout):
    """Gradients of conv: (dx, dW, db) for the upstream gradient dout."""
    C, Z, Y, X = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1)))
    dxp = np.zeros_like(xp)
    dW = np.empty_like(W)
    for dz, dy, dx in _taps():
        sl = (slice(None), slice(dz, dz + Z), slice(dy, dy + Y), slice(dx, dx + X))
        # dW[o, c, t] = sum_p dout[o, p] x[c, p + t];  dx[c, p + t] += sum_o W[o, c, t] dout[o, p]
        dW[:, :, dz, dy, dx] = np.tensordot(dout, xp[sl], axes=([1, 2, 3], [1, 2, 3]))
        dxp[sl] += np.tensordot(W[:, :, dz, dy, dx], dout, axes=(0, 0))
    return dxp[:, 1:-1, 1:-1, 1:-1], dW, dout.sum(axis=(1, 2, 3))


def pooled_shape(shape):
    return tuple((n + 1) // 2 for n in shape)


def pool(x):
    C, Z, Y, X = x.shape
    Zo, Yo, Xo = pooled_shape((Z, Y, X))
    xp = np.zeros((C, 2 * Zo, 2 * Yo, 2 * Xo))
    xp[:, :Z, :Y, :X] = x
    return xp.reshape(C, Zo, 2, Yo, 2, Xo, 2).sum(axis=(2, 4, 6)) / 8.0


def pool_backward(dout, shape):
    C = dout.shape[0]
    Z, Y, X = shape
    d = np.repeat(np.repeat(np.repeat(dout, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0
    return d[:, :Z, :Y, :X].copy()


def up(x, shape):
    Z, Y, X = shape
    return x[:, np.arange(Z) // 2][:, :, np.arange(Y) // 2][:, :, :, np.arange(X) // 2]


def up_backward(dout, shape):
    C, Z, Y, X = dout.shape
    Zi, Yi, Xi = shape
    d = np.zeros((C, 2 * Zi, 2 * Yi, 2 * Xi))
    d[:, :Z, :Y, :X] = dout
    return d.reshape(C, Zi, 2, Yi, 2, Xi, 2).sum(axis=(2, 4, 6))


def relu(x):
    return np.maximum(x, 0.0)


def round_bf16(a):
    """Nearest BF16 value of each element (via binary32; BF16 keeps the sign,
    the 8 exponent bits and the top 7 fraction bits of a binary32 number;
    ties round to an even last kept bit), as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _identity(a):
    return a


def features(r, k, h):
    """Network input of a complex residual r (n'z, n'y, n'x) and its scale s."""
    s = float(np.sqrt(np.mean(np.abs(r) ** 2)))
    x = np.empty((3,) + r.shape)
    x[0] = r.real / s
    x[1] = r.imag / s
    x[2] = complex(k).real * h
    return x, s


def forward(params, x, store=None):
    """Network output y (2, ...) and the saved activations for backward
    (store: the storage rounding, see the module docstring)."""
    st = store or _identity
    x = st(x)
    cache = {"x": x}

    def layer(name, inp):
        W, b = params[name]
        z = conv(inp, W, b)
        cache[name] = (inp, z)
        return z

    n1 = x.shape[1:]
    n2 = pooled_shape(n1)
    a = st(relu(layer("e1a", x)))
    s1 = st(relu(layer("e1b", a)))
    a = st(relu(layer("e2a", st(pool(s1)))))
    s2 = st(relu(layer("e2b", a)))
    a = st(relu(layer("b3a", st(pool(s2)))))
    b3 = st(relu(layer("b3b", a)))
    a = st(relu(layer("d2a", np.concatenate([up(b3, n2), s2]))))
    d2 = st(relu(layer("d2b", a)))
    a = st(relu(layer("d1a", np.concatenate([up(d2, n1), s1]))))
    d1 = st(relu(layer("d1b", a)))
    y = layer("out", d1)
    cache["shapes"] = (n1, n2, pooled_shape(n2))
    return y, cache


def backward(params, cache, dy, store=None):
    """Parameter gradients {name: (dW, db)} and the input gradient, for dL/dy."""
    st = store or _identity
    grads = {}
    n1, n2, n3 = cache["shapes"]

    def back(name, dz):
        inp, z = cache[name]
        if dict((l[0], l[3]) for l in LAYERS)[name]:
            dz = dz * (z > 0.0)
        dinp, dW, db = conv_backward(inp, params[name][0], dz)
        grads[name] = (dW, db)
        return st(dinp)

    d = back("out", st(dy))
    d = back("d1b", d)
    d = back("d1a", d)                    # 48 channels: [up d2 (32), s1 (16)]
    ds1 = d[32:]
    d = back("d2b", st(up_backward(d[:32], n2)))
    d = back("d2a", d)                    # 96 channels: [up b3 (64), s2 (32)]
    ds2 = d[64:]
    d = back("b3b", st(up_backward(d[:64], n3)))
    d = back("b3a", d)
    d = back("e2b", st(ds2 + pool_backward(d, n2)))
    d = back("e2a", d)
    d = back("e1b", st(ds1 + pool_backward(d, n1)))
    dx = back("e1a", d)
    return grads, dx


def correction(params, r, k, h, store=None):
    """c = s (y_0 + i y_1) for the residual r."""
    x, s = features(r, k, h)
    y, _ = forward(params, x, store)
    return s * (y[0] + 1j * y[1])


def loss_and_grads(params, r, k, h, target, store=None):
    """Relative squared error of the correction and its parameter gradients."""
    x, s = features(r, k, h)
    y, cache = forward(params, x, store)
    c = s * (y[0] + 1j * y[1])
    den = float(np.sum(np.abs(target) ** 2))
    diff = c - target
    L = float(np.sum(np.abs(diff) ** 2)) / den
    dy = np.stack([2.0 * s * diff.real, 2.0 * s * diff.imag]) / den
    grads, _ = backward(params, cache, dy, store)
    return L, grads


def loss_and_grads_op(params, r, k, h, target, apply_A, store=None):
    """Operator-weighted relative error L_A = |A (c - t)|^2 / |A t|^2 and its
    parameter gradients (apply_A: vector -> A vector, complex symmetric A)."""
    x, s = features(r, k, h)
    y, cache = forward(params, x, store)
    c = s * (y[0] + 1j * y[1])
    At = apply_A(target)
    den = float(np.sum(np.abs(At) ** 2))
    u = apply_A(c - target)
    L = float(np.sum(np.abs(u) ** 2)) / den
    g = np.conj(apply_A(np.conj(u)))          # A^H u for complex symmetric A
    dy = np.stack([2.0 * s * g.real, 2.0 * s * g.imag]) / den
    grads, _ = backward(params, cache, dy, store)
    return L, grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) of every weight and bias, in place."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for name, (dW, db) in grads.items():
        for idx, g in ((0, dW), (1, db)):
            key = (name, idx)
            m, v = state.get(key, (np.zeros_like(g), np.zeros_like(g)))
            m = beta1 * m + (1 - beta1) * g
            v = beta2 * v + (1 - beta2) * g * g
            state[key] = (m, v)
            mhat = m / (1 - beta1 ** t)
            vhat = v / (1 - beta2 ** t)
            params[name][idx][...] -= lr * mhat / (np.sqrt(vhat) + eps)
