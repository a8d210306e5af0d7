"""Pins of the NumPy CNN oracle: the convolution is checked against its
definition written as nested loops, the backward pass against central finite
differences, and Adam against the update of Kingma & Ba written out."""
import numpy as np

from oracle import cnn as C


def conv_loops(x, W, b):
    n, h, w, c = x.shape
    o = W.shape[0]
    out = np.zeros((n, h, w, o))
    for a in range(n):
        for y in range(h):
            for xx in range(w):
                for oc in range(o):
                    s = b[oc]
                    for ky in range(3):
                        for kx in range(3):
                            yy, xz = y + ky - 1, xx + kx - 1
                            if 0 <= yy < h and 0 <= xz < w:
                                for ic in range(c):
                                    s += W[oc, ky, kx, ic] * x[a, yy, xz, ic]
                    out[a, y, xx, oc] = s
    return out


def test_conv_matches_definition():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 5, 4, 3))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    assert np.allclose(C.conv3x3(x, W, b), conv_loops(x, W, b), rtol=1e-13, atol=1e-13)


def test_param_layout():
    assert C.param_count() == 32 * 9 * 16 + 32 + 4 * (32 * 9 * 32 + 32) + 9 * 32 + 1
    p = C.init_params(1)
    assert np.array_equal(C.pack(C.unpack(p)), p.astype(np.float64))


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    p = C.init_params(5).astype(np.float64)
    p += 0.01 * rng.standard_normal(p.size)  # non-zero biases, ReLUs on both sides
    x = rng.standard_normal((2, 6, 7, 16))
    x[..., 5:] = 0.0
    G = rng.standard_normal((2, 6, 7, 1))
    loss = lambda q: float(np.sum(C.forward(q, x)[-1] * G))
    g = C.backward(p, x, G)
    idx = rng.choice(p.size, 60, replace=False)
    for i in idx:
        e = np.zeros_like(p)
        e[i] = 1e-6
        fd = (loss(p + e) - loss(p - e)) / 2e-6
        assert abs(fd - g[i]) <= 1e-5 * max(1.0, abs(fd))
    # a random direction through every parameter
    d = rng.standard_normal(p.size)
    fd = (loss(p + 1e-7 * d) - loss(p - 1e-7 * d)) / 2e-7
    assert abs(fd - g @ d) <= 1e-5 * max(1.0, abs(fd))


def test_adam_matches_published_update():
    rng = np.random.default_rng(9)
    p = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    ref_p, ref_m, ref_v = p.copy(), m.copy(), v.copy()
    for t in range(1, 6):
        g = rng.standard_normal(50)
        p, m, v = C.adam(p, m, v, g, t, 1e-2)
        for i in range(50):  # Algorithm 1, element by element
            ref_m[i] = 0.9 * ref_m[i] + 0.1 * g[i]
            ref_v[i] = 0.999 * ref_v[i] + 0.001 * g[i] ** 2
            mh = ref_m[i] / (1 - 0.9 ** t)
            vh = ref_v[i] / (1 - 0.999 ** t)
            ref_p[i] -= 1e-2 * mh / (np.sqrt(vh) + 1e-8)
    assert np.allclose(p, ref_p, rtol=1e-14, atol=1e-14)


def test_bce_logits_definition_and_gradient():
    """the cross-entropy against its definition from the logistic function
    (moderate logits, where the direct form is accurate), its value at o = 0
    (log 2 whatever the target), its large-logit limits, and its gradient
    against central differences"""
    rng = np.random.default_rng(7)
    o = rng.normal(0.0, 3.0, (2, 5, 6))
    t = (rng.random(o.shape) < 0.3).astype(np.float64)
    t[0, 0, :3] = 0.25  # soft targets too
    w = rng.random(o.shape)
    loss, g = C.bce_logits(o, t, w)
    s = 1.0 / (1.0 + np.exp(-o))
    direct = -(t * np.log(s) + (1.0 - t) * np.log(1.0 - s))
    assert abs(loss - (w * direct).sum() / w.sum()) <= 1e-12 * abs(loss)
    z = np.zeros((1, 2, 2))
    for tv in (0.0, 0.5, 1.0):
        l0, _ = C.bce_logits(z, np.full(z.shape, tv), np.ones(z.shape))
        assert abs(l0 - np.log(2.0)) <= 1e-15
    big = np.array([[[40.0, -40.0]]])
    lb, gb = C.bce_logits(big, np.array([[[1.0, 0.0]]]), np.ones(big.shape))
    assert 0.0 < lb <= 1e-17 and np.abs(gb).max() <= 1e-17
    lw, _ = C.bce_logits(big, np.array([[[0.0, 1.0]]]), np.ones(big.shape))
    assert abs(lw - 40.0) <= 1e-12
    for idx in [(0, 1, 2), (1, 4, 5), (0, 0, 1)]:
        e = 1e-6
        op, om = o.copy(), o.copy()
        op[idx] += e
        om[idx] -= e
        fd = (C.bce_logits(op, t, w)[0] - C.bce_logits(om, t, w)[0]) / (2 * e)
        assert abs(fd - g[idx]) <= 1e-7 * max(abs(g[idx]), 1e-3)
