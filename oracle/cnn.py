"""Plain FP64 NumPy oracle of the warm-start network (TEST INFRASTRUCTURE ONLY).

Six 3x3 convolution layers with zero padding, channels 16 -> 32 -> 32 -> 32 ->
32 -> 32 -> 1 (the first layer's input has 5 feature channels; the other 11
are zero), ReLU after every layer but the last.  Tensors are NHWC; layer l's
weights are [Cout][3][3][Cin] followed by its Cout biases, all layers packed
in one flat FP32 parameter vector.  The optimiser is Adam (Kingma & Ba 2015,
"Adam: A Method for Stochastic Optimization", Algorithm 1).

The mask proposal trains the same network as a per-cell classifier with the
weighted binary cross-entropy of its logits (bce_logits).

Pinned by tests/test_oracle_cnn.py: the convolution against its definition
written as nested loops, the backward pass against finite differences of a
scalar loss, Adam against the published update written out step by step, the
cross-entropy against its definition -t log s(o) - (1 - t) log(1 - s(o)),
its gradient against finite differences.
"""
import numpy as np

CIN = [16, 32, 32, 32, 32, 32]
COUT = [32, 32, 32, 32, 32, 1]
NLAYER = 6


def layer_sizes():
    return [(co * 9 * ci, co) for ci, co in zip(CIN, COUT)]


def param_count():
    return sum(w + b for w, b in layer_sizes())


def unpack(params):
    params = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for (nw, nb), ci, co in zip(layer_sizes(), CIN, COUT):
        W = params[o:o + nw].reshape(co, 3, 3, ci)
        o += nw
        b = params[o:o + nb]
        o += nb
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def conv3x3(x, W, b):
    """out[n, y, x, o] = b[o] + sum_{ky,kx,c} W[o, ky, kx, c] x[n, y+ky-1, x+kx-1, c]"""
    n, h, w, c = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.broadcast_to(b, (n, h, w, W.shape[0])).copy()
    for ky in range(3):
        for kx in range(3):
            out += xp[:, ky:ky + h, kx:kx + w, :] @ W[:, ky, kx, :].T
    return out


def forward(params, x):
    """returns the list of layer outputs (post-ReLU for layers 0..4; the last is linear)"""
    acts = []
    a = np.asarray(x, dtype=np.float64)
    for l, (W, b) in enumerate(unpack(params)):
        z = conv3x3(a, W, b)
        a = np.maximum(z, 0.0) if l < NLAYER - 1 else z
        acts.append(a)
    return acts


def backward(params, x, dout):
    """gradient of sum(out * dout) with respect to the packed parameters"""
    layers = unpack(params)
    acts = forward(params, x)
    ins = [np.asarray(x, dtype=np.float64)] + acts[:-1]
    grads = [None] * NLAYER
    g = np.asarray(dout, dtype=np.float64)
    for l in range(NLAYER - 1, -1, -1):
        W, b = layers[l]
        a_in = ins[l]
        n, h, w, c = a_in.shape
        ap = np.pad(a_in, ((0, 0), (1, 1), (1, 1), (0, 0)))
        dW = np.zeros_like(W)
        for ky in range(3):
            for kx in range(3):
                dW[:, ky, kx, :] = np.einsum("nyxo,nyxc->oc", g, ap[:, ky:ky + h, kx:kx + w, :])
        db = g.sum(axis=(0, 1, 2))
        grads[l] = (dW, db)
        if l > 0:
            gp = np.pad(g, ((0, 0), (1, 1), (1, 1), (0, 0)))
            dx = np.zeros_like(a_in)
            for ky in range(3):
                for kx in range(3):
                    # x[y + ky - 1] feeds out[y]: out[y'] with y' = y - ky + 1
                    dx += gp[:, 2 - ky:2 - ky + h, 2 - kx:2 - kx + w, :] @ W[:, ky, kx, :]
            g = dx * (a_in > 0.0)  # ReLU of the previous layer
    return pack(grads)


def adam(params, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """one Adam step (step counts from 1); returns new (params, m, v)"""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


def init_params(seed):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases"""
    rng = np.random.default_rng(seed)
    out = []
    for ci, co in zip(CIN, COUT):
        W = rng.standard_normal((co, 3, 3, ci)) * np.sqrt(2.0 / (9 * ci))
        out.append((W, np.zeros(co)))
    return pack(out).astype(np.float32)


def bce_logits(out, target, weight):
    """weighted mean binary cross-entropy of logits o against targets t in
    [0, 1]: loss = sum w l / sum w with l = -t log s(o) - (1 - t) log(1 - s(o)),
    s the logistic function, written in the overflow-free form
    l = max(o, 0) - o t + log(1 + exp(-|o|)); gradient w (s(o) - t) / sum w"""
    o = np.asarray(out, dtype=np.float64)
    t = np.asarray(target, dtype=np.float64)
    w = np.asarray(weight, dtype=np.float64)
    sw = w.sum()
    if sw <= 0.0:
        return 0.0, np.zeros_like(o)
    l = np.maximum(o, 0.0) - o * t + np.log1p(np.exp(-np.abs(o)))
    s = 1.0 / (1.0 + np.exp(-o))
    return float((w * l).sum() / sw), w * (s - t) / sw
