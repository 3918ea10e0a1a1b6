"""Plaquette proposal network of the learned sampler (test infrastructure only).

The paper samples with sequential nearest-neighbour exchanges (Sec. II.A
Eq. (9)).  On top of it the learned sampler adds collective moves: flipping
all four spins of a 2x2 plaquette, proposed with a probability a small
convolutional network predicts from the configuration and corrected exactly
by Metropolis-Hastings.  Nothing here is in the paper; the readings are:

* input: the spins as +1 (s = 0, S^z = +1/2) / -1 (s = 1) in one channel;
* network f: conv3x3(1->32), ReLU, conv3x3(32->32), ReLU, conv3x3(32->32),
  ReLU, conv3x3(32->1); zero padding at the open boundary; each convolution
  is out[co,y,x] = b[co] + sum_{ci,ky,kx} W[co,ci,ky,kx] in[ci,y+ky-1,x+kx-1];
* the logit of plaquette (y, x) -- sites (y,x),(y,x+1),(y+1,x),(y+1,x+1) --
  is the output at its top-left site; the plaquette is movable when it holds
  two up and two down spins (the flip then keeps S^z_tot);
* propensity pi = sigmoid(logit); training target a = min(1, R) with R the
  squared amplitude ratio of the flip; loss = mean binary cross-entropy over
  the movable plaquettes of the batch.

Flat parameter layout: W1[32][1][3][3], b1[32], W2[32][32][3][3], b2[32],
W3[32][32][3][3], b3[32], W4[1][32][3][3], b4[1].

Inference in bfloat16 (``forward_bf16``, the sampler's evaluation in its bf16
mode): every weight rounded to bf16, the input (+-1) exact, each layer's
output accumulated in float64 from those, the bias (float32) added, and the
ReLU output rounded to bf16 before the next layer reads it; the last layer's
output is not rounded.  bf16 rounding: the value rounded to float32, then to
the nearest bf16 (8 significant bits), ties to even.

Parity: the convolution is pinned against scipy's correlate in the tests, the
gradient against finite differences of ``loss``, the bf16 rounding against
torch's float32 -> bfloat16 conversion.
"""
import math

import numpy as np

CH = 32
LAYERS = ((1, CH), (CH, CH), (CH, CH), (CH, 1))


def n_params():
    return sum(co * ci * 9 + co for ci, co in LAYERS)


def unpack(theta):
    """[(W [co][ci][3][3], b [co]) per layer] as float64 views of the flat vector."""
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for ci, co in LAYERS:
        W = theta[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = theta[o:o + co]
        o += co
        out.append((W, b))
    assert o == theta.size
    return out


def _patches(x):
    """P[(ci,ky,kx), (y,x)] = x[ci, y+ky-1, x+kx-1], zero outside the lattice."""
    ci, H, Wd = x.shape
    xp = np.zeros((ci, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1] = x
    P = np.empty((ci, 3, 3, H, Wd))
    for ky in range(3):
        for kx in range(3):
            P[:, ky, kx] = xp[:, ky:ky + H, kx:kx + Wd]
    return P.reshape(ci * 9, H * Wd)


def conv3(x, W, b):
    """out[co,y,x] = b[co] + sum W[co,ci,ky,kx] x[ci,y+ky-1,x+kx-1], x = 0 outside the lattice."""
    _, H, Wd = x.shape
    out = W.reshape(W.shape[0], -1) @ _patches(x) + np.asarray(b)[:, None]
    return out.reshape(W.shape[0], H, Wd)


def spins_input(spins, Ly, Lx):
    s = np.asarray(spins).reshape(Ly, Lx)
    return (1.0 - 2.0 * s.astype(np.float64))[None]


def forward(theta, spins, Ly, Lx):
    """Logit map z [Ly][Lx] (plaquette (y,x) reads z[y,x]) and the activations for ``backward``."""
    layers = unpack(theta)
    a = spins_input(spins, Ly, Lx)
    acts, pre = [a], []
    for i, (W, b) in enumerate(layers):
        zpre = conv3(acts[-1], W, b)
        pre.append(zpre)
        acts.append(np.maximum(zpre, 0.0) if i < len(layers) - 1 else zpre)
    return acts[-1][0], (acts, pre)


def bf16(x):
    """x rounded to float32, then to bfloat16 (round to nearest, ties to even), as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(theta, spins, Ly, Lx):
    """Logit map z [Ly][Lx] of the bf16 inference described above."""
    layers = unpack(theta)
    a = spins_input(spins, Ly, Lx)
    for i, (W, b) in enumerate(layers):
        z = conv3(a, bf16(W), np.asarray(b, dtype=np.float32).astype(np.float64))
        a = bf16(np.maximum(z, 0.0)) if i < len(layers) - 1 else z
    return a[0]


def movable(spins, Ly, Lx):
    """[Ly-1][Lx-1] bool: plaquettes with two up and two down spins."""
    s = np.asarray(spins).reshape(Ly, Lx).astype(np.int64)
    tot = s[:-1, :-1] + s[:-1, 1:] + s[1:, :-1] + s[1:, 1:]
    return tot == 2


def sigmoid(z):
    if z >= 0.0:
        return 1.0 / (1.0 + math.exp(-z))
    e = math.exp(z)
    return e / (1.0 + e)


def propensity(theta, spins, Ly, Lx, y, x):
    z, _ = forward(theta, spins, Ly, Lx)
    return sigmoid(float(z[y, x]))


def _bce(z, a):
    # -[a log s + (1-a) log(1-s)], s = sigmoid(z), in a form that does not overflow
    return max(z, 0.0) - z * a + math.log1p(math.exp(-abs(z)))


def loss(theta, configs, targets, Ly, Lx):
    """Mean BCE over the movable plaquettes of every configuration; targets [n][Ly-1][Lx-1]."""
    tot, cnt = 0.0, 0
    for s, a in zip(configs, targets):
        z, _ = forward(theta, s, Ly, Lx)
        m = movable(s, Ly, Lx)
        for y, x in zip(*np.nonzero(m)):
            tot += _bce(float(z[y, x]), float(a[y, x]))
            cnt += 1
    return tot / max(cnt, 1)


def backward(theta, configs, targets, Ly, Lx):
    """d loss / d theta (flat, float64) by reverse-mode differentiation of ``forward``."""
    layers = unpack(theta)
    grads = [(np.zeros_like(W), np.zeros_like(b)) for W, b in layers]
    cnt = sum(int(movable(s, Ly, Lx).sum()) for s in configs)
    for s, a in zip(configs, targets):
        z, (acts, pre) = forward(theta, s, Ly, Lx)
        m = movable(s, Ly, Lx)
        dz = np.zeros((1, Ly, Lx))
        for y, x in zip(*np.nonzero(m)):
            dz[0, y, x] = (sigmoid(float(z[y, x])) - float(a[y, x])) / max(cnt, 1)
        g = dz
        for i in range(len(layers) - 1, -1, -1):
            W, _ = layers[i]
            x_in = acts[i]
            ci, H, Wd = x_in.shape
            xp = np.zeros((ci, H + 2, Wd + 2))
            xp[:, 1:-1, 1:-1] = x_in
            gW, gb = grads[i]
            gb += g.sum(axis=(1, 2))
            gxp = np.zeros_like(xp)
            for ky in range(3):
                for kx in range(3):
                    win = xp[:, ky:ky + H, kx:kx + Wd]
                    gW[:, :, ky, kx] += np.tensordot(g, win, axes=([1, 2], [1, 2]))
                    gxp[:, ky:ky + H, kx:kx + Wd] += np.tensordot(W[:, :, ky, kx], g, axes=([0], [0]))
            if i > 0:
                g = gxp[:, 1:-1, 1:-1] * (pre[i - 1] > 0.0)
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
