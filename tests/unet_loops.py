"""A second float64 U-Net forward, written from the definitions with numpy
and explicit loops over kernel taps and output positions (no torch, no
convolution or pooling library routine), to pin the wiring of
oracle/unet_ref.py: ReLU after each batch normalisation, 2x2 max pooling of
the skip map, 2x2 stride-2 up-convolution, the concatenation order (up-sampled
map first, skip map second) and the 1x1 head.  Test helper; shares nothing
with the oracle.

Layouts follow unet_ref: activations NCHW; conv3 weight [Cout, 3, 3, Cin];
up2 weight [2, 2, Cin, Cout]; conv1 weight [Cout, Cin]."""
import numpy as np


def conv3(x, w):
    """3x3 convolution, zero padding 1: y[n,o,i,j] = sum_{c,r,s} x[n,c,i+r-1,j+s-1] w[o,r,s,c]."""
    N, C, H, W = x.shape
    O = w.shape[0]
    y = np.zeros((N, O, H, W))
    for n in range(N):
        for o in range(O):
            for i in range(H):
                for j in range(W):
                    acc = 0.0
                    for r in range(3):
                        for s in range(3):
                            ii, jj = i + r - 1, j + s - 1
                            if 0 <= ii < H and 0 <= jj < W:
                                acc += float(np.dot(x[n, :, ii, jj], w[o, r, s, :]))
                    y[n, o, i, j] = acc
    return y


def batch_norm(y, gamma, beta, eps, mean=None, var=None):
    """Per channel (z - mean) / sqrt(var + eps) * gamma + beta; batch mean and
    biased variance over (n, i, j) unless running mean and var are given."""
    N, C, H, W = y.shape
    out = np.empty_like(y)
    for c in range(C):
        v = y[:, c].reshape(-1)
        m = v.sum() / v.size if mean is None else mean[c]
        s2 = ((v - v.sum() / v.size) ** 2).sum() / v.size if var is None else var[c]
        out[:, c] = (y[:, c] - m) / np.sqrt(s2 + eps) * gamma[c] + beta[c]
    return out


def relu(y):
    return np.where(y > 0, y, 0.0)


def maxpool2(x):
    N, C, H, W = x.shape
    y = np.empty((N, C, H // 2, W // 2))
    for i in range(H // 2):
        for j in range(W // 2):
            y[:, :, i, j] = np.maximum(np.maximum(x[:, :, 2 * i, 2 * j], x[:, :, 2 * i, 2 * j + 1]),
                                       np.maximum(x[:, :, 2 * i + 1, 2 * j], x[:, :, 2 * i + 1, 2 * j + 1]))
    return y


def upconv2(x, w, b):
    """y[n, o, 2i+r, 2j+s] = b[o] + sum_c x[n, c, i, j] w[r, s, c, o]."""
    N, C, H, W = x.shape
    O = w.shape[3]
    y = np.empty((N, O, 2 * H, 2 * W))
    for i in range(H):
        for j in range(W):
            for r in range(2):
                for s in range(2):
                    y[:, :, 2 * i + r, 2 * j + s] = x[:, :, i, j] @ w[r, s] + b
    return y


def head(x, w, b):
    N, C, H, W = x.shape
    y = np.empty((N, w.shape[0], H, W))
    for k in range(w.shape[0]):
        y[:, k] = np.tensordot(w[k], x, axes=([0], [1])) + b[k]
    return y


def forward(P, x, widths, eps=1e-5, running=None):
    """Logits for x [N, 3, H, W]; P maps names to numpy arrays.  `running`
    (name -> (mean, var)) switches batch normalisation to running statistics."""
    def cbr(h, name):
        z = conv3(h, P[name + ".w"])
        m, v = running[name] if running is not None else (None, None)
        return relu(batch_norm(z, P[name + ".gamma"], P[name + ".beta"], eps, m, v))

    L = len(widths)
    skips, h = [], x
    for i in range(L):
        name = f"enc{i}" if i < L - 1 else "mid"
        h = cbr(cbr(h, name + ".conv0"), name + ".conv1")
        if i < L - 1:
            skips.append(h)
            h = maxpool2(h)
    for i in reversed(range(L - 1)):
        up = upconv2(h, P[f"dec{i}.up.w"], P[f"dec{i}.up.b"])
        h = np.concatenate([up, skips[i]], axis=1)
        h = cbr(cbr(h, f"dec{i}.conv0"), f"dec{i}.conv1")
    return head(h, P["head.w"], P["head.b"])
