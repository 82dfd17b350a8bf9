"""The float64 U-Net of oracle/unet_ref.py with bf16 rounding inserted
exactly where the GPU implementation stores bf16, and float32 where it keeps
float32: convolution outputs, batch-norm/ReLU outputs, pooled and up-sampled
maps and bf16 weight copies in the forward pass; in the backward pass the
gradients of activations (batch-norm input, layer outputs, both halves of a
concatenation), while weight, bias and batch-norm parameter gradients stay
unrounded.  Batch statistics come, as on the GPU, from the convolution's sums
before its bf16 rounding, and the (mean, rstd) pair is kept in float32.  Test
helper: it shows how far bf16 storage alone moves results from float64, and
the GPU must track it closely."""
import torch
import torch.nn.functional as F


def _bf16(x):
    return x.to(torch.bfloat16).to(x.dtype)


def _f32(x):
    return x.to(torch.float32).to(x.dtype)


class _Round(torch.autograd.Function):
    """bf16 storage of an activation: value and incoming gradient rounded."""

    @staticmethod
    def forward(ctx, x):
        return _bf16(x)

    @staticmethod
    def backward(ctx, g):
        return _bf16(g)


class _RoundValue(torch.autograd.Function):
    """bf16 copy of a float32 master weight: gradient passed on unrounded."""

    @staticmethod
    def forward(ctx, x):
        return _bf16(x)

    @staticmethod
    def backward(ctx, g):
        return g


class _RoundGrad(torch.autograd.Function):
    """A bf16 gradient buffer for one consumer of a tensor (e.g. the skip half
    of a concatenation), before the gradients of its consumers are added."""

    @staticmethod
    def forward(ctx, x):
        return x.clone()

    @staticmethod
    def backward(ctx, g):
        return _bf16(g)


class _BNReLUTrain(torch.autograd.Function):
    """Batch norm with batch statistics + ReLU as the GPU computes it: the
    statistics from the unrounded convolution output zf, normalisation of its
    bf16 copy z, the standard batch-norm gradient evaluated at z, rounded to
    bf16 (the convolution's output gradient)."""

    @staticmethod
    def forward(ctx, zf, gamma, beta, eps):
        n = zf.numel() // zf.shape[1]
        dims = (0, 2, 3)
        mean = zf.sum(dims) / n
        var = ((zf * zf).sum(dims) / n - mean * mean).clamp(min=0)
        rstd = _f32(1.0 / torch.sqrt(var + float(torch.tensor(eps, dtype=torch.float32))))
        mean = _f32(mean)
        z = _bf16(zf)
        zh = (z - mean.view(1, -1, 1, 1)) * rstd.view(1, -1, 1, 1)
        y = zh * gamma.view(1, -1, 1, 1) + beta.view(1, -1, 1, 1)
        ctx.save_for_backward(zh, y, gamma, rstd)
        ctx.n = n
        return F.relu(y)

    @staticmethod
    def backward(ctx, dout):
        zh, y, gamma, rstd = ctx.saved_tensors
        dims = (0, 2, 3)
        d = torch.where(y > 0, dout, torch.zeros((), dtype=dout.dtype))
        s1, s2 = d.sum(dims), (d * zh).sum(dims)
        k = (gamma * rstd).view(1, -1, 1, 1)
        dz = k * (d - (s1.view(1, -1, 1, 1) + zh * s2.view(1, -1, 1, 1)) / ctx.n)
        return _bf16(dz), s2, s1, None


def forward(P, x, widths, eps=1e-5):
    r, rv, rg = _Round.apply, _RoundValue.apply, _RoundGrad.apply

    def cbr(h, name, skip=None):
        hin = h if skip is None else torch.cat([h, rg(skip)], 1)
        zf = F.conv2d(hin, rv(P[name + ".w"]).permute(0, 3, 1, 2), padding=1)
        return r(_BNReLUTrain.apply(zf, P[name + ".gamma"], P[name + ".beta"], eps))

    skips, h, L = [], x, len(widths)
    for i in range(L):
        name = f"enc{i}" if i < L - 1 else "mid"
        h = cbr(cbr(h, name + ".conv0"), name + ".conv1")
        if i < L - 1:
            skips.append(h)
            h = r(F.max_pool2d(h, 2))
    for i in reversed(range(L - 1)):
        w = rv(P[f"dec{i}.up.w"]).permute(2, 3, 0, 1)
        h = r(F.conv_transpose2d(h, w, P[f"dec{i}.up.b"], stride=2))
        h = cbr(cbr(h, f"dec{i}.conv0", skips[i]), f"dec{i}.conv1")
    return F.conv2d(h, P["head.w"][:, :, None, None], P["head.b"])


def grads(P, x, labels, widths):
    Pg = {k: v.detach().clone().requires_grad_(True) for k, v in P.items()}
    F.cross_entropy(forward(Pg, x, widths), labels.long()).backward()
    return {k: v.grad for k, v in Pg.items()}


def forward_infer(P, x, widths, running, eps=1e-5):
    """Inference with running statistics as the GPU runs it: per layer the
    fp32 scale = gamma / sqrt(running_var + eps) and shift = beta -
    running_mean * scale, the convolution's sum, affine and ReLU rounded to
    bf16 once (no bf16 rounding of the convolution output), bf16 pooled and
    up-sampled maps, fp32 head.  P and running hold the GPU's fp32 values as
    float64 tensors."""
    r = _Round.apply

    def f32(t):
        return t.to(torch.float32).to(torch.float64)

    def cbr(h, name, skip=None):
        hin = h if skip is None else torch.cat([h, skip], 1)
        z = F.conv2d(hin, r(P[name + ".w"]).permute(0, 3, 1, 2), padding=1)
        rm, rv = running[name]
        scale = f32(f32(P[name + ".gamma"]) / f32(torch.sqrt(f32(f32(rv) + f32(torch.tensor(eps))))))
        shift = f32(f32(P[name + ".beta"]) - f32(f32(rm) * scale))
        return r(F.relu(z * scale.view(1, -1, 1, 1) + shift.view(1, -1, 1, 1)))

    skips, h, L = [], x, len(widths)
    for i in range(L):
        name = f"enc{i}" if i < L - 1 else "mid"
        h = cbr(cbr(h, name + ".conv0"), name + ".conv1")
        if i < L - 1:
            skips.append(h)
            h = r(F.max_pool2d(h, 2))
    for i in reversed(range(L - 1)):
        w = r(P[f"dec{i}.up.w"]).permute(2, 3, 0, 1)
        h = r(F.conv_transpose2d(h, w, P[f"dec{i}.up.b"], stride=2))
        h = cbr(cbr(h, f"dec{i}.conv0", skips[i]), f"dec{i}.conv1")
    return F.conv2d(h, P["head.w"][:, :, None, None], P["head.b"])
