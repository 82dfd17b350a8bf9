"""The float64 U-Net of oracle/unet_ref.py with bf16 rounding inserted where
the GPU implementation stores bf16 (convolution outputs, batch-norm/ReLU
outputs, pooled and up-sampled maps, bf16 weight copies; the same points in
the backward pass).  Test helper: it bounds how far bf16 storage alone moves
the gradients from float64, which sets the tolerance of the GPU check."""
import torch
import torch.nn.functional as F


class _Round(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x):
        return x.to(torch.bfloat16).to(x.dtype)

    @staticmethod
    def backward(ctx, g):
        return g.to(torch.bfloat16).to(g.dtype)


def forward(P, x, widths, eps=1e-5):
    r = _Round.apply

    def cbr(h, name, skip=None):
        hin = h if skip is None else torch.cat([h, skip], 1)
        z = r(F.conv2d(hin, r(P[name + ".w"]).permute(0, 3, 1, 2), padding=1))
        y = F.batch_norm(z, None, None, P[name + ".gamma"], P[name + ".beta"], training=True,
                         eps=eps)
        return r(F.relu(y))

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


def grads(P, x, labels, widths):
    Pg = {k: v.detach().clone().requires_grad_(True) for k, v in P.items()}
    F.cross_entropy(forward(Pg, x, widths), labels.long()).backward()
    return {k: v.grad for k, v in Pg.items()}
