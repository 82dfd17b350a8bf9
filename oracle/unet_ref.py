"""U-Net oracle in float64 on the CPU -- TEST INFRASTRUCTURE ONLY.

The network the paper trains on the auto-labels (section III-C, "U-Net Model
for Sea-Ice Classification"): a contracting path of two 3x3 convolutions
with ReLU per level followed by 2x2 max pooling (stride 2), a bottleneck,
an expanding path of 2x2 up-convolutions that halve the channels,
concatenation with the skip feature map and two 3x3 convolutions with ReLU,
and a final 1x1 convolution to the 3 classes, trained with categorical
cross-entropy (section III-C, "U-Net Training").

The variant computed here: level widths as given (e.g. 32, 64, 128, 256),
batch normalisation after every 3x3 convolution (batch statistics in
training, running statistics in inference), "same" padding so no cropping,
convolutions without bias (batch normalisation absorbs it), 3 input bands.
The GPU implementation in ``paper_2403_13135_amd/unet.py`` computes the same
function with its own kernels.  Written with plain ``torch.nn.functional``
calls in float64, NCHW; gradients come from autograd and are pinned by finite
differences in the tests, the wiring by a second forward written with loops
(tests/unet_loops.py).
"""
import math
from typing import Dict, Sequence

import torch
import torch.nn.functional as F

BN_EPS = 1e-5


def layer_specs(widths: Sequence[int], in_ch: int = 3, n_classes: int = 3):
    """Ordered parameter specs of the U-Net with level widths ``widths``
    (e.g. 32, 64, 128, 256: three encoder levels and a bottleneck)."""
    specs = []
    c = in_ch
    for i, w in enumerate(widths):
        name = f"enc{i}" if i < len(widths) - 1 else "mid"
        specs.append((f"{name}.conv0", "conv3", c, w))
        specs.append((f"{name}.conv1", "conv3", w, w))
        c = w
    for i in reversed(range(len(widths) - 1)):
        w = widths[i]
        specs.append((f"dec{i}.up", "up2", c, w))
        specs.append((f"dec{i}.conv0", "conv3", 2 * w, w))
        specs.append((f"dec{i}.conv1", "conv3", w, w))
        c = w
    specs.append(("head", "conv1", c, n_classes))
    return specs


def init_params(widths: Sequence[int], seed: int = 0, dtype=torch.float64) -> Dict[str, torch.Tensor]:
    """He-normal weights (std sqrt(2/fan_in)), zero biases, BN gamma 1, beta 0.
    Layouts: conv3 weight [Cout, 3, 3, Cin]; up2 weight [2, 2, Cin, Cout] and
    bias [Cout]; conv1 weight [Cout, Cin] and bias [Cout]; BN gamma/beta [C]."""
    g = torch.Generator().manual_seed(seed)
    P = {}
    for name, kind, cin, cout in layer_specs(widths):
        if kind == "conv3":
            P[name + ".w"] = torch.randn(cout, 3, 3, cin, generator=g, dtype=dtype) * math.sqrt(2.0 / (9 * cin))
            P[name + ".gamma"] = torch.ones(cout, dtype=dtype)
            P[name + ".beta"] = torch.zeros(cout, dtype=dtype)
        elif kind == "up2":
            P[name + ".w"] = torch.randn(2, 2, cin, cout, generator=g, dtype=dtype) * math.sqrt(2.0 / cin)
            P[name + ".b"] = torch.zeros(cout, dtype=dtype)
        else:
            P[name + ".w"] = torch.randn(cout, cin, generator=g, dtype=dtype) * math.sqrt(2.0 / cin)
            P[name + ".b"] = torch.zeros(cout, dtype=dtype)
    return P


def _conv3_bn_relu(x, P, name, running=None):
    w = P[name + ".w"].permute(0, 3, 1, 2)  # [Cout, Cin, 3, 3]
    y = F.conv2d(x, w, padding=1)
    if running is None:
        y = F.batch_norm(y, None, None, P[name + ".gamma"], P[name + ".beta"], training=True,
                         eps=BN_EPS)
    else:
        mean, var = running[name]
        y = F.batch_norm(y, mean, var, P[name + ".gamma"], P[name + ".beta"], training=False,
                         eps=BN_EPS)
    return F.relu(y)


def forward(P: Dict[str, torch.Tensor], x: torch.Tensor, widths: Sequence[int],
            running=None) -> torch.Tensor:
    """Logits [N, 3, H, W] for input x [N, 3, H, W].  Training mode (batch
    statistics in every batch normalisation) unless `running` maps each
    convolution's name to its (running mean, running variance), the inference
    form."""
    skips = []
    h = x
    L = len(widths)
    for i in range(L):
        name = f"enc{i}" if i < L - 1 else "mid"
        h = _conv3_bn_relu(h, P, name + ".conv0", running)
        h = _conv3_bn_relu(h, P, name + ".conv1", running)
        if i < L - 1:
            skips.append(h)
            h = F.max_pool2d(h, 2)
    for i in reversed(range(L - 1)):
        w = P[f"dec{i}.up.w"].permute(2, 3, 0, 1)  # [Cin, Cout, 2, 2]
        h = F.conv_transpose2d(h, w, P[f"dec{i}.up.b"], stride=2)
        h = torch.cat([h, skips[i]], dim=1)
        h = _conv3_bn_relu(h, P, f"dec{i}.conv0", running)
        h = _conv3_bn_relu(h, P, f"dec{i}.conv1", running)
    return F.conv2d(h, P["head.w"][:, :, None, None], P["head.b"])


def loss(logits: torch.Tensor, labels: torch.Tensor) -> torch.Tensor:
    """Categorical cross-entropy, mean over pixels (labels [N, H, W] in 0..2)."""
    return F.cross_entropy(logits, labels.long())


def loss_and_grads(P, x, labels, widths):
    """(loss, logits, {name: dloss/dparam}, dloss/dx) in float64."""
    Pg = {k: v.detach().clone().requires_grad_(True) for k, v in P.items()}
    xg = x.detach().clone().requires_grad_(True)
    logits = forward(Pg, xg, widths)
    l = loss(logits, labels)
    l.backward()
    return l.detach(), logits.detach(), {k: v.grad for k, v in Pg.items()}, xg.grad
