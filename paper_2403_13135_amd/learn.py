"""Training the U-Net on the GPU auto-labels and serving it with the labeller
as fallback (arXiv 2403.13135, section III-C and Fig. "Workflow for Sea Ice
Classification employing cloud-shadow filter and U-net model Inferencing").

* Training data: seeded synthetic scenes (``synth``), auto-labelled by the
  GPU labeller (``sil.label``, filter on), cut into 256 x 256 chips as the
  paper cuts its 2048 x 2048 scenes into 64 chips of 256 x 256.
* The trained network's class maps are compared with the labeller's (pixel
  disagreement) and, since the synthetic scenes carry their class truth, both
  are scored against that truth; so is the unfiltered threshold labelling.
* Serving with fallback: a scene's U-Net class map is used unless it
  disagrees with the labeller on more than a set fraction of pixels, in
  which case the labeller's map is returned.
"""
import time
from dataclasses import dataclass
from typing import List

import numpy as np
import torch

from . import sil, unet

CHIP = 256


def unet_flops_per_image(widths, H=CHIP, W=CHIP) -> float:
    """2 x multiply-adds of one forward pass at H x W: 3x3 convolutions at
    their level's resolution and 2x2 up-convolutions from the level below (the
    1x1 head and element-wise work are not counted)."""
    L = len(widths)
    macs = 0
    for name, kind, cin, cout in unet.layer_specs(widths, in_ch=3):
        if kind == "conv1":
            continue
        # level index of the layer: "enc<i>", "dec<i>", or the bottleneck
        lvl = L - 1 if name.startswith("mid") else int(name.split(".")[0][3:])
        hh, ww = H >> lvl, W >> lvl
        if kind == "conv3":
            macs += 9 * cin * cout * hh * ww
        elif kind == "up2":
            macs += 4 * cin * cout * (hh // 2) * (ww // 2)
    return 2.0 * macs


@dataclass
class Scene:
    scene: torch.Tensor    # [3, H, W] int16 (uint16 reflectance bits), device
    truth: torch.Tensor    # [H, W] uint8, device
    labels: torch.Tensor   # [H, W] uint8 auto-labels (filter on), device
    labels0: torch.Tensor  # [H, W] uint8 thresholds only, device


def make_scenes(n: int, size: int, seed0: int, device="cuda") -> List[Scene]:
    import synth
    out = []
    p1 = sil.Params(dtype=sil.U16)
    p0 = sil.Params(dtype=sil.U16, filter=0)
    for i in range(n):
        seed = seed0 + i
        spec = synth.SceneSpec(size, size, seed, "u16",
                               synth.blobs_for_coverage(size, size, seed, 1, 2, 0.10),
                               synth.blobs_for_coverage(size, size, seed, 2, 1, 0.05))
        s, truth = synth.generate(spec, want_truth=True)
        dev = torch.from_numpy(s.view(np.int16)).to(device)
        lab, _ = sil.label(dev, p1)
        lab0, _ = sil.label(dev, p0)
        out.append(Scene(dev, torch.from_numpy(truth).to(device), lab, lab0))
    torch.cuda.synchronize()
    return out


def interior_origins(H: int, W: int, chip: int = CHIP) -> np.ndarray:
    return np.array([(y, x) for y in range(0, H - chip + 1, chip)
                     for x in range(0, W - chip + 1, chip)], dtype=np.int32)


def all_origins(H: int, W: int, chip: int = CHIP) -> np.ndarray:
    return np.array([(y, x) for y in range(0, H, chip) for x in range(0, W, chip)],
                    dtype=np.int32)


def build_training_set(scenes: List[Scene]):
    """bf16 inputs [n, 256, 256, 8] and uint8 auto-label chips [n, 256, 256]."""
    xs, ys = [], []
    for sc in scenes:
        H, W = sc.labels.shape
        org = interior_origins(H, W)
        o = torch.from_numpy(org).to(sc.scene.device)
        xs.append(unet.chips_input(sc.scene, o))
        lab = sc.labels.unfold(0, CHIP, CHIP).unfold(1, CHIP, CHIP)  # [ny, nx, 256, 256]
        ys.append(lab.reshape(-1, CHIP, CHIP).contiguous())
    return torch.cat(xs), torch.cat(ys)


def train(model: unet.UNet, X: torch.Tensor, Y: torch.Tensor, steps: int, batch: int = 32,
          lr: float = 1e-3, seed: int = 0, log_every: int = 0, graph: bool = False):
    """Adam on random batches; returns (losses, seconds per step after warm-up).
    With graph=True the first two steps run eagerly and every later step
    replays one recorded HIP graph of the whole step (unet.CapturedStep)."""
    opt = unet.Adam(model.params, lr=lr)
    g = torch.Generator().manual_seed(seed)
    losses, t_steps = [], []
    captured = None
    for step in range(steps):
        idx = torch.randint(0, X.shape[0], (batch,), generator=g).to(X.device)
        xb, yb = X.index_select(0, idx), Y.index_select(0, idx)
        if graph and captured is None and step >= 2:
            captured = unet.CapturedStep(model, opt, xb, yb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if captured is not None:
            loss = captured(xb, yb)
        else:
            opt.zero_grad()
            loss = model.forward(xb, yb, with_logits=False)[0]
            model.backward(loss)
            opt.step()
            model.update_running_stats()
        torch.cuda.synchronize()
        t_steps.append(time.perf_counter() - t0)
        losses.append(loss.item())
        loss = None  # no autograd graph of an eager step may be alive when the step is recorded
        if log_every and step % log_every == 0:
            print(f"step {step} loss {losses[-1]:.4f} {t_steps[-1] * 1e3:.1f} ms", flush=True)
    opt.sync_step()
    warm = t_steps[min(5, len(t_steps) - 1):]
    return losses, float(np.median(warm))


@torch.no_grad()
def predict_scene(model: unet.UNet, scene: torch.Tensor, batch: int = 64) -> torch.Tensor:
    """U-Net class map [H, W] of a whole scene (edge chips zero-padded)."""
    _, H, W = scene.shape
    org = torch.from_numpy(all_origins(H, W)).to(scene.device)
    out = torch.empty((H, W), dtype=torch.uint8, device=scene.device)
    for i in range(0, org.shape[0], batch):
        o = org[i:i + batch]
        x = unet.chips_input(scene, o)
        logits = model.infer_logits(x)
        unet.scatter_argmax(logits, o, out, H, W)
    return out


def accuracy(a: torch.Tensor, b: torch.Tensor) -> float:
    return (a == b).float().mean().item()


def confusion(pred: torch.Tensor, truth: torch.Tensor, k: int = 3) -> np.ndarray:
    """k x k pixel counts: rows the true class, columns the predicted class."""
    idx = truth.reshape(-1).long() * k + pred.reshape(-1).long()
    return torch.bincount(idx, minlength=k * k).reshape(k, k).cpu().numpy()


def class_scores(cm: np.ndarray) -> dict:
    """Per-class precision, recall and F1 from a confusion matrix (rows true,
    columns predicted), and the column-normalised matrix (each predicted class's
    column sums to 1), as the paper reports them."""
    tp = np.diag(cm).astype(np.float64)
    pred_tot = cm.sum(axis=0).astype(np.float64)
    true_tot = cm.sum(axis=1).astype(np.float64)
    prec = np.divide(tp, pred_tot, out=np.zeros_like(tp), where=pred_tot > 0)
    rec = np.divide(tp, true_tot, out=np.zeros_like(tp), where=true_tot > 0)
    f1 = np.divide(2 * prec * rec, prec + rec, out=np.zeros_like(tp), where=(prec + rec) > 0)
    colnorm = np.divide(cm, pred_tot[None, :], out=np.zeros(cm.shape), where=pred_tot[None, :] > 0)
    return {"precision": prec.tolist(), "recall": rec.tolist(), "f1": f1.tolist(),
            "confusion_col_normalised": colnorm.round(4).tolist()}


def evaluate(model: unet.UNet, scenes: List[Scene]) -> dict:
    """Pixel accuracies against the synthetic truth, the U-Net's disagreement
    with the labeller, and how that disagreement splits: pixels where the U-Net
    matches the truth (it corrects the labeller), where the labeller does, and
    where neither does.  Per class (0 water, 1 thin ice, 2 thick ice):
    precision, recall, F1 and the column-normalised confusion matrix of each
    of the U-Net, the labeller and the unfiltered thresholds against the
    truth."""
    acc_u, acc_l, acc_0, dis = [], [], [], []
    n_dis = n_u = n_l = 0
    cms = {"unet": np.zeros((3, 3), np.int64), "labeller": np.zeros((3, 3), np.int64),
           "thresholds_only": np.zeros((3, 3), np.int64)}
    for sc in scenes:
        pred = predict_scene(model, sc.scene)
        cms["unet"] += confusion(pred, sc.truth)
        cms["labeller"] += confusion(sc.labels, sc.truth)
        cms["thresholds_only"] += confusion(sc.labels0, sc.truth)
        acc_u.append(accuracy(pred, sc.truth))
        acc_l.append(accuracy(sc.labels, sc.truth))
        acc_0.append(accuracy(sc.labels0, sc.truth))
        dis.append(1.0 - accuracy(pred, sc.labels))
        d = pred != sc.labels
        n_dis += int(d.sum().item())
        n_u += int((d & (pred == sc.truth)).sum().item())
        n_l += int((d & (sc.labels == sc.truth)).sum().item())
    n = max(n_dis, 1)
    return {"unet_vs_truth": float(np.mean(acc_u)), "labeller_vs_truth": float(np.mean(acc_l)),
            "thresholds_only_vs_truth": float(np.mean(acc_0)),
            "unet_labeller_disagreement": float(np.mean(dis)),
            "disagreement_unet_right": n_u / n, "disagreement_labeller_right": n_l / n,
            "disagreement_neither_right": (n_dis - n_u - n_l) / n,
            "per_class_vs_truth": {k: class_scores(v) for k, v in cms.items()}}


@torch.no_grad()
def serve_with_fallback(model: unet.UNet, scenes: List[torch.Tensor], threshold: float = 0.02,
                        batch: int = 64, outputs: list = None):
    """Each scene: labeller and U-Net on the same GPU; the U-Net map is kept
    unless it disagrees with the labeller on more than `threshold` of the
    pixels.  Returns per-request records (latency ms, disagreement, fallback);
    the served class maps are appended to `outputs` when given."""
    p = sil.Params(dtype=sil.U16)
    recs = []
    for s in scenes:
        _, H, W = s.shape
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        lab, hist = sil.label(s, p)
        pred = predict_scene(model, s, batch=batch)
        mism = (pred != lab).sum()
        e1.record()
        e1.synchronize()
        d = mism.item() / (H * W)
        recs.append({"H": H, "W": W, "ms": e0.elapsed_time(e1), "disagreement": d,
                     "fallback": d > threshold})
        if outputs is not None:
            outputs.append(lab if d > threshold else pred)
    return recs


@dataclass
class Served:
    """One request of serve_mix: its arrival and completion (ms from the
    start), pixel disagreement with the labeller and whether the labeller's
    map was served; `labels` holds the served map when kept."""
    H: int
    W: int
    arrival_ms: float
    done_ms: float = 0.0
    disagreement: float = 0.0
    fallback: bool = False
    labels: torch.Tensor = None


@torch.no_grad()
def serve_mix(model: unet.UNet, scenes: List[torch.Tensor], arrivals_ms, threshold: float = 0.02,
              batch: int = 128, max_inflight: int = 2, keep: bool = False,
              progress=None) -> List[Served]:
    """Continuous batching of the learned path: requests (scenes [3, H, W] on
    the GPU) arrive at `arrivals_ms` (ms from the start, non-decreasing).  An
    arrived request is labelled at once (sil.label) and its 256 x 256 chips
    join a FIFO of chips; each inference launch takes up to `batch` chips from
    the head of that FIFO, whatever request they belong to, so chips of
    requests that overlap in time share launches.  When a request's last chip
    is inferred its U-Net map is compared with the labeller's and the labeller
    map is served if they disagree on more than `threshold` of the pixels.
    Every kernel treats chips independently, so a request's result does not
    depend on what it shared launches with.  At most `max_inflight` launches
    are queued ahead of the GPU.  `progress(done, n)` (optional) is called
    after every 100 completed requests.  Returns one record per request, in
    order."""
    dev = scenes[0].device
    p = sil.Params(dtype=sil.U16)
    recs = [Served(int(s.shape[1]), int(s.shape[2]), float(a)) for s, a in zip(scenes, arrivals_ms)]
    xbuf = torch.empty((batch, CHIP, CHIP, unet.IN_CH), dtype=torch.bfloat16, device=dev)
    origins_of = {}
    stream = torch.cuda.current_stream(dev)
    start = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    start.synchronize()
    t0 = time.perf_counter()
    pending = 0              # next request to admit
    fifo = []                # [request, origins, next chip, labels, pred]
    launches = []            # events of queued launches
    finishing = []           # (request index, event, pinned mismatch count, labels, pred)
    n = len(scenes)
    done = 0
    while done < n:
        now = (time.perf_counter() - t0) * 1e3
        while pending < n and recs[pending].arrival_ms <= now:
            s = scenes[pending]
            H, W = recs[pending].H, recs[pending].W
            if (H, W) not in origins_of:
                origins_of[(H, W)] = torch.from_numpy(all_origins(H, W)).to(dev)
            lab, _ = sil.label(s, p)
            pred = torch.empty((H, W), dtype=torch.uint8, device=dev)
            fifo.append([pending, origins_of[(H, W)], 0, lab, pred])
            pending += 1
        if fifo:
            # one launch: chips from the head of the FIFO, across requests
            slices, used = [], 0
            for item in fifo:
                if used == batch:
                    break
                i, org, k0, _, _ = item
                k1 = min(org.shape[0], k0 + batch - used)
                unet.chips_input(scenes[i], org[k0:k1], out=xbuf[used:used + k1 - k0])
                slices.append((item, k0, k1, used))
                used += k1 - k0
                item[2] = k1
            logits = model.infer_logits(xbuf[:used])
            for item, k0, k1, off in slices:
                i, org, _, lab, pred = item
                unet.scatter_argmax(logits[off:off + k1 - k0], org[k0:k1], pred, recs[i].H, recs[i].W)
                if k1 == org.shape[0]:
                    mism = (pred != lab).sum().to(torch.int64)
                    host = torch.empty((), dtype=torch.int64, pin_memory=True)
                    host.copy_(mism, non_blocking=True)
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(stream)
                    finishing.append((i, ev, host, lab, pred))
            fifo = [item for item in fifo if item[2] < item[1].shape[0]]
            ev = torch.cuda.Event()
            ev.record(stream)
            launches.append(ev)
            while len(launches) > max_inflight:
                launches.pop(0).synchronize()
        elif not finishing:
            # idle until the next arrival
            if pending < n:
                wait = recs[pending].arrival_ms - (time.perf_counter() - t0) * 1e3
                if wait > 0.2:
                    time.sleep((wait - 0.1) / 1e3)
            continue
        elif not launches or pending >= n:
            finishing[0][1].synchronize()
        still = []
        for i, ev, host, lab, pred in finishing:
            if ev.query():
                r = recs[i]
                r.done_ms = start.elapsed_time(ev)
                r.disagreement = int(host.item()) / (r.H * r.W)
                r.fallback = r.disagreement > threshold
                if keep:
                    r.labels = lab if r.fallback else pred
                done += 1
                if progress is not None and done % 100 == 0:
                    progress(done, n)
            else:
                still.append((i, ev, host, lab, pred))
        finishing = still
    return recs
