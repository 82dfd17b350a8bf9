"""GPU tests of the learned part: U-Net inference is the same for a chip
alone and in a batch; a short training on the GPU auto-labels learns the
labeller's classes, and networks trained from two seeds score better than
the labeller against the synthetic truth; the labeller takes over when the
U-Net disagrees with it; in continuous-batched serving every request gets the
same map as when served alone."""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_13135_amd import learn, sil, unet
    sil.lib()
    unet._lib()
    return learn, sil, unet


@pytest.fixture(scope="module")
def data(mods):
    learn, sil, unet = mods
    train_sc = learn.make_scenes(6, 1024, seed0=7100)
    test_sc = learn.make_scenes(2, 1024, seed0=7200)
    X, Y = learn.build_training_set(train_sc)
    return X, Y, test_sc


def _train(mods, data, seed):
    learn, sil, unet = mods
    X, Y, _ = data
    model = unet.UNet((16, 32, 32, 64), seed=seed)
    _say(f"case training seed {seed} on {X.shape[0]} auto-labelled chips")
    losses, sec = learn.train(model, X, Y, steps=150, batch=16, lr=2e-3, seed=seed)
    _say(f"loss {losses[0]:.3f} -> {np.mean(losses[-10:]):.3f}, {sec * 1e3:.1f} ms/step")
    return model, losses


@pytest.fixture(scope="module")
def trained(mods, data):
    model, losses = _train(mods, data, 3)
    return model, losses, data[2]


def test_inference_is_batch_invariant(mods, trained):
    learn, sil, unet = mods
    model, _, test_sc = trained
    sc = test_sc[0].scene
    org = torch.from_numpy(learn.all_origins(1024, 1024)).cuda()
    x = unet.chips_input(sc, org)
    full = model.infer_logits(x)
    for k in (0, 5, 15):
        alone = model.infer_logits(x[k:k + 1].contiguous())
        assert torch.equal(alone[0], full[k]), f"chip {k} differs alone vs in the batch"
    pair = model.infer_logits(x[[3, 9]].contiguous())
    assert torch.equal(pair[0], full[3]) and torch.equal(pair[1], full[9])


def test_training_learns_the_auto_labels(mods, trained):
    learn, sil, unet = mods
    model, losses, test_sc = trained
    assert np.mean(losses[-10:]) < 0.5 * losses[0]
    ev = learn.evaluate(model, test_sc)
    _say(f"held-out: {ev}")
    # the network reproduces the labeller it was trained on...
    assert ev["unet_labeller_disagreement"] < 0.10
    # ...and, like the labeller, beats the unfiltered thresholds against the truth
    assert ev["unet_vs_truth"] > ev["thresholds_only_vs_truth"]


def test_network_beats_the_labeller(mods, trained, data):
    """Networks trained from two seeds on the auto-labels score better than
    the labeller that produced those labels, against the synthetic truth of
    held-out scenes (the paper's comparison of U-Net with and without its
    auto-labelled training, on synthetic truth instead of manual labels)."""
    learn, sil, unet = mods
    model, _, test_sc = trained
    gains = []
    for seed, m in ((3, model), (4, _train(mods, data, 4)[0])):
        ev = learn.evaluate(m, test_sc)
        gains.append(ev["unet_vs_truth"] - ev["labeller_vs_truth"])
        _say(f"seed {seed}: unet {ev['unet_vs_truth']:.4f} labeller {ev['labeller_vs_truth']:.4f} "
             f"gain {gains[-1]:.4f}")
    assert min(gains) > 0.005, gains


def test_fallback_to_the_labeller(mods, trained):
    learn, sil, unet = mods
    model, _, test_sc = trained
    scenes = [sc.scene for sc in test_sc]
    recs = learn.serve_with_fallback(model, scenes, threshold=0.02)
    assert all(r["ms"] > 0 for r in recs)
    # a corrupted network (head biases forcing one class) must fall back
    saved = model.params["head.b"].detach().clone()
    with torch.no_grad():
        model.params["head.b"].copy_(torch.tensor([50.0, 0.0, 0.0], device="cuda"))
    bad = learn.serve_with_fallback(model, scenes, threshold=0.02)
    with torch.no_grad():
        model.params["head.b"].copy_(saved)
    assert all(r["fallback"] for r in bad)
    assert all(r["disagreement"] > 0.02 for r in bad)


def test_checkpoint_round_trip(mods, trained, tmp_path):
    """A trained model and its optimizer state survive save/load: identical
    inference logits and Adam moments and step count; a corrupted file is
    refused."""
    learn, sil, unet = mods
    model, _, test_sc = trained
    opt = unet.Adam(model.params, lr=1e-3)
    X, Y = learn.build_training_set(test_sc[:1])
    for k in range(3):  # gives the optimizer a history
        opt.zero_grad()
        loss, _ = model.forward(X[4 * k:4 * k + 4].contiguous(), Y[4 * k:4 * k + 4].contiguous())
        loss.backward()
        opt.step()
        model.update_running_stats()
    torch.cuda.synchronize()
    path = str(tmp_path / "unet.safetensors")
    unet.save_checkpoint(path, model, opt, extra={"step": 3, "seed": 7})
    m2, o2, extra = unet.load_checkpoint(path)
    assert extra == {"step": 3, "seed": 7} and o2.t == opt.t
    x = X[:2].contiguous()
    assert torch.equal(model.infer_logits(x), m2.infer_logits(x))
    for k in opt.m:
        assert torch.equal(opt.m[k], o2.m[k]) and torch.equal(opt.v[k], o2.v[k])
    # a corrupted file is refused
    raw = bytearray(open(path, "rb").read())
    raw[-5] ^= 0xFF
    bad = str(tmp_path / "bad.safetensors")
    open(bad, "wb").write(bytes(raw))
    with pytest.raises(ValueError):
        unet.load_checkpoint(bad)


def test_continuous_batched_serving_equals_solo(mods, trained):
    """Requests of mixed sizes arriving together and staggered share inference
    launches; each served map (the U-Net's, threshold 1) equals the map of the
    same request served alone and the sequential path's; with threshold 0
    every request falls back to its labeller map."""
    learn, sil, unet = mods
    import synth
    model = trained[0]
    scenes = []
    for i, (H, W) in enumerate([(512, 512), (700, 900), (1024, 1024), (300, 2048), (512, 512),
                                (1500, 1100)]):
        spec = synth.SceneSpec(H, W, 7300 + i, "u16",
                               synth.blobs_for_coverage(H, W, 7300 + i, 1, 1, 0.10),
                               synth.blobs_for_coverage(H, W, 7300 + i, 2, 1, 0.05))
        scenes.append(torch.from_numpy(synth.generate(spec).view(np.int16)).cuda())
    solo = [learn.serve_mix(model, [s], [0.0], threshold=1.0, batch=8, keep=True)[0]
            for s in scenes]
    seq = []
    learn.serve_with_fallback(model, scenes, threshold=1.0, outputs=seq)
    for arrivals in ([0.0] * len(scenes), [0.0, 1.0, 2.0, 2.0, 3.0, 30.0]):
        _say(f"case serve_mix arrivals {arrivals}")
        mixed = learn.serve_mix(model, scenes, arrivals, threshold=1.0, batch=8, keep=True)
        for i, (m, a) in enumerate(zip(mixed, solo)):
            assert not m.fallback and m.done_ms >= m.arrival_ms
            assert torch.equal(m.labels, a.labels), f"request {i} differs in the mix"
            assert torch.equal(m.labels, seq[i]), f"request {i} differs from the sequential path"
            assert m.disagreement == a.disagreement
    fb = learn.serve_mix(model, scenes, [0.0] * len(scenes), threshold=0.0, batch=8, keep=True)
    p = sil.Params(dtype=sil.U16)
    for s, r in zip(scenes, fb):
        assert r.fallback and torch.equal(r.labels, sil.label(s, p)[0])
