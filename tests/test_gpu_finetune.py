"""Fine-tuning steps on the GPU (Sec. 3.5) against the oracle: the
photometric loss and its image gradient over ragged multi-view batches
(including images smaller than the SSIM window and more views than one
launch holds), the Adam step, and a fine-tuning run whose loss falls."""
import numpy as np
import pytest
import torch

import synthetic
from oracle import loss as oloss
from paper_2503_05168_amd import GaussianTensors, Renderer, Settings
from paper_2503_05168_amd.finetune import (AdamOpts, FineTuner, seele_adam_step,
                                           seele_photometric_loss, zeros_like_gaussians)

pytestmark = pytest.mark.gpu

import gpu_util as gu  # noqa: E402


def _cams(sizes):
    return [synthetic.look_at((0.0, 0.0, -3.0), width=w, height=h) for w, h in sizes]


CASES = {
    "ragged": [(37, 23), (64, 48), (5, 3), (16, 16)],
    "one-1080p-strip": [(1920, 12)],
    "70-tiny": [(4 + k % 5, 3 + k % 4) for k in range(70)],
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("kind", ["random", "near"])
def test_photometric_loss_matches_oracle(name, kind):
    gu.log(f"[case] photometric loss {name} {kind}")
    cams = _cams(CASES[name])
    rng = np.random.default_rng(len(cams))
    tg = [rng.random((3, c.height, c.width)).astype(np.float32) for c in cams]
    if kind == "random":
        im = [rng.random((3, c.height, c.width)).astype(np.float32) for c in cams]
    else:  # the fine-tuning regime: a render close to its target
        im = [np.clip(t + rng.normal(0, 0.02, t.shape), 0, 1).astype(np.float32) for t in tg]
    img = torch.from_numpy(np.concatenate([a.ravel() for a in im])).cuda()
    tgt = torch.from_numpy(np.concatenate([a.ravel() for a in tg])).cuda()
    for lam in (0.2, 0.0, 1.0):
        loss, grad, _ = seele_photometric_loss(img, tgt, cams, lam)
        torch.cuda.synchronize()
        ol, og = oloss.loss_and_grad(im, tg, lam)
        np.testing.assert_allclose(loss.cpu().numpy(), ol, rtol=2e-5, atol=1e-7)
        g = grad.cpu().numpy()
        off = 0
        for a, b in zip(im, og):
            n = a.size
            gv = g[off:off + n].reshape(a.shape)
            scale = np.abs(b).max()
            assert np.abs(gv - b).max() <= 2e-4 * scale + 1e-12, (lam, np.abs(gv - b).max(), scale)
            off += n


@pytest.mark.parametrize("n", [1003, 1024])
def test_adam_matches_oracle(n):
    """n = 1003 runs the scalar kernel, n = 1024 the four-wide one."""
    gu.log(f"[case] adam n={n}")
    rng = np.random.default_rng(9)
    for deg in (3, 1):
        p = GaussianTensors.from_arrays(synthetic.ball_scene(3, n, sh_degree=deg))
        p0 = {k: getattr(p, k).clone() for k in ("means", "log_scales", "quats", "opacity_logits",
                                                  "sh")}
        g, m, v = zeros_like_gaussians(p), zeros_like_gaussians(p), zeros_like_gaussians(p)
        for t in (g, m, v):
            for k in ("means", "log_scales", "quats", "opacity_logits", "sh"):
                x = getattr(t, k)
                x.copy_(torch.from_numpy(rng.normal(size=x.shape).astype(np.float32)))
        v.sh.abs_(), v.means.abs_(), v.log_scales.abs_(), v.quats.abs_(), v.opacity_logits.abs_()
        m0 = {k: getattr(m, k).clone() for k in p0}
        v0 = {k: getattr(v, k).clone() for k in p0}
        opts = AdamOpts(lr_means=1e-3, eps=1e-8)
        seele_adam_step(p, g, m, v, 7, opts, extent=2.0)
        torch.cuda.synchronize()
        n_sh = 3 * (deg + 1) ** 2
        lrs = dict(means=2e-3, log_scales=opts.lr_log_scales, quats=opts.lr_quats,
                   opacity_logits=opts.lr_opacity)
        for k in ("means", "log_scales", "quats", "opacity_logits", "sh"):
            P0, G, M0, V0 = (d[k].cpu().numpy().astype(np.float64) for d in
                             (p0, {k: getattr(g, k)}, m0, v0))
            if k == "sh":
                P0, G, M0, V0 = (a.reshape(48, n) for a in (P0, G, M0, V0))
                parts = [(slice(0, 3), opts.lr_sh_dc), (slice(3, n_sh), opts.lr_sh_rest)]
                got = getattr(p, k).cpu().numpy().reshape(48, n)
                # rows the degree does not use are untouched
                np.testing.assert_array_equal(got[n_sh:], P0[n_sh:].astype(np.float32))
            else:
                parts = [(slice(None), lrs[k])]
                got = getattr(p, k).cpu().numpy()
            for sl, lr in parts:
                # the ABI carries the betas as float32: the oracle takes those values
                want, wm, wv = oloss.adam_step(P0[sl], G[sl], M0[sl], V0[sl], lr, 7,
                                               b1=float(np.float32(0.9)),
                                               b2=float(np.float32(0.999)), eps=1e-8)
                # float32 rounding of the parameter and of the step itself
                err = np.abs(got[sl] - want)
                assert (err <= 1e-6 * np.abs(want) + 1e-6 * np.abs(want - P0[sl])).all(), \
                    (k, err.max())


def test_finetune_reduces_loss_and_composes():
    gu.log("[case] finetune run")
    scene = synthetic.ball_scene(4, 3000, log_scale_mu=-3.0)
    target_scene = synthetic.perturbed_scene(scene, 41, mean_sigma=0.02, logit_sigma=0.3)
    cams = [synthetic.look_at((0.0, 0.0, -3.0), width=96, height=72),
            synthetic.look_at((1.5, 0.5, -2.5), width=80, height=64)]
    st = Settings()
    target = Renderer(st).render(GaussianTensors.from_arrays(target_scene), cams).image.clone()
    g = GaussianTensors.from_arrays(scene)
    opts = AdamOpts(lr_means=2e-4, eps=1e-8)
    ft = FineTuner(g, st, opts=opts, extent=1.0, gamma=0.0)
    losses = []
    for it in range(40):
        before = {k: getattr(g, k).clone() for k in ("means", "opacity_logits")}
        m_before = {k: getattr(ft.m, k).clone() for k in ("means", "opacity_logits")}
        v_before = {k: getattr(ft.v, k).clone() for k in ("means", "opacity_logits")}
        losses.append(float(ft.step(cams, target).mean().item()))
        if it == 3:  # the update is the oracle's Adam on the step's gradients
            for k, lr in (("means", 2e-4), ("opacity_logits", opts.lr_opacity)):
                want, _, _ = oloss.adam_step(before[k].cpu().numpy(),
                                             getattr(ft.grads, k).cpu().numpy(),
                                             m_before[k].cpu().numpy(), v_before[k].cpu().numpy(),
                                             lr, it + 1, b1=float(np.float32(0.9)),
                                             b2=float(np.float32(0.999)), eps=1e-8)
                err = np.abs(getattr(g, k).cpu().numpy() - want)
                assert (err <= 1e-6 * np.abs(want) + 1e-6 * np.abs(want - before[k].cpu().numpy())
                        ).all(), (k, err.max())
    gu.log(f"[done] finetune loss {losses[0]:.5f} -> {losses[-1]:.5f}")
    assert losses[-1] < 0.8 * losses[0]


def test_finetune_with_flip_term_sums_gradients():
    """With the FLIP term (gamma = 0.1, 7 consecutive views per step) a run's
    photometric loss and FLIP both fall."""
    gu.log("[case] finetune with FLIP term")
    scene = synthetic.ball_scene(4, 3000, log_scale_mu=-3.0)
    target_scene = synthetic.perturbed_scene(scene, 41, mean_sigma=0.02, logit_sigma=0.3)
    cams = synthetic.orbit_cameras(7, 3.0, 64, 48)
    st = Settings()
    target = Renderer(st).render(GaussianTensors.from_arrays(target_scene), cams).image.clone()
    g = GaussianTensors.from_arrays(scene)
    ft = FineTuner(g, st, opts=AdamOpts(lr_means=2e-4, eps=1e-8), gamma=0.1)
    losses, flips = [], []
    for it in range(30):
        losses.append(float(ft.step(cams, target).mean().item()))
        flips.append(float(ft.last_flip.mean().item()))
    gu.log(f"[done] loss {losses[0]:.5f} -> {losses[-1]:.5f}, FLIP {flips[0]:.4f} -> {flips[-1]:.4f}")
    assert losses[-1] < 0.8 * losses[0] and flips[-1] < flips[0]


def test_integrated_finetune_with_hp_and_cr():
    """Sec. 3.5's integrated setting on a small built representation: hybrid
    preprocessing (the union of the step's selected clusters) and
    contribution-aware rasterization in the loop.  From a perturbed model
    the loss on a fixed window falls, and Gaussians outside every selected
    segment (never rendered, zero gradient, zero moments) stay bit-identical."""
    from paper_2503_05168_amd import seele_hp_segments, seele_hp_select
    from paper_2503_05168_amd.hp_build import build_view_dependent, seele_gather_gaussians
    gu.log("[case] integrated finetune HP + CR")
    scene = synthetic.cluster_scene(5, 12_000, n_clusters=24)
    g = GaussianTensors.from_arrays(scene)
    poses = synthetic.sampled_orbit_poses(8, 40, 96, 72)
    vd = build_view_dependent(g, poses, 6, k=8, settings=Settings(), views_per_call=8)
    start = seele_gather_gaussians(
        GaussianTensors.from_arrays(synthetic.perturbed_scene(scene, 41, 0.02, 0.3)), vd.perm)
    path = synthetic.orbit_cameras(28, 4.0, 96, 72)
    target = Renderer(Settings()).render(vd.gaussians, path).image.clone()
    npx = 3 * 96 * 72
    st = Settings(mode="contrib", extent="opacity")
    ft = FineTuner(start, st, opts=AdamOpts(lr_means=2e-4, eps=1e-8), gamma=0.1)

    def segs(cams):
        cl = sorted({c for cam in cams for c in seele_hp_select(vd.centroids, cam, vd.pos_scale,
                                                                vd.beta, 1)})
        return seele_hp_segments(vd.seg_begin, vd.seg_count, cl), cl

    unused0 = int(vd.seg_begin[-1] + vd.seg_count[-1])
    before = start.opacity_logits[unused0:].clone()
    losses = []
    for it in range(60):
        s0 = (it * 7) % 21
        cams = path[s0:s0 + 7]
        sg, _ = segs(cams)
        l = ft.step(cams, target[s0 * npx:(s0 + 7) * npx], sg)
        if s0 == 0:
            losses.append(float(l.mean().item()))
    torch.cuda.synchronize()
    gu.log(f"[done] window-0 loss {losses[0]:.5f} -> {losses[-1]:.5f}")
    assert losses[-1] < 0.8 * losses[0]
    assert torch.equal(start.opacity_logits[unused0:], before)
