"""FLIP on the GPU (the view-consistency term of Sec. 3.5) against the
float64 oracle: per-view scores and the gradient with respect to the test
image over ragged multi-view batches, images smaller than the filters, the
accumulate mode and the error paths."""
import numpy as np
import pytest
import torch

import synthetic
from oracle import flip as oflip
from paper_2503_05168_amd.finetune import seele_flip_loss

pytestmark = pytest.mark.gpu

import gpu_util as gu  # noqa: E402


def _cams(sizes):
    return [synthetic.look_at((0.0, 0.0, -3.0), width=w, height=h) for w, h in sizes]


CASES = {
    "ragged": [(40, 30), (23, 17), (5, 4), (70, 9)],
    "single-64": [(64, 48)],
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("kind", ["near", "random"])
@pytest.mark.parametrize("ppd", [oflip.PPD, 120.0])
def test_flip_matches_oracle(name, kind, ppd):
    """ppd 67 runs the LDS-tiled kernels (radii 10 and 9), ppd 120 the
    untiled ones (radii 17 and 15)."""
    gu.log(f"[case] flip {name} {kind} ppd={ppd:.1f}")
    cams = _cams(CASES[name])
    rng = np.random.default_rng(3 + len(cams))
    ref = [rng.uniform(0.0, 1.0, (3, c.height, c.width)) for c in cams]
    if kind == "near":
        test = [np.clip(r + rng.normal(0, 0.03, r.shape), -0.05, 1.05) for r in ref]
    else:
        test = [rng.uniform(-0.05, 1.05, (3, c.height, c.width)) for c in cams]
    test = [t.astype(np.float32) for t in test]
    ref = [r.astype(np.float32) for r in ref]
    img = torch.from_numpy(np.concatenate([a.ravel() for a in test])).cuda()
    rf = torch.from_numpy(np.concatenate([a.ravel() for a in ref])).cuda()
    val, grad, _ = seele_flip_loss(img, rf, cams, ppd=ppd, scale=0.1)
    torch.cuda.synchronize()
    ov, og = oflip.flip_and_grad(test, ref, ppd)
    np.testing.assert_allclose(val.cpu().numpy(), ov, rtol=2e-4)
    g = grad.cpu().numpy()
    off = 0
    for a, b in zip(test, og):
        n = a.size
        gv = g[off:off + n].reshape(a.shape)
        want = 0.1 * b
        err = np.abs(gv - want)
        scale = np.abs(want).max()
        gu.log(f"  view {a.shape}: max err/scale {err.max() / scale:.2e}")
        # float32 colour transforms, powers and filters against float64
        assert err.max() <= 5e-4 * scale
        off += n
    # accumulate adds onto what the buffer holds
    base = torch.ones_like(grad)
    _, g2, _ = seele_flip_loss(img, rf, cams, ppd=ppd, scale=0.1, accumulate=True, grad=base)
    torch.cuda.synchronize()
    torch.testing.assert_close(g2, grad + 1.0, rtol=0, atol=1e-6)


def test_flip_identical_images_and_errors():
    cams = _cams([(32, 24)])
    x = torch.rand(3 * 32 * 24, device="cuda")
    val, grad, _ = seele_flip_loss(x, x.clone(), cams)
    torch.cuda.synchronize()
    assert float(val[0]) < 1e-5
    from paper_2503_05168_amd import SeeleError
    with pytest.raises(SeeleError, match="pixels per degree"):
        seele_flip_loss(x, x, cams, ppd=400.0)
    with pytest.raises(SeeleError):
        seele_flip_loss(x, x, cams, ppd=-1.0)
