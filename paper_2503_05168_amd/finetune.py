"""Fine-tuning through the unchanged pipeline (Sec. 3.5): the photometric
loss of 3DGS training with its image gradient (seele_photometric_loss), the
library's backward (seele_rasterize_bwd) and an Adam step over the Gaussian
attributes (seele_adam_step).  Rendering may use hybrid preprocessing
(active segments) and contribution-aware rasterization: neither changes the
backward, whose decisions are the forward's."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _abi as A
from .pipeline import (GaussianTensors, Renderer, Settings, _need, _p, _stream, pixel_count,
                       seele_rasterize_bwd)


def seele_photometric_loss(image, target, cams, lam: float = 0.2, workspace=None, loss=None,
                           grad=None, stream=None):
    """(per-view losses [V], dL/dimage of their mean, workspace)."""
    cam_arr = A.camera_array(cams)
    V = len(cams)
    need = A.lib().seele_photometric_loss_workspace_size(cam_arr, V)
    dev = image.device
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    if loss is None:
        loss = torch.empty(V, dtype=torch.float32, device=dev)
    if grad is None:
        grad = torch.empty_like(image)
    npx = 3 * pixel_count(cams)
    _need(image, npx, torch.float32, "image")
    _need(target, npx, torch.float32, "target")
    _need(grad, npx, torch.float32, "grad")
    _need(loss, V, torch.float32, "loss")
    _need(workspace, need, torch.uint8, "workspace")
    st = A.lib().seele_photometric_loss(_p(image), _p(target), cam_arr, V, float(lam),
                                        _p(workspace), workspace.numel(), _p(loss), _p(grad),
                                        _stream(stream))
    A.check(st, "seele_photometric_loss")
    return loss, grad, workspace


@dataclass
class AdamOpts:
    """Learning rates of 3DGS training at the end of its schedule (the means'
    rate is multiplied by the scene extent), betas and eps as 3DGS."""
    lr_means: float = 1.6e-6
    lr_log_scales: float = 5e-3
    lr_quats: float = 1e-3
    lr_opacity: float = 5e-2
    lr_sh_dc: float = 2.5e-3
    lr_sh_rest: float = 2.5e-3 / 20.0
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15

    def struct(self, extent: float = 1.0) -> A.seele_adam_opts:
        o = A.seele_adam_opts()
        o.lr_means = self.lr_means * extent
        o.lr_log_scales, o.lr_quats = self.lr_log_scales, self.lr_quats
        o.lr_opacity, o.lr_sh_dc, o.lr_sh_rest = self.lr_opacity, self.lr_sh_dc, self.lr_sh_rest
        o.beta1, o.beta2, o.eps = self.beta1, self.beta2, self.eps
        return o


def _desc(t: GaussianTensors, n: int, name: str) -> A.seele_gaussian_grads:
    """Descriptor of n Gaussians' attribute arrays (sizes checked)."""
    t.check(n, name)
    d = A.seele_gaussian_grads()
    for attr in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        x = getattr(t, attr)
        setattr(d, attr, x.data_ptr() if x.numel() else None)
    return d


def zeros_like_gaussians(g: GaussianTensors) -> GaussianTensors:
    return GaussianTensors(torch.zeros_like(g.means), torch.zeros_like(g.log_scales),
                           torch.zeros_like(g.quats), torch.zeros_like(g.opacity_logits),
                           torch.zeros_like(g.sh), g.sh_degree)


def seele_adam_step(params: GaussianTensors, grads: GaussianTensors, m: GaussianTensors,
                    v: GaussianTensors, step: int, opts: AdamOpts | None = None,
                    extent: float = 1.0, stream=None):
    o = (opts or AdamOpts()).struct(extent)
    n = params.n
    st = A.lib().seele_adam_step(ctypes.byref(_desc(params, n, "params")),
                                 ctypes.byref(_desc(grads, n, "grads")),
                                 ctypes.byref(_desc(m, n, "m")), ctypes.byref(_desc(v, n, "v")), n,
                                 params.sh_degree, ctypes.byref(o), int(step), _stream(stream))
    A.check(st, "seele_adam_step")


class FineTuner:
    """Fine-tunes a scene (in place) against target images with the loss of
    Sec. 3.5, L_3DGS + gamma * FLIP over the step's views (gamma = 0.1; the
    paper's steps take 7 consecutive frames): each step renders the views
    (optionally with active segments), takes both loss terms with their
    image gradients, runs the backward and one Adam step."""

    def __init__(self, g: GaussianTensors, settings: Settings | None = None, lam: float = 0.2,
                 opts: AdamOpts | None = None, extent: float = 1.0, capacity: int = 1 << 22,
                 gamma: float = 0.1, ppd: float | None = None, lists: str = "super"):
        """lists: "super" (super-tile lists; the backward flushes each record
        once per 2 x 2-tile quadrant; 16 x 16 tiles) or "tile" (per-tile
        lists, any tile size)."""
        self.g = g
        self.settings = settings or Settings()
        self.lam = lam
        self.gamma = gamma
        self.ppd = ppd
        self.opts = opts or AdamOpts()
        self.extent = extent
        self.m = zeros_like_gaussians(g)
        self.v = zeros_like_gaussians(g)
        self.grads = zeros_like_gaussians(g)
        if lists == "super" and self.settings.tile != 16:
            lists = "tile"  # the super-tile backward takes 16 x 16 tiles
        self.renderer = Renderer(self.settings, capacity=capacity, lists=lists, last_entry=True)
        self.t = 0
        self._ws = None
        self._fws = None
        self._grad2d = None
        self._pairs = None
        self.last_flip = None

    def renderer_last_pairs(self):
        """Device count of the stored list length of the last step's render
        (super-tile entries, or pairs for per-tile lists), to check the
        capacity after steps run with check=False."""
        return self._pairs

    def step(self, cams, target, segments=None, check: bool = True, events=None):
        """One step; returns the per-view photometric losses (device; the
        per-view FLIP is kept in last_flip).  events, if given, are five CUDA
        events recorded after render, photometric loss, FLIP, backward,
        Adam."""
        f = self.renderer.render(self.g, cams, segments, check=check)
        self._pairs = f.num_entries if f.num_entries is not None else f.num_pairs
        if events is not None:
            events[0].record()
        loss, dL, self._ws = seele_photometric_loss(f.image, target, cams, self.lam, self._ws)
        if events is not None:
            events[1].record()
        if self.gamma:
            self.last_flip, _, self._fws = seele_flip_loss(
                f.image, target, cams, self.ppd or FLIP_PPD, self.gamma, True, dL, self._fws)
        if events is not None:
            events[2].record()
        n_rec = len(cams) * self.g.n
        if self._grad2d is None or self._grad2d.shape[0] < n_rec:
            self._grad2d = torch.empty((n_rec, 9), dtype=torch.float32, device=self.g.means.device)
        seele_rasterize_bwd(self.g, cams, self.settings, f.splats, f.n_tiles, f.sorted_ids,
                            f.tile_ranges, f.final_T, f.n_contrib, dL, segments,
                            self._grad2d[:n_rec], self.grads, entry_keys=f.entry_keys,
                            last_entry=f.last_entry)
        if events is not None:
            events[3].record()
        self.t += 1
        seele_adam_step(self.g, self.grads, self.m, self.v, self.t, self.opts, self.extent)
        if events is not None:
            events[4].record()
        return loss


FLIP_PPD = 0.7 * (3840 / 0.7) * 3.141592653589793 / 180.0  # FLIP's default viewer


def seele_flip_loss(image, reference, cams, ppd: float = FLIP_PPD, scale: float = 1.0,
                    accumulate: bool = False, grad=None, workspace=None, flip=None,
                    stream=None):
    """(per-view mean FLIP [V], gradient buffer, workspace): the gradient of
    scale * (mean over views) is written into `grad`, or added to it with
    accumulate=True."""
    cam_arr = A.camera_array(cams)
    V = len(cams)
    need = A.lib().seele_flip_loss_workspace_size(cam_arr, V)
    dev = image.device
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    if flip is None:
        flip = torch.empty(V, dtype=torch.float32, device=dev)
    if grad is None:
        if accumulate:
            raise ValueError("accumulate needs a gradient buffer")
        grad = torch.empty_like(image)
    npx = 3 * pixel_count(cams)
    _need(image, npx, torch.float32, "image")
    _need(reference, npx, torch.float32, "reference")
    _need(grad, npx, torch.float32, "grad")
    _need(flip, V, torch.float32, "flip")
    _need(workspace, need, torch.uint8, "workspace")
    st = A.lib().seele_flip_loss(_p(image), _p(reference), cam_arr, V, float(ppd), float(scale),
                                 int(bool(accumulate)), _p(workspace), workspace.numel(), _p(flip),
                                 _p(grad), _stream(stream))
    A.check(st, "seele_flip_loss")
    return flip, grad, workspace
