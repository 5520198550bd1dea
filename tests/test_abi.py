"""The C ABI without a GPU: every declared symbol is exported, the struct
layouts agree between the header (compiled by gcc) and the binding, argument
validation rejects bad calls before anything is enqueued, and the host-only
hybrid-preprocessing selection matches the oracle."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import synthetic
from oracle import hp as ohp
from paper_2503_05168_amd import _abi as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "seele.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(seele_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = A.lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(A.SIGNATURES)


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    structs = {
        "seele_gaussians": [f for f, _ in A.seele_gaussians._fields_],
        "seele_gaussian_grads": [f for f, _ in A.seele_gaussian_grads._fields_],
        "seele_camera": [f for f, _ in A.seele_camera._fields_],
        "seele_splat": [f for f, _ in A.seele_splat._fields_],
        "seele_preprocess_opts": [f for f, _ in A.seele_preprocess_opts._fields_],
        "seele_raster_opts": [f for f, _ in A.seele_raster_opts._fields_],
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(){"]
    for s, fields in structs.items():
        lines.append(f'printf("{s} %zu\\n", sizeof({s}));')
        for f in fields:
            lines.append(f'printf("{s}.{f} %zu\\n", offsetof({s}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = dict(l.rsplit(" ", 1) for l in out.strip().splitlines())
    for s, fields in structs.items():
        cls = getattr(A, s)
        assert int(got[s]) == ctypes.sizeof(cls), s
        for f in fields:
            assert int(got[f"{s}.{f}"]) == getattr(cls, f).offset, (s, f)
    assert int(got["seele_splat"]) == 64 and int(got["seele_camera"]) == 72


def _cam(w=64, h=48):
    return A.camera_array([synthetic.look_at((0, 0, -3), width=w, height=h)])


def _popts(tile=16, extent=0):
    o = A.seele_preprocess_opts()
    o.tile, o.extent, o.alpha_min, o.lowpass, o.z_near, o.n_segs = tile, extent, 1 / 255, 0.3, 0.2, 0
    return o


def _ropts(tile=16, mode=0, gw=2, gh=2):
    o = A.seele_raster_opts()
    o.tile, o.mode, o.group_w, o.group_h = tile, mode, gw, gh
    o.alpha_min, o.alpha_max, o.T_min = 1 / 255, 0.99, 1e-4
    return o


FAKE = ctypes.c_void_p(0x10000)  # aligned, never dereferenced: every call below fails validation


def _gauss(n=10, deg=3, null_field=None):
    g = A.seele_gaussians()
    g.n, g.sh_degree = n, deg
    for f in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        setattr(g, f, None if f == null_field else 0x10000)
    return g


@pytest.mark.parametrize("case", ["null_g", "neg_n", "deg4", "null_means", "tile12", "extent7",
                                  "alpha0", "nviews0", "cam0x0", "seg_oob", "segs_too_many",
                                  "splats_misaligned"])
def test_preprocess_rejects_bad_arguments(case):
    L = A.lib()
    g, cams, nv, o, sp = _gauss(), _cam(), 1, _popts(), ctypes.c_void_p(0x10000)
    keep = None
    if case == "null_g":
        g = None
    elif case == "neg_n":
        g = _gauss(n=-1)
    elif case == "deg4":
        g = _gauss(deg=4)
    elif case == "null_means":
        g = _gauss(null_field="means")
    elif case == "tile12":
        o = _popts(tile=12)
    elif case == "extent7":
        o = _popts(extent=7)
    elif case == "alpha0":
        o.alpha_min = 0.0
    elif case == "nviews0":
        nv = 0
    elif case == "cam0x0":
        cams = _cam(0, 0)
    elif case == "seg_oob":
        b, c = (ctypes.c_int64 * 1)(5), (ctypes.c_int64 * 1)(6)
        o.n_segs, o.seg_begin, o.seg_count = 1, b, c
        keep = (b, c)
    elif case == "segs_too_many":
        b, c = (ctypes.c_int64 * 17)(), (ctypes.c_int64 * 17)()
        o.n_segs, o.seg_begin, o.seg_count = 17, b, c
        keep = (b, c)
    elif case == "splats_misaligned":
        sp = ctypes.c_void_p(0x10004)
    st = L.seele_preprocess(ctypes.byref(g) if g is not None else None, cams, nv,
                            ctypes.byref(o), sp, FAKE, None)
    assert st in (A.SEELE_ERR_INVALID_ARG, A.SEELE_ERR_UNSUPPORTED), (case, st)
    assert L.seele_last_error()
    del keep


def test_bin_sort_rejects_bad_arguments():
    L = A.lib()
    cams = _cam()
    need = L.seele_bin_sort_workspace_size(10, 1000, 12)
    assert need > 0
    args = lambda ws_bytes, cap, ws=FAKE, nv=1: L.seele_bin_sort(
        FAKE, FAKE, 10, cams, nv, 16, ws, ws_bytes, FAKE, cap, FAKE, FAKE, None)
    assert args(need - 1, 1000) == A.SEELE_ERR_CAPACITY
    assert args(need, -1) == A.SEELE_ERR_INVALID_ARG
    assert args(need, 1 << 31) == A.SEELE_ERR_INVALID_ARG
    assert args(need, 1000, ws=ctypes.c_void_p(0x10010)) == A.SEELE_ERR_INVALID_ARG
    assert args(need, 1000, nv=300) == A.SEELE_ERR_UNSUPPORTED
    assert L.seele_bin_sort(FAKE, FAKE, 10, cams, 1, 16, FAKE, need, FAKE, 1000, FAKE,
                            ctypes.c_void_p(0x10004), None) == A.SEELE_ERR_INVALID_ARG


def test_bin_sort_noalloc_refuses_before_touching_the_device():
    """The no-allocation binning refuses staged input and any frame whose
    workspace exceeds its scratch array, with no GPU call (runs on CPU)."""
    L = A.lib()
    cams = _cam()
    call = lambda flags, n, cap: L.seele_bin_sort_noalloc(flags, FAKE, FAKE, n, cams, 1, 16, FAKE,
                                                           FAKE, cap, FAKE, FAKE, None)
    assert call(A.SEELE_BIN_STAGED, 10, 1000) == A.SEELE_ERR_INVALID_ARG
    assert call(4, 10, 1000) == A.SEELE_ERR_INVALID_ARG
    assert call(0, -1, 1000) == A.SEELE_ERR_INVALID_ARG
    assert call(0, 10, 1 << 31) == A.SEELE_ERR_INVALID_ARG
    big = 4 << 20
    assert L.seele_bin_sort_workspace_size(big, 1, 12) > A.SEELE_NOALLOC_SCRATCH_BYTES
    assert call(0, big, 1) == A.SEELE_ERR_CAPACITY
    assert call(A.SEELE_BIN_SUPER, 1000, 20 << 20) == A.SEELE_ERR_CAPACITY
    assert b"scratch" in L.seele_last_error()


def test_total_tiles_and_workspace_size():
    L = A.lib()
    cams = A.camera_array([synthetic.look_at((0, 0, -3), width=w, height=h)
                           for w, h in ((1920, 1080), (37, 23), (1, 1))])
    assert L.seele_total_tiles(cams, 3, 16) == 120 * 68 + 3 * 2 + 1
    assert L.seele_total_tiles(cams, 3, 8) == 240 * 135 + 5 * 3 + 1
    assert L.seele_total_tiles(cams, 3, 12) == -1
    assert L.seele_bin_sort_workspace_size(100, 1000, 64) >= 4 * (4 * 100 + 3 * 1000)


@pytest.mark.parametrize("mutate", ["tile", "mode", "group3", "group_big", "amax", "tmin", "null"])
def test_raster_rejects_bad_arguments(mutate):
    L = A.lib()
    o = _ropts(mode=1)
    out = FAKE
    if mutate == "tile":
        o.tile = 32
    elif mutate == "mode":
        o.mode = 5
    elif mutate == "group3":
        o.group_w = 3
    elif mutate == "group_big":
        o.group_w, o.group_h = 4, 8
    elif mutate == "amax":
        o.alpha_max = 1.0
    elif mutate == "tmin":
        o.T_min = 0.0
    elif mutate == "null":
        out = None
    st = L.seele_rasterize_fwd(FAKE, FAKE, FAKE, _cam(), 1, ctypes.byref(o), out, FAKE, FAKE, None)
    assert st == A.SEELE_ERR_INVALID_ARG, mutate


def test_hp_select_matches_oracle():
    L = A.lib()
    rng = np.random.default_rng(0)
    K = 24
    cents = rng.normal(size=(K, 6)).astype(np.float32)
    cbuf = (ctypes.c_float * (K * 6))(*cents.ravel().tolist())
    for k in range(40):
        d = rng.normal(size=3)
        cam = synthetic.look_at(d / np.linalg.norm(d) * rng.uniform(2, 6))
        for M in (0, 1, 3):
            out = (ctypes.c_int32 * (1 + M))()
            assert L.seele_hp_select(cbuf, K, ctypes.byref(A.make_camera(cam)), 4.0, 1.0, M,
                                     out) == A.SEELE_OK
            want = ohp.select_clusters(cents.astype(np.float64), ohp.camera_feature(cam, 4.0), M)
            assert list(out) == want


def test_hp_segments_match_oracle():
    L = A.lib()
    cfg = synthetic.config(3, n=5000)
    lay = cfg["hp"]
    K = len(lay.seg_begin) - 1
    lb = (ctypes.c_int64 * (K + 1))(*lay.seg_begin.tolist())
    lc = (ctypes.c_int64 * (K + 1))(*lay.seg_count.tolist())
    for sel in ([0], [3, 4], [7, 0, 1, 2], [5, 5]):
        cl = (ctypes.c_int32 * len(sel))(*sel)
        ob, oc, no = (ctypes.c_int64 * 8)(), (ctypes.c_int64 * 8)(), ctypes.c_int32()
        assert L.seele_hp_segments(lb, lc, K, cl, len(sel), ob, oc, ctypes.byref(no)) == A.SEELE_OK
        got = [(ob[i], oc[i]) for i in range(no.value)]
        assert got == ohp.active_segments(lay.seg_begin, lay.seg_count, sel)
    cl = (ctypes.c_int32 * 1)(9)
    ob, oc, no = (ctypes.c_int64 * 2)(), (ctypes.c_int64 * 2)(), ctypes.c_int32()
    assert L.seele_hp_segments(lb, lc, K, cl, 1, ob, oc, ctypes.byref(no)) == A.SEELE_ERR_INVALID_ARG


def test_bindings_refuse_undersized_buffers():
    # the library sees plain pointers; the binding checks sizes before the call
    import torch
    from paper_2503_05168_amd import pipeline as pl
    ok = torch.empty(64, dtype=torch.float32)
    assert pl._need(ok, 64, torch.float32, "x") is ok
    for bad in (torch.empty(63, dtype=torch.float32), torch.empty(64, dtype=torch.int32),
                torch.empty(128, dtype=torch.float32)[::2]):
        with pytest.raises(ValueError):
            pl._need(bad, 64, torch.float32, "x")


def test_loss_optimizer_and_builder_bindings_refuse_undersized_buffers():
    # CPU tensors: every check runs before the library is handed a pointer
    import torch
    from paper_2503_05168_amd import finetune as ft
    from paper_2503_05168_amd import hp_build as hb
    from paper_2503_05168_amd.pipeline import GaussianTensors
    cams = [synthetic.look_at((0, 0, -3), width=8, height=6),
            synthetic.look_at((0, 0, -3), width=5, height=4)]
    npx = 3 * (48 + 20)
    f = lambda k, dt=torch.float32: torch.zeros(k, dtype=dt)
    for args in ((f(npx - 1), f(npx), {}), (f(npx), f(npx - 1), {}),
                 (f(npx), f(npx), dict(grad=f(npx - 1))), (f(npx), f(npx), dict(loss=f(1)))):
        with pytest.raises(ValueError):
            ft.seele_photometric_loss(args[0], args[1], cams, 0.2, **args[2])
        with pytest.raises(ValueError):
            kw = dict(args[2])
            if "loss" in kw:
                kw["flip"] = kw.pop("loss")
            ft.seele_flip_loss(args[0], args[1], cams, **kw)
    n = 10
    g = lambda m: GaussianTensors(f(3 * m).reshape(3, m), f(3 * m).reshape(3, m),
                                  f(4 * m).reshape(4, m), f(m), f(48 * m).reshape(16, 3, m))
    short = g(n)
    short.sh = f(48 * n - 1)
    for bad in ("grads", "m", "v"):
        ts = dict(grads=g(n), m=g(n), v=g(n))
        ts[bad] = g(n - 1)
        with pytest.raises(ValueError):
            ft.seele_adam_step(g(n), ts["grads"], ts["m"], ts["v"], 1)
    with pytest.raises(ValueError):
        ft.seele_adam_step(g(n), short, g(n), g(n), 1)
    u8 = lambda k: f(k, torch.uint8)
    ok = dict(mark=u8(2 * n), sums=f(2 * n), shared=u8(n), best_sum=f(n),
              best_cluster=f(n, torch.int32))
    for k, small in (("mark", u8(2 * n - 1)), ("sums", f(2 * n - 1)), ("shared", u8(n - 1)),
                     ("best_sum", f(n - 1)), ("best_cluster", f(n - 1, torch.int32))):
        a = dict(ok)
        a[k] = small
        with pytest.raises(ValueError):
            hb.seele_hp_accumulate(a["mark"], a["sums"], 2, n, 0, a["shared"], a["best_sum"],
                                   a["best_cluster"])
    with pytest.raises(ValueError):
        hb.seele_gather_gaussians(short, torch.arange(n, dtype=torch.int64))


def test_hp_kmeans_matches_oracle():
    # host routine: labels exactly, centroids to float32 rounding
    from paper_2503_05168_amd.hp_build import seele_hp_kmeans
    rng = np.random.default_rng(11)
    for trial in range(6):
        n = int(rng.integers(5, 60))
        cams = []
        for _ in range(n):
            d = rng.normal(size=3)
            cams.append(synthetic.look_at(d / np.linalg.norm(d) * rng.uniform(2, 6)))
        cams += synthetic.orbit_cameras(int(rng.integers(1, 12)), 4.0, 64, 64)
        K = int(rng.integers(1, min(8, len(cams)) + 1))
        beta = float(rng.choice([0.5, 1.0, 2.0]))
        cents, lab = seele_hp_kmeans(cams, 6.0, beta, K, 50)
        f = np.stack([ohp.camera_feature(c, 6.0, beta) for c in cams])
        oc, ol = ohp.kmeans(f, K, 50)
        assert lab.tolist() == ol.tolist()
        np.testing.assert_allclose(cents, oc, rtol=0, atol=1e-6)


def test_hp_kmeans_rejects_bad_args():
    L = A.lib()
    cams = A.camera_array([synthetic.look_at((0, 0, -4))] * 3)
    c = (ctypes.c_float * 24)()
    lab = (ctypes.c_int32 * 3)()
    for K, ps in ((0, 1.0), (4, 1.0), (2, float("nan")), (2, float("inf"))):
        assert L.seele_hp_kmeans(cams, 3, ps, 1.0, K, 10, c, lab) == A.SEELE_ERR_INVALID_ARG
    # pos_scale <= 0 takes the library default, which needs a centre away from the origin
    origin = A.camera_array([synthetic.look_at((0, 0, -4))])
    origin[0].t[0] = origin[0].t[1] = origin[0].t[2] = 0.0
    assert L.seele_hp_kmeans(origin, 1, 0.0, 1.0, 1, 10, c, lab) == A.SEELE_ERR_INVALID_ARG
    assert L.seele_hp_pos_scale(origin, 0) < 0 and L.seele_hp_pos_scale(None, 1) < 0


def test_hp_kmeans_default_pos_scale_matches_oracle():
    from paper_2503_05168_amd.hp_build import seele_hp_kmeans, seele_hp_pos_scale
    rng = np.random.default_rng(12)
    cams = []
    for _ in range(40):
        d = rng.normal(size=3)
        cams.append(synthetic.look_at(d / np.linalg.norm(d) * rng.uniform(2, 7)))
    ps = ohp.default_pos_scale(cams)
    assert abs(seele_hp_pos_scale(cams) - ps) <= 1e-6 * ps
    for p_in in (0.0, -3.0):
        cents, lab = seele_hp_kmeans(cams, p_in, 1.0, 5, 50)
        cents2, lab2 = seele_hp_kmeans(cams, seele_hp_pos_scale(cams), 1.0, 5, 50)
        assert lab.tolist() == lab2.tolist()
        np.testing.assert_array_equal(cents, cents2)
    f = np.stack([ohp.camera_feature(c, ps, 1.0) for c in cams])
    oc, ol = ohp.kmeans(f, 5, 50)
    assert lab.tolist() == ol.tolist()
    np.testing.assert_allclose(cents, oc, rtol=0, atol=1e-6)


def test_hp_partition_matches_oracle():
    from paper_2503_05168_amd.hp_build import seele_hp_partition
    rng = np.random.default_rng(12)
    for n, K in ((0, 1), (1, 1), (37, 3), (2000, 8)):
        marks = [rng.random(n) < 0.1 for _ in range(K)]
        # dyadic sums with many ties and zeros
        sums = [np.where(rng.random(n) < 0.6, rng.integers(0, 5, n) / 8.0, 0.0).astype(np.float32)
                for _ in range(K)]
        # the fold the device performs cluster by cluster (strictly larger wins)
        shared = np.any(marks, axis=0).astype(np.uint8) if n else np.zeros(0, np.uint8)
        best = np.zeros(n, np.float32)
        bc = np.full(n, -1, np.int32)
        for c in range(K):
            up = sums[c] > best
            best[up], bc[up] = sums[c][up], c
        perm, begin, count = seele_hp_partition(shared, best, bc, K)
        op, ob, oc = ohp.partition(marks, [s.astype(np.float64) for s in sums], n)
        assert perm.tolist() == op.tolist()
        assert begin.tolist() == ob.tolist() and count.tolist() == oc.tolist()


def test_pose_extrapolate_matches_oracle():
    from oracle import prefetch as opf
    from paper_2503_05168_amd.prefetch import seele_pose_extrapolate
    rng = np.random.default_rng(21)
    cams = synthetic.sampled_orbit_poses(4, 30, 64, 48)
    cams += synthetic.orbit_cameras(8, 4.0, 64, 48)
    for i in range(len(cams) - 1):
        a, b = cams[i], cams[i + 1]
        for s in (0.0, 1.0, 2.5, -1.0, float(rng.uniform(-3, 3))):
            got = seele_pose_extrapolate(a, b, s)
            R, t = opf.extrapolate_pose(a.R, a.t, b.R, b.t, s)
            np.testing.assert_allclose(got.R, R, atol=2e-6)
            np.testing.assert_allclose(got.t, t, atol=2e-5 * max(1.0, abs(s)))
            assert (got.width, got.height, got.fx) == (b.width, b.height, np.float32(b.fx))
    # half a turn between the frames (the near-pi branch of the rotation log)
    a = synthetic.look_at((0.0, 0.0, -4.0))
    b = synthetic.look_at((0.0, 0.0, 4.0))
    got = seele_pose_extrapolate(a, b, 1.0)
    R, t = opf.extrapolate_pose(a.R, a.t, b.R, b.t, 1.0)
    np.testing.assert_allclose(got.R, R, atol=2e-6)


def test_resident_plan_matches_oracle():
    from oracle import prefetch as opf
    from paper_2503_05168_amd.prefetch import seele_resident_plan
    rng = np.random.default_rng(22)
    for K, S in ((6, 4), (24, 8), (3, 3)):
        cnt = rng.integers(0, 50, K).astype(np.int64)
        sc = np.full(S, -1, np.int32)
        ss = np.zeros(S, np.int64)
        osc, oss = list(sc), list(ss)
        for frame in range(1, 300):
            need = [int(x) for x in rng.choice(K, size=int(rng.integers(1, min(S, 4) + 1)),
                                                replace=False)]
            want = [int(x) for x in rng.choice(K, size=int(rng.integers(0, min(K, 6) + 1)),
                                                replace=False)]
            loads, nd = seele_resident_plan(sc, ss, cnt, 50, need, want, frame)
            osc, oss, oloads, ond = opf.plan(osc, oss, cnt, 50, need, want, frame)
            assert loads == oloads and nd == ond, frame
            assert sc.tolist() == osc and ss.tolist() == oss


def test_resident_plan_and_load_reject_bad_args():
    from paper_2503_05168_amd import SeeleError
    from paper_2503_05168_amd.prefetch import seele_resident_plan
    cnt = np.array([5, 60], np.int64)
    sc = np.full(2, -1, np.int32)
    ss = np.zeros(2, np.int64)
    with pytest.raises(SeeleError):
        seele_resident_plan(sc, ss, cnt, 50, [1], [], 1)  # larger than a slot
    with pytest.raises(SeeleError):
        seele_resident_plan(np.full(1, -1, np.int32), np.zeros(1, np.int64), cnt[:1] * 0, 50,
                            [0, 1], [], 1)  # two clusters, one slot
    with pytest.raises(SeeleError):
        seele_resident_plan(np.array([0, 0], np.int32), ss, cnt, 50, [0], [], 1)  # duplicate
    L = A.lib()
    b = (ctypes.c_int64 * 1)(5)
    d = (ctypes.c_int64 * 1)(0)
    c = (ctypes.c_int64 * 1)(10)
    # columns 5..15 of a 12-column table: refused before anything is enqueued
    assert L.seele_load_segments(FAKE, 12, FAKE, 100, 59, b, d, c, 1, None) == \
        A.SEELE_ERR_INVALID_ARG
    assert L.seele_load_segments(FAKE, 100, FAKE, 8, 59, b, d, c, 1, None) == \
        A.SEELE_ERR_INVALID_ARG
