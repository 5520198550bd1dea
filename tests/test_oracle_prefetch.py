"""Pins for the oracle's scene prefetching (Sec. 3.3 "Scene Prefetching"):
closed forms of linear pose extrapolation and hand-worked resident-set
plans with their invariants (CPU only)."""
import math

import numpy as np

import synthetic
from oracle import prefetch as opf


def _rt(cam):
    return np.asarray(cam.R, np.float64), np.asarray(cam.t, np.float64)


def test_extrapolate_straight_dolly():
    # fixed orientation, centre moving along a line: the next point on it
    a = synthetic.look_at((0.0, 0.0, -4.0))
    R = np.asarray(a.R, np.float64)
    c0, c1 = np.array([0.3, -0.2, -4.0]), np.array([0.5, -0.1, -3.8])
    R2, t2 = opf.extrapolate_pose(R, -R @ c0, R, -R @ c1, 2.0)
    np.testing.assert_allclose(R2, R, atol=1e-12)
    np.testing.assert_allclose(opf.camera_centre(R2, t2), c1 + 2 * (c1 - c0), atol=1e-12)


def test_extrapolate_orbit_rotation():
    # orbit poses k-1, k: the rotation part of the extrapolation is pose
    # k+1's (a constant-rate turn about the world y axis); the centre moves
    # along the chord: 2 c_k - c_{k-1}
    cams = synthetic.orbit_cameras(36, 4.0, 64, 64)
    for k in (1, 10, 35):
        Rp, tp = _rt(cams[k - 1])
        Rc, tc = _rt(cams[k])
        Rn, _ = _rt(cams[(k + 1) % 36])
        R2, t2 = opf.extrapolate_pose(Rp, tp, Rc, tc, 1.0)
        np.testing.assert_allclose(R2, Rn, atol=1e-6)
        cp, cc = opf.camera_centre(Rp, tp), opf.camera_centre(Rc, tc)
        np.testing.assert_allclose(opf.camera_centre(R2, t2), 2 * cc - cp, atol=1e-5)


def test_extrapolate_special_steps():
    a, b = synthetic.look_at((1.0, 0.5, -4.0)), synthetic.look_at((1.4, 0.2, -3.7))
    Rp, tp = _rt(a)
    Rc, tc = _rt(b)
    R0, t0 = opf.extrapolate_pose(Rp, tp, Rc, tc, 0.0)
    np.testing.assert_allclose(R0, Rc, atol=1e-12)
    # (the float32 rotations are orthonormal to ~1e-7, so t = -R c holds to that)
    np.testing.assert_allclose(t0, tc, atol=1e-6)
    Rm, tm = opf.extrapolate_pose(Rp, tp, Rc, tc, -1.0)
    np.testing.assert_allclose(Rm, Rp, atol=1e-6)
    np.testing.assert_allclose(tm, tp, atol=1e-6)
    # half a step twice equals one step
    Rh, th = opf.extrapolate_pose(Rp, tp, Rc, tc, 0.5)
    R1, t1 = opf.extrapolate_pose(Rp, tp, Rc, tc, 1.0)
    R11, t11 = opf.extrapolate_pose(Rc, tc, Rh, th, 1.0)
    np.testing.assert_allclose(R11, R1, atol=1e-6)
    np.testing.assert_allclose(t11, t1, atol=1e-6)
    # a quarter turn about z per frame, by the rotation-vector rule
    Rz = lambda a_: np.array([[math.cos(a_), -math.sin(a_), 0], [math.sin(a_), math.cos(a_), 0],
                              [0, 0, 1.0]])
    R3, _ = opf.extrapolate_pose(np.eye(3), np.zeros(3), Rz(math.pi / 2), np.zeros(3), 1.0)
    np.testing.assert_allclose(R3, Rz(math.pi), atol=1e-12)


def test_plan_hand_worked():
    cnt = [5, 5, 5, 5, 5, 9]
    # 3 slots, empty: needs fill the lowest slots, then one prediction fits
    sc, ss, loads, nd = opf.plan([-1, -1, -1], [0, 0, 0], cnt, 8, [2, 0], [4, 1], 1)
    assert loads == [(2, 0), (0, 1), (4, 2)] and nd == 2 and sc == [2, 0, 4]
    # next frame needs 0 and 1: 0 is resident and held; 1 evicts the
    # unpredicted slot of the lower (stamp, index) among slots 0 and 2 (both
    # stamped 1): slot 0; prediction 3 then takes slot 2 (stamped 1 < 2)
    sc, ss, loads, nd = opf.plan(sc, ss, cnt, 8, [0, 1], [3], 2)
    assert loads == [(1, 0), (3, 2)] and nd == 1 and sc == [1, 0, 3] and ss == [2, 2, 2]
    # a demand load prefers an unpredicted victim even if it is newer
    sc, ss, loads, nd = opf.plan([0, 1, 2], [5, 1, 3], cnt, 8, [4], [1, 2], 6)
    assert loads == [(4, 0)] and nd == 1
    # an oversize cluster is refused
    try:
        opf.plan([-1], [0], cnt, 8, [5], [], 1)
        raise AssertionError("accepted an oversize cluster")
    except ValueError:
        pass


def test_plan_invariants_on_random_sequences():
    rng = np.random.default_rng(3)
    K, S = 12, 5
    cnt = rng.integers(0, 100, K)
    sc, ss = [-1] * S, [0] * S
    for frame in range(1, 400):
        need = list(rng.choice(K, size=int(rng.integers(1, 4)), replace=False))
        want = list(rng.choice(K, size=int(rng.integers(0, 5)), replace=False))
        before = list(sc)
        sc, ss, loads, nd = opf.plan(sc, ss, cnt, 100, need, want, frame)
        assert all(c in sc for c in need)
        assert len(set(c for c in sc if c >= 0)) == len([c for c in sc if c >= 0])
        assert [c for c, _ in loads[:nd]] == [c for c in need if c not in before]
        for c, s in loads:
            assert sc[s] == c and ss[s] == frame
        # a load never replaced a cluster needed this frame
        for c, s in loads:
            assert before[s] not in need or before[s] < 0
