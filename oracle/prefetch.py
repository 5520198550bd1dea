"""Scene prefetching (Sec. 3.3 "Scene Prefetching"), in float64 (test
infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use the oracle).

The paper predicts future camera poses by linear extrapolation and loads the
clusters those poses select ahead of time on a dedicated stream.  Readings:
extrapolation is linear in the camera centre and in the rotation's tangent
space (the relative rotation from the previous frame to the current one,
applied s more times as a rotation vector scaled by s); the resident set is
a fixed number of equal slots beside the always-resident shared segment,
filled by the policy written out in plan() (demand loads first, then the
predicted clusters, least recently used slots evicted first).
"""
from __future__ import annotations

import numpy as np
from scipy.spatial.transform import Rotation


def camera_centre(R, t):
    return -np.asarray(R, np.float64).T @ np.asarray(t, np.float64)


def extrapolate_pose(R_prev, t_prev, R_cur, t_cur, s: float):
    """(R, t) of the pose s frames after the current one."""
    Rp, Rc = np.asarray(R_prev, np.float64), np.asarray(R_cur, np.float64)
    cp, cc = camera_centre(Rp, t_prev), camera_centre(Rc, t_cur)
    c = cc + s * (cc - cp)
    rel = Rotation.from_matrix(Rc @ Rp.T).as_rotvec()
    R = Rotation.from_rotvec(s * rel).as_matrix() @ Rc
    return R, -R @ c


def plan(slot_cluster, slot_stamp, cluster_count, slot_cap, need, want, frame):
    """One frame of resident-set planning.  Returns (new slot_cluster, new
    slot_stamp, loads [(cluster, slot)], number of demand loads).

    Policy: a needed cluster already resident keeps its slot and is stamped
    with the frame; a needed cluster that is not resident goes to the lowest
    empty slot, else evicts the slot, among those not holding a needed
    cluster, that ranks first by (its cluster is predicted, stamp, index);
    then each predicted cluster, in order, that is not resident goes to the
    lowest empty slot, else evicts the lowest (stamp, index) slot that holds
    neither a needed nor a predicted cluster nor anything stamped this frame;
    the first predicted cluster without such a slot ends the planning."""
    sc = list(slot_cluster)
    ss = list(slot_stamp)
    S = len(sc)
    for c in list(need) + list(want):
        if cluster_count[c] > slot_cap:
            raise ValueError("cluster larger than a slot")
    if len(set(need)) > S:
        raise ValueError("more needed clusters than slots")
    held = set()
    loads = []

    def resident(c):
        return c in sc

    for c in need:
        if resident(c):
            held.add(sc.index(c))
            ss[sc.index(c)] = frame

    def put(c, s):
        sc[s] = c
        ss[s] = frame
        held.add(s)
        loads.append((c, s))

    for c in need:
        if resident(c):
            continue
        empty = [s for s in range(S) if sc[s] < 0]
        if empty:
            put(c, empty[0])
            continue
        cand = [s for s in range(S) if s not in held]
        put(c, min(cand, key=lambda s: (sc[s] in want, ss[s], s)))
    n_demand = len(loads)
    for c in want:
        if resident(c):
            held.add(sc.index(c))
            continue
        empty = [s for s in range(S) if sc[s] < 0]
        if empty:
            put(c, empty[0])
            continue
        cand = [s for s in range(S) if s not in held and sc[s] not in want and ss[s] < frame]
        if not cand:
            break
        put(c, min(cand, key=lambda s: (ss[s], s)))
    return sc, ss, loads, n_demand
