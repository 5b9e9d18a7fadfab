"""View-order oracle -- TEST INFRASTRUCTURE ONLY (plain Python, float64).

The training-view order of Sec. 3.5 and App. A: a clustered
travelling-salesperson order of the camera poses.  The paper names the
method without its parts; the steps below are the reading the tests hold the
library to:

  d(i, j) = |p_i - p_j| + w |f_i - f_j|        p centre, f viewing direction
  k = ceil(n / s) clusters of the centres       farthest-point seeds from view
                                                0, Lloyd until stable (<= 100)
  cluster path over centroids from view 0's     nearest neighbour, then 2-opt
  cluster                                       with the first element fixed
  path inside each cluster, entered at the      nearest neighbour, then 2-opt
  view nearest the previous cluster's last

Ties go to the lower index; a 2-opt move must gain more than 1e-9.
Cameras are rows of ``synth.cams_array``: R (9, row-major, world to camera),
t (3), ...
"""
from __future__ import annotations

import math


def _centre_and_direction(row):
    R = [float(x) for x in row[0:9]]
    t = [float(x) for x in row[9:12]]
    # centre c = -R^T t (world to camera is x_c = R x + t); direction = R's row 3
    c = (-(R[0] * t[0] + R[3] * t[1] + R[6] * t[2]),
         -(R[1] * t[0] + R[4] * t[1] + R[7] * t[2]),
         -(R[2] * t[0] + R[5] * t[1] + R[8] * t[2]))
    return c, (R[6], R[7], R[8])


def _sq(a, b):
    dx, dy, dz = a[0] - b[0], a[1] - b[1], a[2] - b[2]
    return dx * dx + dy * dy + dz * dz


def _len(a, b):
    return math.sqrt(_sq(a, b))


def _nearest_neighbour_path(items, start, cost):
    path = [start]
    left = [x for x in items if x != start]
    while left:
        here = path[-1]
        pick = min(range(len(left)), key=lambda a: (cost(here, left[a]), a))
        path.append(left.pop(pick))
    return path


def _two_opt(path, cost):
    """Reverse path[i..j] (i >= 1) while that shortens the open path."""
    m = len(path)
    changed = True
    while changed:
        changed = False
        for i in range(1, m - 1):
            for j in range(i + 1, m):
                old = cost(path[i - 1], path[i])
                new = cost(path[i - 1], path[j])
                if j + 1 < m:
                    old += cost(path[j], path[j + 1])
                    new += cost(path[i], path[j + 1])
                if new < old - 1e-9:
                    path[i:j + 1] = path[i:j + 1][::-1]
                    changed = True
    return path


def view_order(cams, cluster_size: int, dir_weight: float, details: bool = False):
    """Permutation of the cameras (rows of cams).  With details, also the
    clusters in visiting order (each its views in visiting order), the
    cluster assignment and the centroids."""
    n = len(cams)
    if n == 0:
        return ([], [], [], []) if details else []
    cf = [_centre_and_direction(r) for r in cams]
    P = [c for c, _ in cf]
    F = [f for _, f in cf]
    w = float(dir_weight)

    def d(i, j):
        return _len(P[i], P[j]) + w * _len(F[i], F[j])

    k = -(-n // cluster_size)
    # farthest-point seeds
    cent = [P[0]]
    near = [_sq(p, cent[0]) for p in P]
    while len(cent) < k:
        far = max(range(n), key=lambda i: (near[i], -i))
        cent.append(P[far])
        near = [min(near[i], _sq(P[i], cent[-1])) for i in range(n)]
    # Lloyd iterations
    assign = [-1] * n
    for _ in range(100):
        new = [min(range(k), key=lambda m: (_sq(P[i], cent[m]), m)) for i in range(n)]
        if new == assign:
            break
        assign = new
        for m in range(k):
            mine = [i for i in range(n) if assign[i] == m]
            if mine:
                sx = sy = sz = 0.0
                for i in mine:
                    sx += P[i][0]
                    sy += P[i][1]
                    sz += P[i][2]
                cnt = float(len(mine))
                cent[m] = (sx / cnt, sy / cnt, sz / cnt)
    members = {m: [i for i in range(n) if assign[i] == m] for m in range(k)}
    used = [m for m in range(k) if members[m]]
    tour = _two_opt(_nearest_neighbour_path(used, assign[0], lambda a, b: _len(cent[a], cent[b])),
                    lambda a, b: _len(cent[a], cent[b]))
    order, groups, prev = [], [], None
    for m in tour:
        views = members[m]
        if prev is None:
            entry = 0
        else:
            entry = min(views, key=lambda i: (d(prev, i), i))
        path = _two_opt(_nearest_neighbour_path(views, entry, d), d)
        groups.append(path)
        order.extend(path)
        prev = path[-1]
    if details:
        return order, groups, assign, cent
    return order
