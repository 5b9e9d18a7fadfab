"""Pins of the view-order oracle (Sec. 3.5, App. A) against facts that do not
come from the oracle itself: the unique optimum of a line, the single
direction switch forced by a large direction weight, group contiguity and
the shortest group path on well-separated groups (brute force), the k-means
fixed point and 2-opt local optimality (checked by brute force over every
move), and permutation validity."""
import itertools
import math

import numpy as np

from oracle.ordering import view_order
from paper_2605_20150_amd import synth


def cam(eye, fwd):
    eye = np.asarray(eye, float)
    return synth.look_at(eye, eye + np.asarray(fwd, float), (0, 0, 1), 64, 64, 50.0)


def rows(cams):
    return synth.cams_array(cams)


def centre(c):
    return -np.asarray(c.R).T @ np.asarray(c.t)


def path_len(order, D):
    return sum(D(a, b) for a, b in zip(order, order[1:]))


def test_line_from_its_end_is_visited_in_order():
    xs = [0.0, 7.0, 3.0, 9.0, 1.0, 4.0, 8.0, 2.0, 6.0]
    cams = [cam((x, 0.0, 1.7), (0, 1, 0)) for x in xs]
    order = view_order(rows(cams), cluster_size=len(xs), dir_weight=0.0)
    assert [xs[i] for i in order] == sorted(xs)


def test_large_direction_weight_switches_direction_once():
    """Views 0-5 face +x and 6-11 face -x at the same six positions: with a
    large weight the only optimal open path from view 0 walks the +x row,
    turns once and walks the -x row back."""
    cams = [cam((float(x), 0.0, 1.7), (1, 0, 0)) for x in range(6)]
    cams += [cam((float(x), 0.0, 1.7), (-1, 0, 0)) for x in range(6)]
    order = view_order(rows(cams), cluster_size=12, dir_weight=100.0)
    assert order == [0, 1, 2, 3, 4, 5, 11, 10, 9, 8, 7, 6]
    # without the direction term the co-located pairs are free to interleave
    flat = view_order(rows(cams), cluster_size=12, dir_weight=0.0)
    switches = sum((a < 6) != (b < 6) for a, b in zip(flat, flat[1:]))
    assert switches > 1


def test_separated_groups_stay_contiguous_on_a_shortest_group_path():
    rng = np.random.default_rng(3)
    corners = np.array([[0, 0], [1000, 0], [1000, 1400], [0, 1400.0]])
    cams, group = [], []
    # view 0 in group 2; groups listed in a scrambled order
    for g in (2, 0, 3, 1):
        for _ in range(6):
            xy = corners[g] + rng.normal(0, 5, size=2)
            cams.append(cam((xy[0], xy[1], 1.7), rng.normal(size=3) * [1, 1, 0] + [0, 0, 1e-3]))
            group.append(g)
    order = view_order(rows(cams), cluster_size=6, dir_weight=10.0)
    seq = [group[i] for i in order]
    runs = [g for g, _ in itertools.groupby(seq)]
    assert len(runs) == 4 and sorted(runs) == [0, 1, 2, 3]
    cen = {g: np.mean([centre(c) for c, gg in zip(cams, group) if gg == g], axis=0) for g in range(4)}
    best = min(path_len((2,) + p, lambda a, b: np.linalg.norm(cen[a] - cen[b]))
               for p in itertools.permutations([0, 1, 3]))
    got = path_len(runs, lambda a, b: np.linalg.norm(cen[a] - cen[b]))
    assert got <= best + 1e-6


def street_views(n, seed):
    rng = np.random.default_rng(seed)
    cams = []
    for _ in range(n):
        eye = (rng.uniform(-200, 200), rng.uniform(-200, 200), 1.7)
        a = rng.uniform(0, 2 * np.pi)
        cams.append(cam(eye, (math.cos(a), math.sin(a), 0.0)))
    return cams


def test_kmeans_fixed_point_and_two_opt_local_optimality():
    cams = street_views(90, 5)
    R = rows(cams)
    w = 25.0
    order, groups, assign, cent = view_order(R, cluster_size=12, dir_weight=w, details=True)
    assert sorted(order) == list(range(90)) and order[0] == 0
    P = np.array([centre(c) for c in cams])
    F = np.array([np.asarray(c.R)[2] for c in cams])
    # k-means fixed point: centroids are member means, every view is nearest its own
    for m, c in enumerate(cent):
        mine = [i for i in range(90) if assign[i] == m]
        if mine:
            assert np.allclose(c, P[mine].mean(axis=0), atol=1e-9)
    for i in range(90):
        dd = [np.sum((P[i] - np.asarray(c)) ** 2) for c in cent]
        assert dd[assign[i]] <= min(dd) + 1e-9
    # each group is one cluster, visited contiguously
    for g in groups:
        assert len({assign[i] for i in g}) == 1

    def D(i, j):
        return np.linalg.norm(P[i] - P[j]) + w * np.linalg.norm(F[i] - F[j])

    # no 2-opt move (first element fixed) shortens any group's path
    for g in groups:
        base = path_len(g, D)
        for i in range(1, len(g) - 1):
            for j in range(i + 1, len(g)):
                alt = g[:i] + g[i:j + 1][::-1] + g[j + 1:]
                assert path_len(alt, D) >= base - 1e-6
    # the cluster path is 2-opt optimal over the centroids too
    seq = [assign[g[0]] for g in groups]

    def Dc(a, b):
        return np.linalg.norm(np.asarray(cent[a]) - np.asarray(cent[b]))

    base = path_len(seq, Dc)
    for i in range(1, len(seq) - 1):
        for j in range(i + 1, len(seq)):
            alt = seq[:i] + seq[i:j + 1][::-1] + seq[j + 1:]
            assert path_len(alt, Dc) >= base - 1e-6


def test_degenerate_inputs():
    assert view_order([], 4, 1.0) == []
    one = [cam((1.0, 2.0, 1.7), (1, 0, 0))]
    assert view_order(rows(one), 4, 1.0) == [0]
    # duplicates: more clusters than distinct positions leaves some empty
    dup = [cam((0.0, 0.0, 1.7), (1, 0, 0)) for _ in range(5)]
    assert sorted(view_order(rows(dup), 1, 0.0)) == list(range(5))
