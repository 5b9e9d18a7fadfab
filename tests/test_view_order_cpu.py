"""The library's view order (tide_view_order, host code) against the
oracle's, permutation for permutation: street-level and aerial view sets,
several cluster sizes and direction weights, a ragged last cluster, one
cluster, one view per cluster, and the degenerate cases."""
import math

import numpy as np
import pytest

from oracle.ordering import view_order as oracle_order
from paper_2605_20150_amd import synth
from paper_2605_20150_amd.train import view_order


def street(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        eye = np.array([rng.uniform(-500, 500), rng.uniform(-500, 500), 1.7])
        a = rng.uniform(0, 2 * np.pi)
        out.append(synth.look_at(eye, eye + [math.cos(a), math.sin(a), 0.0], (0, 0, 1), 1600, 900, 1385.6))
    return out


def aerial(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        a = rng.uniform(0, 2 * np.pi)
        eye = np.array([250 * math.cos(a), 250 * math.sin(a), 150.0 + rng.normal(0, 5)])
        out.append(synth.look_at(eye, (rng.normal(0, 20), rng.normal(0, 20), 0.0), (0, 0, 1), 1920, 1080, 1662.8))
    return out


@pytest.mark.parametrize("kind,n,s,w", [("street", 400, 16, 10.0), ("street", 397, 16, 0.0), ("street", 250, 7, 50.0),
                                        ("aerial", 400, 25, 100.0), ("aerial", 64, 64, 1.0), ("street", 30, 1, 5.0)])
def test_library_matches_oracle(kind, n, s, w):
    cams = (street if kind == "street" else aerial)(n, 7 + n)
    got = view_order(cams, cluster_size=s, dir_weight=w)
    ref = oracle_order(synth.cams_array(cams), s, w)
    assert got.tolist() == ref


def test_degenerate_and_bad_arguments():
    assert view_order([], 4, 1.0).tolist() == []
    one = street(1, 3)
    assert view_order(one, 4, 1.0).tolist() == [0]
    dup = [street(1, 3)[0]] * 6
    assert view_order(dup, 2, 0.0).tolist() == oracle_order(synth.cams_array(dup), 2, 0.0)
    with pytest.raises(RuntimeError):
        view_order(one, 0, 1.0)
    with pytest.raises(RuntimeError):
        view_order(one, 4, -1.0)
