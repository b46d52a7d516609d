"""Pins of the oracle's closest-hit definition and of its independent BVH.

* The watertight triangle test in float32 against an exact rational solve of
  o + t d = v0 + u e1 + v e2 (Cramer's rule over Fractions) on random
  rays and triangles, wherever the exact answer is not within rounding of a
  boundary.
* Analytic t for axis-aligned triangles; open interval (tmin, tmax); ties to
  the lower triangle index.
* The oracle BVH returns exactly what brute force returns.
"""
from fractions import Fraction

import numpy as np
import pytest

from paper_1505_06022_amd import scenes


def _exact(o, d, tri):
    F = [Fraction(float(x)) for x in o], [Fraction(float(x)) for x in d]
    o, d = F
    v0, v1, v2 = ([Fraction(float(x)) for x in v] for v in tri)
    e1 = [v1[i] - v0[i] for i in range(3)]
    e2 = [v2[i] - v0[i] for i in range(3)]
    s = [o[i] - v0[i] for i in range(3)]
    # columns: -d, e1, e2 ; unknowns t, u, v
    cols = [[-d[i] for i in range(3)], e1, e2]

    def det3(c0, c1, c2):
        return (c0[0] * (c1[1] * c2[2] - c1[2] * c2[1]) - c1[0] * (c0[1] * c2[2] - c0[2] * c2[1])
                + c2[0] * (c0[1] * c1[2] - c0[2] * c1[1]))
    D = det3(*cols)
    if D == 0:
        return None
    t = det3(s, cols[1], cols[2]) / D
    u = det3(cols[0], s, cols[2]) / D
    v = det3(cols[0], cols[1], s) / D
    return t, u, v


def test_triangle_test_against_exact_rational_solve(oracle_lib):
    rng = np.random.default_rng(1)
    ntri, nray = 24, 150
    verts = rng.uniform(-1, 1, (ntri, 3, 3)).astype(np.float32)
    rays = np.zeros((nray, 8), np.float32)
    rays[:, :3] = rng.uniform(-2, 2, (nray, 3))
    tgt = rng.uniform(-0.5, 0.5, (nray, 3))
    d = tgt - rays[:, :3]
    rays[:, 4:7] = d / np.linalg.norm(d, axis=1, keepdims=True)
    rays[:, 7] = np.inf
    hit, t = oracle_lib.trace_brute_force(verts, rays)
    checked = hits = 0
    for r in range(nray):
        cands = []
        ambiguous = False
        for i in range(ntri):
            ex = _exact(rays[r, :3], rays[r, 4:7], verts[i])
            if ex is None:
                continue
            tt, u, v = ex
            margin = min(u, v, 1 - u - v)
            if abs(margin) < 1e-4 or abs(tt) < 1e-4:
                ambiguous = True
                continue
            if margin > 0 and tt > 0:
                cands.append((float(tt), i))
        cands.sort()
        if ambiguous or (len(cands) > 1 and cands[1][0] - cands[0][0] < 1e-4):
            continue
        checked += 1
        if not cands:
            assert hit[r] == -1 and np.isinf(t[r])
        else:
            hits += 1
            assert hit[r] == cands[0][1]
            assert abs(t[r] - cands[0][0]) <= 1e-5 * cands[0][0]
    assert checked > 100 and hits > 20


def test_axis_aligned_triangle_exact_t(oracle_lib):
    verts = np.array([[[0, 0, 3], [1, 0, 3], [0, 1, 3]]], np.float32)
    rays = np.array([[0.25, 0.25, 0, 0, 0, 0, 1, np.inf],
                     [0.25, 0.25, 0, 0, 0, 0, 2, np.inf],
                     [0.25, 0.25, 5, 0, 0, 0, -1, np.inf],
                     [0.75, 0.75, 0, 0, 0, 0, 1, np.inf]], np.float32)
    hit, t = oracle_lib.trace_brute_force(verts, rays)
    assert list(hit) == [0, 0, 0, -1]
    assert t[0] == 3.0 and t[1] == 1.5 and t[2] == 2.0 and np.isinf(t[3])


def test_open_interval_and_ties(oracle_lib):
    tri = [[0, 0, 2], [1, 0, 2], [0, 1, 2]]
    verts = np.array([tri, [[0, 0, 5], [1, 0, 5], [0, 1, 5]], tri, tri], np.float32)
    base = [0.2, 0.2, 0, 0, 0, 0, 1, np.inf]
    rays = np.array([base,
                     base[:7] + [2.0],          # tmax == t: excluded
                     base[:7] + [2.0001],
                     base[:3] + [2.0] + base[4:],  # tmin == t: excluded -> next at 5
                     ], np.float32)
    hit, t = oracle_lib.trace_brute_force(verts, rays)
    assert hit[0] == 0 and t[0] == 2.0         # three coincident copies: lowest index
    assert hit[1] == -1
    assert hit[2] == 0
    assert hit[3] == 1 and t[3] == 5.0


@pytest.mark.parametrize("seed,n", [(0, 17), (1, 100), (2, 700), (3, 3000)])
def test_oracle_bvh_equals_brute_force(oracle_lib, seed, n):
    sc = scenes.small_soup(n, seed, spread=0.5 / np.cbrt(n))
    # some degenerate (zero-area) and axis-aligned triangles
    sc.verts[::13, 2] = sc.verts[::13, 1]
    sc.verts[1::17, :, 2] = sc.verts[1::17, 0:1, 2]
    rays = np.concatenate([scenes.random_rays(2000, seed), scenes.pinhole_rays(
        scenes.Camera((0.5, 0.5, -1.5), (0.5, 0.5, 0.5), (0, 1, 0), 0.5, 40, 30))])
    rays[::7, 4:7] = np.array([0, 0, 1], np.float32)   # axis-parallel directions
    o_bvh = oracle_lib.OracleScene(sc, use_bvh=True)
    h1, t1 = o_bvh.trace(rays)
    h2, t2 = o_bvh.trace(rays, brute_force=True)
    assert np.array_equal(h1, h2)
    assert np.array_equal(t1, t2)
    assert (h1 >= 0).mean() > 0.05


def test_oracle_bvh_equals_brute_force_on_soup_subset(oracle_lib):
    sc = scenes.soup_scene(1 << 15, seed=4)
    rays = np.concatenate([scenes.random_rays(3000, 4), scenes.pinhole_rays(
        scenes.Camera((0.5, 0.5, -1.5), (0.5, 0.5, 0.5), (0, 1, 0), 0.4, 64, 36))])
    o = oracle_lib.OracleScene(sc, use_bvh=True)
    h1, t1 = o.trace(rays)
    h2, t2 = o.trace(rays, brute_force=True)
    assert np.array_equal(h1, h2) and np.array_equal(t1, t2)
