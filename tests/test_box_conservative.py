"""The traversal's box test is conservative and the triangle test watertight
(Sec. 3.1 leaves both tests open), checked on a float32 model of the device
walk against the brute-force closest hit for rays that stress them:

* rays arriving at grazing angles (1e-1 down to 1e-6 rad) to the triangle
  they aim at, at interior points and at edges and vertices (hits on the faces
  of the leaf boxes);
* rays from origins 10^2 to 10^5 times the scene's extent away, where the
  slab distances carry an error relative to the distance travelled;
* rays from inside a closed mesh aimed exactly at its shared edges and
  vertices.

Error bounds (u = 2^-24, ext the scene extent, L a triangle's longest edge):
a slab distance fma(q, s, b) is within 4u |t| + 2u ext / |d_a| of the exact
one; the triangle test's weights are the exact barycentric coordinates of the
ray in the sheared, rounded vertices (Kahan's determinant gives the edge
functions' exact signs), so an accepted hit's point o + t d lies within
22u (|t d_a| + L) of the triangle's box along each axis a (pinned below with
exact rational arithmetic).  The padding (at least 2^-15 ext) covers the
absolute parts, the slack 2^-16 on a box's exit distance the relative ones.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from bvh_structure import BOX_SLACK, box_hit32, fma32, link_sets, ray_shear32, walk32, walker_consts, wt32
from paper_1505_06022_amd import api, scenes

U = 2.0 ** -24


def _scene(kind):
    if kind == "soup":
        return scenes.small_soup(4096, 11, spread=0.03).verts
    return scenes.box_scene(8, 8).verts


def _check(oracle_lib, verts, rays, alpha=0.0):
    """alpha > 0: a BVH with spatial splits, whose leaves hold the boxes of
    clipped parts of triangles (rounded outward, then padded like any box)."""
    nodes, tris, info = api.build_bvh_host(verts, split_alpha=alpha)
    assert (info["n_refs"] > info["n_tri"]) == (alpha > 0)
    h_ref, t_ref = oracle_lib.trace_brute_force(verts, rays)
    h, t, _ = walk32(nodes, tris, info, rays)
    bad = np.nonzero(h != h_ref)[0]
    assert len(bad) == 0, (len(bad), bad[:10])
    hit = h_ref >= 0
    assert np.array_equal(t[hit], t_ref[hit])
    return h_ref


@pytest.mark.parametrize("kind,alpha", [("soup", 0.0), ("box", 0.0), ("soup", 1e-5)])
@pytest.mark.parametrize("on_edges", [False, True])
def test_grazing_rays_walk_equals_brute_force(oracle_lib, kind, alpha, on_edges):
    verts = _scene(kind)
    angles = [1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6]
    rays = scenes.grazing_rays(verts, 3000, angles, seed=21 + on_edges, on_edges=on_edges)
    h = _check(oracle_lib, verts, rays, alpha)
    assert (h >= 0).mean() > 0.5


@pytest.mark.parametrize("kind,alpha", [("soup", 0.0), ("box", 0.0), ("soup", 1e-5)])
def test_far_origin_rays_walk_equals_brute_force(oracle_lib, kind, alpha):
    verts = _scene(kind)
    rays = scenes.far_origin_rays(verts, 2000, seed=31)
    h = _check(oracle_lib, verts, rays, alpha)
    assert (h >= 0).mean() > 0.5


def test_slack_is_needed_for_far_origins_and_covers_the_bound(oracle_lib):
    """Without the relative slack the walk loses hits of far-origin rays (the
    slab and hit-point errors grow with the distance travelled); with it,
    every box on the path of the closest hit passes when tested against
    t_best = the closest hit's t, the tightest bound the walk ever uses."""
    verts = _scene("soup")
    rays = scenes.far_origin_rays(verts, 4000, scales=(1e4, 1e5, 1e6), seed=33)
    nodes, tris, info = api.build_bvh_host(verts)
    h_ref, t_ref = oracle_lib.trace_brute_force(verts, rays)
    h0, _, _ = walk32(nodes, tris, info, rays, slack=np.float32(0.0))
    h1, _, _ = walk32(nodes, tris, info, rays)
    assert np.array_equal(h1, h_ref)
    lost = int((h0 != h_ref).sum())
    assert lost > 0, "the far-origin rays do not stress the slab error"
    # the sufficient condition, node by node: for the hit rays, every ancestor of the
    # closest triangle's leaf passes with t_best = t*
    o, d = rays[:, 0:3], rays[:, 4:7]
    s, b = walker_consts(info, o, d)
    sets = link_sets(d)
    pos = {int(k): j for j, k in enumerate(tris[:, 9])}
    for r in np.nonzero(h_ref >= 0)[0][:500]:
        leaf_pos = pos[int(h_ref[r])]
        nod = nodes[sets[r]]
        w = nod[:, 3].astype(np.int64)
        n = len(nod)
        skip = np.where((w >> 31) != 0, np.arange(n) + 1, w)
        i = 0
        while i < n:   # descend: the child whose subtree holds the leaf of the closest triangle
            ok = box_hit32(nod[i:i + 1, 0:3], s[r:r + 1], b[r:r + 1], rays[r:r + 1, 3], t_ref[r:r + 1])[0]
            assert ok, (r, i)
            if (w[i] >> 31) != 0:
                first, cnt = (w[i] >> 3) & 0x0fffffff, w[i] & 7
                assert first <= leaf_pos < first + cnt
                break
            a = i + 1
            c = skip[a]
            i = a if _holds(nod, w, skip, a, leaf_pos) else c


def _holds(nod, w, skip, i, leaf_pos):
    """Whether the subtree rooted at node i holds triangle position leaf_pos."""
    j, end = i, skip[i]
    while j < end:
        if (w[j] >> 31) != 0:
            first, cnt = (w[j] >> 3) & 0x0fffffff, w[j] & 7
            if first <= leaf_pos < first + cnt:
                return True
        j += 1
    return False


def test_box_model_matches_padding_bound():
    """The slack 2^-16 on the exit distance covers the relative error terms
    (4u per plane distance, 22u of the hit point per axis, 52u in all) four
    times over; the padding 2^-15 ext covers the absolute ones (2u ext for a
    plane distance, 22u L <= 22 sqrt(3) u ext for the hit point) more than ten
    times over."""
    assert float(BOX_SLACK) == 2.0 ** -16
    assert float(BOX_SLACK) >= 4 * (2 * (4 + 22)) * U
    assert 2.0 ** -15 >= 10 * (2 + 22 * np.sqrt(3)) * U


def _exact_sign(x):
    return (x > 0) - (x < 0)


def _sheared(o, d, tri):
    """The float32 sheared vertices (x, y) of the triangle test, per vertex."""
    kx, ky, kz, sx, sy, _ = ray_shear32(d[None])
    out = []
    for i in range(3):
        a = (tri[3 * i:3 * i + 3] - o).astype(np.float32)
        out.append((float(fma32(-sx, a[kz], a[kx])[0]), float(fma32(-sy, a[kz], a[ky])[0])))
    return out


def test_hit_point_bound_and_exact_edge_signs_exact_rational():
    """For rays at grazing angles down to 1e-7 rad, origins from 1 to 10^6
    triangle sizes away and triangles from equilateral to slivers (aspect
    1e4), against exact rational arithmetic over the same float inputs:
    * the signs of the edge functions U, V, W equal the exact signs of the
      2x2 determinants of the rounded, sheared vertices (Kahan's algorithm);
    * every accepted hit's point o + t d (t as computed) lies within
      22u (|t d_a| + L) of the triangle's box along each axis a."""
    rng = np.random.default_rng(5)
    n_ok, worst = 0, 0.0
    for trial in range(2500):
        scale = 10.0 ** rng.uniform(-3, 2)
        a = rng.standard_normal(3)
        b = rng.standard_normal(3)
        sliver = 10.0 ** -rng.uniform(0, 4)
        c = a + (b - a) * rng.random() + sliver * rng.standard_normal(3)
        v = (np.stack([a, b, c]) * scale + rng.uniform(-5, 5, 3) * scale).astype(np.float32)
        n = np.cross((v[1] - v[0]).astype(np.float64), (v[2] - v[0]).astype(np.float64))
        if not np.linalg.norm(n) > 0:
            continue
        nh = n / np.linalg.norm(n)
        g = 10.0 ** -rng.uniform(0, 7)
        w = rng.standard_normal(3)
        w -= (w @ nh) * nh
        w /= np.linalg.norm(w)
        dd = np.sqrt(1 - g * g) * w + g * nh * rng.choice([-1.0, 1.0])
        uu, vv = rng.random(2)
        if uu + vv > 1:
            uu, vv = 1 - uu, 1 - vv
        if trial % 3 == 0:       # on an edge
            vv = 0.0
        P = v[0] + uu * (v[1] - v[0]).astype(np.float64) + vv * (v[2] - v[0]).astype(np.float64)
        Ledge = max(np.linalg.norm((v[i] - v[(i + 1) % 3]).astype(np.float64)) for i in range(3))
        dist = Ledge * 10.0 ** rng.uniform(0, 6)
        o = (P - dist * dd).astype(np.float32)
        d = (dd * 10.0 ** rng.uniform(-2, 2)).astype(np.float32)
        tri = v.reshape(9)
        ok, t, (Uf, Vf, Wf) = wt32(o[None], d[None], tri[None])
        # exact signs of the edge functions of the rounded sheared vertices
        (x0, y0), (x1, y1), (x2, y2) = ((Fr(p), Fr(q)) for p, q in _sheared(o, d, tri))
        for fv, ex in ((Uf[0], x2 * y1 - y2 * x1), (Vf[0], x0 * y2 - y0 * x2), (Wf[0], x1 * y0 - y1 * x0)):
            assert _exact_sign(float(fv)) == _exact_sign(ex), trial
        if not ok[0]:
            continue
        n_ok += 1
        tf = Fr(float(t[0]))
        lo, hi = v.min(0), v.max(0)
        for ax in range(3):
            X = Fr(float(o[ax])) + tf * Fr(float(d[ax]))
            out = max(Fr(float(lo[ax])) - X, X - Fr(float(hi[ax])), Fr(0))
            bound = 22 * U * (abs(float(t[0]) * float(d[ax])) + Ledge)
            worst = max(worst, float(out) / bound)
            assert float(out) <= bound, (trial, ax, float(out), bound)
    print(f"accepted hits {n_ok}, worst out-of-box distance / bound {worst:.3f}")
    assert n_ok > 800
    assert worst < 0.5      # the bound holds with room to spare


@pytest.mark.parametrize("level,seed", [(1, 0), (2, 1), (3, 2)])
def test_closed_mesh_is_watertight_at_shared_edges_and_vertices(oracle_lib, level, seed):
    """Rays from points inside a closed icosphere aimed exactly at its
    vertices (float32) and at points of its shared edges always hit it: the
    edge functions of a shared edge have exactly opposite signs in the two
    triangles.  The float32 device model agrees with the oracle."""
    rng = np.random.default_rng(seed)
    scale = 10.0 ** rng.uniform(-2, 2)
    shift = rng.uniform(-3, 3, 3) * scale
    verts = (scenes._icosphere(level) * scale + shift).astype(np.float32)
    pts = np.unique(verts.reshape(-1, 3), axis=0)
    edges = []
    for f in verts:
        for i in range(3):
            a, b = f[i].astype(np.float64), f[(i + 1) % 3].astype(np.float64)
            for lam in (0.5, rng.random()):
                edges.append(a + lam * (b - a))
    targets = np.concatenate([pts, np.asarray(edges)]).astype(np.float32)
    n = len(targets)
    o = (shift + 0.5 * scale * rng.uniform(-1, 1, (n, 3)) / np.sqrt(3)).astype(np.float32)
    d = (targets - o).astype(np.float32)
    rays = np.zeros((n, 8), np.float32)
    rays[:, 0:3], rays[:, 4:7], rays[:, 7] = o, d, np.inf
    h, t = oracle_lib.trace_brute_force(verts, rays)
    assert (h >= 0).all(), int((h < 0).sum())
    nodes, tris, info = api.build_bvh_host(verts)
    h2, t2, _ = walk32(nodes, tris, info, rays)
    assert np.array_equal(h, h2) and np.array_equal(t, t2)


def _nearest_f32(x):
    """float32 nearest to the rational x, ties to even."""
    lo = np.float32(float(x))
    cand = {lo, np.nextafter(lo, np.float32(np.inf)), np.nextafter(lo, np.float32(-np.inf))}
    return min(cand, key=lambda y: (abs(Fr(float(y)) - x), int(np.float32(y).view(np.uint32)) & 1))


def test_fma32_rounds_once_against_exact_rational():
    """The model's fused multiply-add equals the correctly rounded a b + c,
    also where the float64 sum lands on a float32 midpoint with a tail that
    decides the direction."""
    rng = np.random.default_rng(3)
    a = rng.standard_normal(3000).astype(np.float32)
    b = rng.standard_normal(3000).astype(np.float32)
    c = (-(a.astype(np.float64) * b) * (1 + rng.standard_normal(3000) * 1e-6)).astype(np.float32)
    # (1 + 2^-12)^2 = 1 + 2^-11 + 2^-24; with c = -2^-11 the sum is 1 + 2^-24,
    # a midpoint of float32 at 1, and c's low bits move it off the midpoint
    p = np.float32(1.0 + 2.0 ** -12)
    c2 = np.asarray([-2.0 ** -11, -(2.0 ** -11 + 2.0 ** -34), -(2.0 ** -11 - 2.0 ** -34), 2.0 ** -60], np.float32)
    a = np.concatenate([a, np.full(4, p)])
    b = np.concatenate([b, np.full(4, p)])
    c = np.concatenate([c, c2])
    got = fma32(a, b, c)
    for i in range(len(a)):
        x = Fr(float(a[i])) * Fr(float(b[i])) + Fr(float(c[i]))
        assert got[i] == _nearest_f32(x), (i, a[i], b[i], c[i])
