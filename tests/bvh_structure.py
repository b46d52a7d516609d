"""Structure checks of a multiple-threaded BVH in the layout of the C ABI
(six preorder node arrays of 4 words, triangles of 12 words), shared by the
host-build and GPU-build tests."""
import numpy as np


def f32(words):
    return words.view(np.float32)


def decode(nodes_s, info):
    """Dequantised boxes (float64), leaf flags, leaf ranges and next-on-miss links."""
    w = nodes_s.astype(np.int64)
    q = np.stack([w[:, 0] & 0xffff, w[:, 1] & 0xffff, w[:, 2] & 0xffff,
                  w[:, 0] >> 16, w[:, 1] >> 16, w[:, 2] >> 16], 1).astype(np.float64)
    g0 = np.asarray(info["grid_lo"], np.float64)
    gs = np.asarray(info["grid_step"], np.float64)
    lo = g0 + q[:, 0:3] * gs
    hi = g0 + q[:, 3:6] * gs
    leaf = (w[:, 3] >> 31) != 0
    first = (w[:, 3] >> 3) & 0x0fffffff
    cnt = w[:, 3] & 7
    n = len(w)
    skip = np.where(leaf, np.arange(n) + 1, w[:, 3])
    return lo, hi, leaf, first, cnt, skip


def _sample_points(verts, k=12, seed=0):
    """Points on each triangle, float64 [T, 3 + 3 + k, 3]: the vertices, the
    edge midpoints and k random barycentric points."""
    v = np.asarray(verts, np.float64)
    rng = np.random.default_rng(seed)
    a = rng.random((len(v), k, 1))
    b = rng.random((len(v), k, 1))
    flip = (a + b) > 1
    a, b = np.where(flip, 1 - a, a), np.where(flip, 1 - b, b)
    rnd = v[:, None, 0] + a * (v[:, None, 1] - v[:, None, 0]) + b * (v[:, None, 2] - v[:, None, 0])
    mid = 0.5 * (v[:, [0, 1, 2]] + v[:, [1, 2, 0]])
    return np.concatenate([v, mid, rnd], 1)


def check_structure(verts, nodes, tris, max_leaf, info):
    """Without spatial splits (n_refs == n_tri) every triangle is in exactly
    one leaf and inside its box.  With them a triangle may be in several
    leaves, and sample points of it (vertices, edge midpoints, random
    interior points) must each lie in the box of one of its leaves."""
    T = len(verts)
    S, n, _ = nodes.shape
    assert S == 6
    R = info.get("n_refs", T)
    assert len(tris) == R and R >= T
    # records: every original index at least once (exactly once without
    # spatial splits), each with its three vertices as given
    ids = tris[:, 9].astype(np.int64)
    if R == T:
        assert np.array_equal(np.sort(ids), np.arange(T))
    else:
        assert np.array_equal(np.unique(ids), np.arange(T))
    tf = f32(tris)
    v = verts[ids]
    assert np.array_equal(tf[:, 0:9], v.reshape(-1, 9))
    assert np.all(tris[:, 11] == 0)
    pts = None if R == T else _sample_points(verts)
    for s in range(6):
        lo, hi, is_leaf, first, cnt, skip = decode(nodes[s], info)
        assert skip[0] == n                              # root's miss link ends the walk
        assert np.all(skip > np.arange(n)) and np.all(skip <= n)
        assert np.all(cnt[is_leaf] >= 1) and np.all(cnt[is_leaf] <= max_leaf)
        # every record in exactly one leaf
        cover = np.zeros(R, np.int64)
        leaves = np.nonzero(is_leaf)[0]
        for i in leaves:
            cover[first[i]:first[i] + cnt[i]] += 1
        assert np.all(cover == 1)
        rec_leaf = np.zeros(R, np.int64)
        for i in leaves:
            rec_leaf[first[i]:first[i] + cnt[i]] = i
        if R == T:
            # each triangle inside its leaf's (padded, quantised) box
            tv = verts[ids].astype(np.float64)
            assert np.all(tv > lo[rec_leaf][:, None]) and np.all(tv < hi[rec_leaf][:, None])
        else:
            # each sample point inside the box of at least one of its triangle's leaves
            inside = np.zeros(pts.shape[:2], bool)
            for r in range(R):
                p = pts[ids[r]]
                i = rec_leaf[r]
                inside[ids[r]] |= np.all((p > lo[i]) & (p < hi[i]), axis=1)
            assert inside.all()
        # inner nodes: children are i+1 and skip[i+1]; their boxes nest
        for i in np.nonzero(~is_leaf)[0]:
            a = i + 1
            b = skip[a]
            assert skip[b] == skip[i]
            for c in (a, b):
                assert np.all(lo[c] >= lo[i]) and np.all(hi[c] <= hi[i])
            # children pre-sorted along the set's direction (centres of the
            # quantised boxes can tie; the order then follows the exact boxes)
            axis, neg = s // 2, s % 2
            ka = lo[a][axis] + hi[a][axis]
            kb = lo[b][axis] + hi[b][axis]
            tol = 4 * info["grid_step"][axis]
            assert (ka >= kb - tol) if neg else (ka <= kb + tol)
    return True


# --------------------------------------------------------------------------
# float32 model of the device walk: the box test and the watertight triangle
# test with the device's operation order and roundings, vectorised over rays.
# --------------------------------------------------------------------------
BOX_SLACK = np.float32(2.0 ** -16)   # relative slack on a box's exit distance
F32 = np.float32


def fma32(a, b, c):
    """float32 fused multiply-add: a * b + c rounded once.  The product is
    exact in float64; the float64 sum s and its exact error e (two-sum) give
    x = s + e exactly, and s rounds to float32 like x except where s is a
    float32 midpoint and e is not zero, which decides the direction."""
    a, b, c = (np.asarray(x, np.float32).astype(np.float64) for x in (a, b, c))
    with np.errstate(invalid="ignore", over="ignore"):
        p = a * b
        s = p + c
        bb = s - p
        e = (p - (s - bb)) + (c - bb)
        r = s.astype(np.float32)
        other = np.nextafter(r, np.where(s > r.astype(np.float64), np.float32(np.inf),
                                         np.float32(-np.inf)).astype(np.float32))
        mid = (r.astype(np.float64) + other.astype(np.float64)) * 0.5
        fix = (s != r.astype(np.float64)) & (s == mid) & (e != 0) & np.isfinite(s)
        up = np.maximum(r, other)
        dn = np.minimum(r, other)
        return np.where(fix, np.where(e > 0, up, dn), r).astype(np.float32)


def link_sets(d):
    ax = np.abs(d)
    x = (ax[:, 0] >= ax[:, 1]) & (ax[:, 0] >= ax[:, 2])
    y = ~x & (ax[:, 1] >= ax[:, 2])
    axis = np.where(x, 0, np.where(y, 1, 2))
    neg = d[np.arange(len(d)), axis] < 0
    return 2 * axis + neg


def walker_consts(info, o, d):
    """Per-ray slab constants: s = qstep / d and b = (qlo - o) / d with the
    reciprocal, product and difference each rounded to float32."""
    qlo = np.asarray(info["grid_lo"], np.float32)
    qstep = np.asarray(info["grid_step"], np.float32)
    dd = np.where(np.abs(d) > F32(1e-30), d, np.copysign(F32(1e-30), d)).astype(np.float32)
    ix = (F32(1.0) / dd).astype(np.float32)
    s = (qstep[None] * ix).astype(np.float32)
    b = ((qlo[None] - o).astype(np.float32) * ix).astype(np.float32)
    return s, b


def box_hit32(words, s, b, tmin, tbest, slack=BOX_SLACK):
    """words [n, 3] uint32 (lo | hi << 16 per axis); s, b [n, 3]; tmin, tbest [n]."""
    w = words.astype(np.int64)
    lo, hi = (w & 0xffff).astype(np.float32), (w >> 16).astype(np.float32)
    back = s < 0
    near = np.where(back, hi, lo)
    far = np.where(back, lo, hi)
    tn = np.maximum(fma32(near, s, b).max(1), tmin)
    tf = np.minimum(fma32(far, s, b).min(1), tbest)
    if float(slack) == 0.0:
        return tn <= tf
    return tn <= fma32(np.abs(tf), slack, tf)


def ray_shear32(d):
    """(kx, ky, kz, sx, sy, sz) per ray: kz the major axis of d (ties x, y, z),
    kx = kz + 1, ky = kz + 2 (mod 3), sx = d_kx / d_kz, sy = d_ky / d_kz,
    sz = 1 / d_kz, each rounded once."""
    d = np.asarray(d, np.float32)
    r = np.arange(len(d))
    ad = np.abs(d)
    kz = np.where((ad[:, 0] >= ad[:, 1]) & (ad[:, 0] >= ad[:, 2]), 0, np.where(ad[:, 1] >= ad[:, 2], 1, 2))
    kx, ky = (kz + 1) % 3, (kz + 2) % 3
    with np.errstate(divide="ignore", invalid="ignore"):
        dz = d[r, kz]
        return kx, ky, kz, d[r, kx] / dz, d[r, ky] / dz, (F32(1.0) / dz).astype(np.float32)


def kahan32(a, b, c, d):
    """a b - c d as the device forms it: w = c d, e = fma(-c, d, w),
    f = fma(a, b, -w), f + e."""
    w = (np.asarray(c, np.float32) * np.asarray(d, np.float32)).astype(np.float32)
    e = fma32(-np.asarray(c, np.float32), d, w)
    f = fma32(a, b, -w)
    return (f + e).astype(np.float32)


def wt32(o, d, tri):
    """Watertight test of rays o, d [n, 3] against triangles tri [n, 9]
    (v0, v1, v2): (hit mask, t, (U, V, W)), float32 with the device's operation
    order (the mask leaves the interval test to the caller)."""
    o, d, tri = (np.asarray(x, np.float32) for x in (o, d, tri))
    r = np.arange(len(o))
    kx, ky, kz, sx, sy, sz = ray_shear32(d)
    x, y, z = [], [], []
    with np.errstate(invalid="ignore", over="ignore", divide="ignore"):
        for i in range(3):
            a = (tri[:, 3 * i:3 * i + 3] - o).astype(np.float32)
            x.append(fma32(-sx, a[r, kz], a[r, kx]))
            y.append(fma32(-sy, a[r, kz], a[r, ky]))
            z.append(a[r, kz])
        U = kahan32(x[2], y[1], y[2], x[1])
        V = kahan32(x[0], y[2], y[0], x[2])
        W = kahan32(x[1], y[0], y[1], x[0])
        neg = (U < 0) | (V < 0) | (W < 0)
        pos = (U > 0) | (V > 0) | (W > 0)
        det = ((U + V).astype(np.float32) + W).astype(np.float32)
        ok = ~(neg & pos) & (det != 0)
        z0, z1, z2 = ((sz * zi).astype(np.float32) for zi in z)
        T = fma32(W, z2, fma32(V, z1, (U * z0).astype(np.float32)))
        t = (T / det).astype(np.float32)
    return ok, t, (U, V, W)


def walk32(nodes, tris, info, rays, sets=None, slack=BOX_SLACK):
    """Stackless walk of each ray (link set by direction unless given), in
    lockstep over the rays: the device's step() with the float32 box test.
    Returns (closest original index or -1, t, box tests per ray)."""
    rays = np.asarray(rays, np.float32)
    n_r = len(rays)
    o, d = rays[:, 0:3], rays[:, 4:7]
    tmin = rays[:, 3].copy()
    tb = rays[:, 7].copy()
    s, b = walker_consts(info, o, d)
    sets = link_sets(d) if sets is None else np.broadcast_to(np.asarray(sets), (n_r,))
    tf32 = f32(tris)
    ids = tris[:, 9].astype(np.int64)
    n = nodes.shape[1]
    i = np.zeros(n_r, np.int64)
    best = np.full(n_r, -1, np.int64)
    boxes = np.zeros(n_r, np.int64)
    while True:
        act = np.nonzero(i < n)[0]
        if len(act) == 0:
            break
        q = nodes[sets[act], i[act]]
        leaf = (q[:, 3] >> 31) != 0
        hit = box_hit32(q[:, 0:3], s[act], b[act], tmin[act], tb[act], slack)
        boxes[act] += 1
        lh = act[hit & leaf]
        if len(lh):
            ql = nodes[sets[lh], i[lh]][:, 3].astype(np.int64)
            first, cnt = (ql >> 3) & 0x0fffffff, ql & 7
            for k in range(int(cnt.max())):
                sel = k < cnt
                r = lh[sel]
                j = first[sel] + k
                ok, t, _ = wt32(o[r], d[r], tf32[j, 0:9])
                idx = ids[j]
                acc = ok & (t > tmin[r]) & ((t < tb[r]) | ((t == tb[r]) & (best[r] >= 0) & (idx < best[r])))
                tb[r[acc]] = t[acc]
                best[r[acc]] = idx[acc]
        nxt = np.where(hit | leaf, i[act] + 1, q[:, 3].astype(np.int64))
        i[act] = nxt
    t_out = np.where(best >= 0, tb, np.float32(np.inf))
    return best, t_out, boxes
