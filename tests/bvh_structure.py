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


def check_structure(verts, nodes, tris, max_leaf, info):
    T = len(verts)
    S, n, _ = nodes.shape
    assert S == 6
    # triangles: every original index exactly once, edges = fl32(v - v0)
    ids = tris[:, 9].astype(np.int64)
    assert np.array_equal(np.sort(ids), np.arange(T))
    tf = f32(tris)
    v = verts[ids]
    assert np.array_equal(tf[:, 0:3], v[:, 0])
    assert np.array_equal(tf[:, 3:6], (v[:, 1] - v[:, 0]).astype(np.float32))
    assert np.array_equal(tf[:, 6:9], (v[:, 2] - v[:, 0]).astype(np.float32))
    for s in range(6):
        lo, hi, is_leaf, first, cnt, skip = decode(nodes[s], info)
        assert skip[0] == n                              # root's miss link ends the walk
        assert np.all(skip > np.arange(n)) and np.all(skip <= n)
        assert np.all(cnt[is_leaf] >= 1) and np.all(cnt[is_leaf] <= max_leaf)
        # every triangle in exactly one leaf, inside its (padded, quantised) box
        cover = np.zeros(T, np.int64)
        for i in np.nonzero(is_leaf)[0]:
            cover[first[i]:first[i] + cnt[i]] += 1
            tv = verts[ids[first[i]:first[i] + cnt[i]]].reshape(-1, 3).astype(np.float64)
            assert np.all(tv > lo[i]) and np.all(tv < hi[i])
        assert np.all(cover == 1)
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
