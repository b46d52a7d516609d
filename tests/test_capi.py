"""The C ABI on the CPU: the library loads, exports every declared symbol,
validates arguments on the host, and its host-built multiple-threaded BVH has
the structure the traversal relies on (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from bvh_structure import check_structure, decode, f32, wt32
from paper_1505_06022_amd import api, scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "pm.h")).read()
    return sorted(set(re.findall(r"PM_API\s+[\w\s\*]*?\b(pm_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = api.lib()
    decl = _declared_symbols()
    assert len(decl) >= 15
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(api.EXPORTS) == decl
    assert api.abi_version() == 2


def test_host_validation_errors_without_gpu():
    L = api.lib()
    v = np.zeros((1, 3, 3), np.float32)
    nn = C.c_int64()
    assert L.pm_build_bvh_host(None, None, 1, None, C.byref(nn), None, None, None) == api.PM_ERR_ARG
    assert L.pm_build_bvh_host(v.ctypes.data, None, 0, None, C.byref(nn), None, None, None) == api.PM_ERR_ARG
    bad = v.copy()
    bad[0, 1, 2] = np.nan
    assert L.pm_build_bvh_host(bad.ctypes.data, None, 1, None, C.byref(nn), None, None, None) == api.PM_ERR_ARG
    assert b"non-finite" in L.pm_last_error()
    o = api.BvhOpts(C.sizeof(api.BvhOpts), 32, 9, 0, 0.0)
    assert L.pm_build_bvh_host(v.ctypes.data, None, 1, C.byref(o), C.byref(nn), None, None, None) == api.PM_ERR_ARG
    assert L.pm_trace_rays(None, None, 0, None, None, None) == api.PM_ERR_ARG
    # builder selection is validated before any device work
    o = api._opts(32, 4, 0, 0.0, builder=2)
    out_bvh = C.c_void_p()
    assert L.pm_build_bvh(v.ctypes.data, None, 1, C.byref(o), None, C.byref(out_bvh)) == api.PM_ERR_ARG
    assert b"builder" in L.pm_last_error()
    o = api._opts(32, 4, 0, 0.0, builder=api.BUILD_GPU_LBVH)
    assert L.pm_build_bvh_host(v.ctypes.data, None, 1, C.byref(o), C.byref(nn), None, None, None) == api.PM_ERR_ARG
    for a in (-1e-3, 1.5, float("nan")):
        o = api._opts(32, 4, 0, 0.0, split_alpha=a)
        assert L.pm_build_bvh_host(v.ctypes.data, None, 1, C.byref(o), C.byref(nn), None, None, None) == api.PM_ERR_ARG
        assert b"split_alpha" in L.pm_last_error()
    # spatial splits are a host-build option
    o = api._opts(32, 4, 0, 0.0, builder=api.BUILD_GPU_LBVH, split_alpha=1e-3)
    assert L.pm_build_bvh(v.ctypes.data, None, 1, C.byref(o), None, C.byref(out_bvh)) == api.PM_ERR_ARG
    assert b"split_alpha" in L.pm_last_error()
    assert L.pm_bvh_download(None, None, None, None) == api.PM_ERR_ARG
    # scene/param validation happens before any device work
    sc = scenes.box_scene(8, 8)
    args = api._SceneArgs(sc)
    p = api.sppm_params(0)
    out = C.c_void_p()
    assert L.pm_sppm_create(C.byref(args.desc), C.byref(p), None, C.byref(out)) == api.PM_ERR_ARG
    p = api.sppm_params(1024, single_link_set=7)
    assert L.pm_sppm_create(C.byref(args.desc), C.byref(p), None, C.byref(out)) == api.PM_ERR_ARG
    assert b"single_link_set" in L.pm_last_error()
    p = api.sppm_params(1024, gather_mode=2)
    assert L.pm_sppm_create(C.byref(args.desc), C.byref(p), None, C.byref(out)) == api.PM_ERR_ARG
    p = api.sppm_params(1024, gather_mode=1, record_iterations=2)
    assert L.pm_sppm_create(C.byref(args.desc), C.byref(p), None, C.byref(out)) == api.PM_ERR_ARG
    assert b"adjoint" in L.pm_last_error()
    p = api.sppm_params(1024, alpha=1.5)
    assert L.pm_sppm_create(C.byref(args.desc), C.byref(p), None, C.byref(out)) == api.PM_ERR_ARG
    assert b"alpha" in L.pm_last_error()
    # the one-bounce-per-pass photon schedule and its two knobs
    for bad in (dict(photon_kernel=7), dict(photon_kernel=-1)):
        p = api.sppm_params(1024, **bad)
        assert L.pm_sppm_create(C.byref(args.desc), C.byref(p), None, C.byref(out)) == api.PM_ERR_ARG
        assert b"photon_kernel" in L.pm_last_error()
    # profiling flags, and counting only where instrumented kernels exist
    for bad in (dict(profile=4), dict(profile=-1), dict(profile=api.PROFILE_COUNT, gather_mode=1),
                dict(profile=api.PROFILE_COUNT, photon_kernel=api.PHOTON_PER_PATH)):
        p = api.sppm_params(1024, **bad)
        assert L.pm_sppm_create(C.byref(args.desc), C.byref(p), None, C.byref(out)) == api.PM_ERR_ARG
        assert b"PROFILE" in L.pm_last_error() or b"profile" in L.pm_last_error()
    for bad in (dict(photon_kernel=api.PHOTON_PASSES, pass_threads=-1),
                dict(photon_kernel=api.PHOTON_PASSES, pass_threads=(1 << 26) + 1),
                dict(photon_kernel=api.PHOTON_PASSES, passes=1025),
                dict(photon_kernel=api.PHOTON_PASSES, passes=-2)):
        p = api.sppm_params(1024, **bad)
        assert L.pm_sppm_create(C.byref(args.desc), C.byref(p), None, C.byref(out)) == api.PM_ERR_ARG
        assert b"pass_threads" in L.pm_last_error()
    for kern in (api.PHOTON_AUTO, api.PHOTON_PER_PATH, api.PHOTON_REGEN):
        for knob in (dict(pass_threads=64), dict(passes=4)):
            p = api.sppm_params(1024, photon_kernel=kern, **knob)
            assert L.pm_sppm_create(C.byref(args.desc), C.byref(p), None, C.byref(out)) == api.PM_ERR_ARG
            assert b"PM_PHOTON_PASSES only" in L.pm_last_error()
    sc.tri_mat[3] = 99
    args = api._SceneArgs(sc)
    p = api.sppm_params(1024)
    assert L.pm_render(C.byref(args.desc), C.byref(p), 1, C.c_void_p(1), None) == api.PM_ERR_ARG
    assert L.pm_sppm_iterate(None, 1, None) == api.PM_ERR_ARG
    assert L.pm_sppm_resolve(None, None, None) == api.PM_ERR_ARG
    n = C.c_uint64(0)
    assert L.pm_sppm_save(None, None, C.byref(n), None) == api.PM_ERR_ARG
    assert L.pm_sppm_load(None, None, 0, None) == api.PM_ERR_ARG
    one = C.c_void_p(16)  # never dereferenced: every call below fails validation first
    assert L.pm_probe_chase(None, 4, 1, 1, one, None) == api.PM_ERR_ARG
    assert L.pm_probe_chase(one, 4, 1, 1, None, None) == api.PM_ERR_ARG
    for log2_rows, n_lanes, steps in ((0, 1, 1), (29, 1, 1), (4, 0, 1), (4, 1 << 31, 1), (4, 1, 0)):
        assert L.pm_probe_chase(one, log2_rows, n_lanes, steps, one, None) == api.PM_ERR_ARG
    # pm_trace_rays_multi: every batch is checked before anything is enqueued (the handle is never touched here)
    ok = api.TraceBatch(C.sizeof(api.TraceBatch), None, 0, None, None, None)
    reo = api._trace_opts(reorder=1)
    two = (api.TraceBatch * 2)(ok, ok)
    assert L.pm_trace_rays_multi(None, 1, two, None) == api.PM_ERR_ARG
    assert L.pm_trace_rays_multi(one, 1, None, None) == api.PM_ERR_ARG
    assert L.pm_trace_rays_multi(one, 0, two, None) == api.PM_ERR_ARG
    assert L.pm_trace_rays_multi(one, api.MAX_TRACE_BATCHES + 1, two, None) == api.PM_ERR_ARG
    small = (api.TraceBatch * 2)(ok, api.TraceBatch(4, None, 0, None, None, None))
    assert L.pm_trace_rays_multi(one, 2, small, None) == api.PM_ERR_ARG
    neg = (api.TraceBatch * 2)(ok, api.TraceBatch(C.sizeof(api.TraceBatch), None, -1, None, None, None))
    assert L.pm_trace_rays_multi(one, 2, neg, None) == api.PM_ERR_ARG
    assert b"batch 1" in L.pm_last_error()
    both = (api.TraceBatch * 2)(*[api.TraceBatch(C.sizeof(api.TraceBatch), None, 0, None, None,
                                                 C.cast(C.pointer(reo), C.c_void_p)) for _ in range(2)])
    assert L.pm_trace_rays_multi(one, 2, both, None) == api.PM_ERR_ARG
    assert b"at most one batch" in L.pm_last_error()


def _py_traverse(nodes, tris, info, ray, s):
    """Stackless walk of one link set (hit link = next node, miss = skip)."""
    lo, hi, leaf, first, cnt, skip = decode(nodes[s], info)
    o, d = ray[0:3].astype(np.float64), ray[4:7].astype(np.float64)
    tmin, tmax = float(ray[3]), float(ray[7])
    tf = f32(tris)
    best, tb = -1, tmax
    i, n = 0, nodes.shape[1]
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
    while i < n:
        t0 = (lo[i] - o) * inv
        t1 = (hi[i] - o) * inv
        tn = np.nanmax(np.concatenate([np.minimum(t0, t1), [tmin]]))
        tf_ = np.nanmin(np.concatenate([np.maximum(t0, t1), [tb]]))
        hit = tn <= tf_ + abs(tf_) * 2.0 ** -16 + 1e-12
        if hit and leaf[i]:
            for k in range(first[i], first[i] + cnt[i]):
                t = _wt32(ray, tf[k])
                idx = int(tris[k, 9])
                if t is not None and t > tmin and (t < tb or (t == tb and best >= 0 and idx < best)):
                    tb, best = t, idx
        i = i + 1 if (hit or leaf[i]) else skip[i]
    return best, tb


def _wt32(ray, tri):
    """The device's float32 watertight triangle test for one ray: t or None."""
    ok, t, _ = wt32(ray[None, 0:3], ray[None, 4:7], tri[None, 0:9])
    return float(t[0]) if ok[0] else None


@pytest.mark.parametrize("seed,n,spread,alpha", [(0, 1, None, 0.0), (1, 5, None, 0.0), (2, 33, None, 0.0),
                                                 (3, 64, None, 0.0), (4, 300, None, 0.0), (3, 64, None, 1e-4),
                                                 (4, 300, None, 1e-4), (5, 200, 0.3, 1e-5)])
def test_host_bvh_structure_and_every_link_set_matches_brute_force(oracle_lib, seed, n, spread, alpha):
    """alpha > 0: spatial splits put triangles in several leaves, each with the
    box of its clipped part; the walk must still find the brute-force hit."""
    sc = scenes.small_soup(n, seed, spread=0.4 / max(1.0, np.cbrt(n)) if spread is None else spread)
    nodes, tris, info = api.build_bvh_host(sc.verts, sc.tri_mat, split_alpha=alpha)
    assert check_structure(sc.verts, nodes, tris, 4, info)
    assert info["n_nodes"] == nodes.shape[1] and info["n_tri"] == n
    assert (info["n_refs"] > n) if alpha > 0 else (info["n_refs"] == n)
    assert info["device_bytes"] == 6 * 16 * info["n_nodes"] + 48 * info["n_refs"]
    rays = scenes.random_rays(60, seed)
    h_ref, t_ref = oracle_lib.trace_brute_force(sc.verts, rays)
    for s in range(6):
        for r in range(len(rays)):
            h, t = _py_traverse(nodes, tris, info, rays[r], s)
            assert h == h_ref[r], (s, r)
            if h >= 0:
                assert np.float32(t) == t_ref[r]


def _py_wave_postponed(nodes, tris, info, rays, s, late, steps=1):
    """Lockstep model of one wavefront running the postponed-leaf walk: box
    visits until at most `late` lanes still search (and one lane holds a leaf),
    then every held leaf is tested; a holding lane halts at its next leaf hit.
    The wave votes once per `steps` box visits."""
    lo, hi, leaf, first, cnt, skip = decode(nodes[s], info)
    tf = f32(tris)
    L, n = len(rays), nodes.shape[1]
    o = rays[:, 0:3].astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / rays[:, 4:7].astype(np.float64)
    tmin = rays[:, 3].astype(np.float64)
    tb = rays[:, 7].astype(np.float64).copy()
    best = np.full(L, -1)
    i = np.zeros(L, np.int64)
    held = np.full(L, -1)
    halted = np.zeros(L, bool)
    visits = 0

    def box_hit(r, k):
        t0, t1 = (lo[k] - o[r]) * inv[r], (hi[k] - o[r]) * inv[r]
        with np.errstate(invalid="ignore"):
            tn = np.nanmax(np.concatenate([np.minimum(t0, t1), [tmin[r]]]))
            tf_ = np.nanmin(np.concatenate([np.maximum(t0, t1), [tb[r]]]))
        return tn <= tf_ + abs(tf_) * 2.0 ** -16 + 1e-12

    while True:
        while True:
            searching = (i < n) & (held < 0)
            if not searching.any():
                break
            if searching.sum() <= late and (held >= 0).any():
                break
            visits += 1
            assert visits < 64 * n, "box loop does not end"
            for _ in range(steps):
                for r in range(L):
                    if i[r] >= n or halted[r]:
                        continue
                    k = i[r]
                    hit = box_hit(r, k)
                    if hit and leaf[k]:
                        if held[r] < 0:
                            held[r], i[r] = k, k + 1
                        else:
                            halted[r] = True
                    else:
                        i[r] = k + 1 if (hit or leaf[k]) else skip[k]
        if not (held >= 0).any():
            break
        for r in np.nonzero(held >= 0)[0]:
            k = held[r]
            for j in range(first[k], first[k] + cnt[k]):
                t = _wt32(rays[r], tf[j])
                idx = int(tris[j, 9])
                if t is not None and t > tmin[r] and (t < tb[r] or (t == tb[r] and best[r] >= 0 and idx < best[r])):
                    tb[r], best[r] = t, idx
        held[:] = -1
        halted[:] = False
    return best, tb


@pytest.mark.parametrize("late,steps", [(0, 1), (5, 1), (63, 1), (16, 8), (0, 8), (63, 3)])
def test_postponed_leaf_walk_model_matches_brute_force(oracle_lib, late, steps):
    """The wave schedule of the postponed traversal kernel, modelled on the
    CPU: it ends, and every lane's closest hit equals brute force, whether
    the wave votes after every box visit or after several."""
    sc = scenes.small_soup(300, 4, spread=0.4 / np.cbrt(300))
    nodes, tris, info = api.build_bvh_host(sc.verts, sc.tri_mat)
    rays = scenes.random_rays(64, 4)
    h_ref, t_ref = oracle_lib.trace_brute_force(sc.verts, rays)
    for s in (0, 3):
        h, t = _py_wave_postponed(nodes, tris, info, rays, s, late, steps)
        assert np.array_equal(h, h_ref)
        assert np.array_equal(np.float32(t[h >= 0]), t_ref[h >= 0])


def _py_wave_slices(nodes, tris, info, rays, s, late, steps, n_rays):
    """Lockstep model of one wavefront of the slice kernel over rays
    0 .. n_rays - 1: the postponed walk in which an idle lane takes the
    slice's next ray (lanes in order) at the top of each round, and the box
    loop also stops once at most `late` lanes search while a lane could take
    a new ray.  Returns (best, t) per ray and the number of rounds."""
    lo, hi, leaf, first, cnt, skip = decode(nodes[s], info)
    tf = f32(tris)
    L, n = 64, nodes.shape[1]
    o_all = rays[:, 0:3].astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv_all = 1.0 / rays[:, 4:7].astype(np.float64)
    best_out = np.full(n_rays, -2)
    t_out = np.full(n_rays, np.nan)
    ray = np.full(L, -1)             # the lane's ray, -1 idle
    i = np.zeros(L, np.int64)
    nn = np.zeros(L, np.int64)       # walk length: n while walking, 0 before the first ray
    tb = np.zeros(L)
    best = np.full(L, -1)
    held = np.full(L, -1)
    halted = np.zeros(L, bool)
    cursor, rounds = 0, 0

    def box_hit(r, k):
        rr = ray[r]
        t0, t1 = (lo[k] - o_all[rr]) * inv_all[rr], (hi[k] - o_all[rr]) * inv_all[rr]
        with np.errstate(invalid="ignore"):
            tn = np.nanmax(np.concatenate([np.minimum(t0, t1), [float(rays[rr, 3])]]))
            tf_ = np.nanmin(np.concatenate([np.maximum(t0, t1), [tb[r]]]))
        return tn <= tf_ + abs(tf_) * 2.0 ** -16 + 1e-12

    while True:
        rounds += 1
        assert rounds < 64 * n * (n_rays + 1), "the slice walk does not end"
        idle = ray < 0
        if idle.any() and cursor < n_rays:
            rank = np.cumsum(idle) - 1
            for r in np.nonzero(idle & (rank < n_rays - cursor))[0]:
                ray[r] = cursor + rank[r]
                i[r], nn[r], tb[r], best[r] = 0, n, float(rays[ray[r], 7]), -1
            cursor = min(n_rays, cursor + int(idle.sum()))
        if not (ray >= 0).any():
            break
        while True:
            searching = (i < nn) & (held < 0)
            if not searching.any():
                break
            free = (i >= nn) & (held < 0)
            if searching.sum() <= late and ((held >= 0).any() or (cursor < n_rays and free.any())):
                break
            for _ in range(steps):
                for r in range(L):
                    if i[r] >= nn[r] or halted[r]:
                        continue
                    k = i[r]
                    hit = box_hit(r, k)
                    if hit and leaf[k]:
                        if held[r] < 0:
                            held[r], i[r] = k, k + 1
                        else:
                            halted[r] = True
                    else:
                        i[r] = k + 1 if (hit or leaf[k]) else skip[k]
        for r in np.nonzero(held >= 0)[0]:
            k = held[r]
            for j in range(first[k], first[k] + cnt[k]):
                t = _wt32(rays[ray[r]], tf[j])
                idx = int(tris[j, 9])
                if t is not None and t > rays[ray[r], 3] and (t < tb[r] or (t == tb[r] and best[r] >= 0 and idx < best[r])):
                    tb[r], best[r] = t, idx
        held[:] = -1
        halted[:] = False
        for r in np.nonzero((ray >= 0) & (i >= nn))[0]:
            best_out[ray[r]] = best[r]
            t_out[ray[r]] = tb[r] if best[r] >= 0 else np.inf
            ray[r] = -1
    return best_out, t_out, rounds


@pytest.mark.parametrize("late,steps,n_rays", [(0, 1, 300), (5, 8, 300), (32, 8, 300), (63, 1, 300), (16, 3, 17),
                                               (32, 8, 64), (0, 8, 129)])
def test_slice_walk_model_matches_brute_force(oracle_lib, late, steps, n_rays):
    """The wave schedule of the slice traversal kernel, modelled on the CPU:
    it ends, every ray of the slice (also fewer rays than lanes, and a
    ragged last refill) is written once, and each equals brute force."""
    sc = scenes.small_soup(300, 4, spread=0.4 / np.cbrt(300))
    nodes, tris, info = api.build_bvh_host(sc.verts, sc.tri_mat)
    rays = scenes.random_rays(n_rays, 5)
    rays[::4, 4:7] = np.abs(rays[::4, 4:7]) * [1, 0.1, 0.1]   # a share of the rays in one link set
    h_ref, t_ref = oracle_lib.trace_brute_force(sc.verts, rays)
    for s in (0, 3):
        h, t, rounds = _py_wave_slices(nodes, tris, info, rays, s, late, steps, n_rays)
        assert np.all(h >= -1), "a ray of the slice was not written"
        assert np.array_equal(h, h_ref)
        assert np.array_equal(np.float32(t[h >= 0]), t_ref[h >= 0])
        assert np.all(np.isinf(t[h < 0]))


def test_host_bvh_box_scene_and_soup_statistics():
    sc = scenes.box_scene()
    nodes, tris, info = api.build_bvh_host(sc.verts, sc.tri_mat)
    check_structure(sc.verts, nodes, tris, 4, info)
    assert np.array_equal(tris[:, 10], sc.tri_mat[tris[:, 9]])
    sc = scenes.soup_scene(1 << 14, seed=9)
    nodes, tris, info = api.build_bvh_host(sc.verts, sc.tri_mat, max_leaf=2, bins=8)
    check_structure(sc.verts, nodes, tris, 2, info)
    # SAH tree: cheaper than the worst case of one leaf per 2 triangles in a chain
    assert info["depth"] < 64 and info["sah_cost"] > 0
    # a costlier node visit gives fewer nodes and fuller leaves
    n2, t2, info2 = api.build_bvh_host(sc.verts, sc.tri_mat, max_leaf=2, bins=8, trav_cost=4.0)
    check_structure(sc.verts, n2, t2, 2, info2)
    assert info2["n_nodes"] < info["n_nodes"]
    # storage: 6 link sets x 16 B per node + 48 B per triangle
    assert info["device_bytes"] == 6 * 16 * info["n_nodes"] + 48 * info["n_tri"]
    # spatial splits: more records, a lower SAH cost, and the same BVH from two builds
    n3, t3, info3 = api.build_bvh_host(sc.verts, sc.tri_mat, max_leaf=2, bins=8, split_alpha=1e-5)
    check_structure(sc.verts, n3, t3, 2, info3)
    assert info3["n_refs"] > info3["n_tri"] and info3["sah_cost"] < info["sah_cost"]
    n4, t4, info4 = api.build_bvh_host(sc.verts, sc.tri_mat, max_leaf=2, bins=8, split_alpha=1e-5, n_threads=3)
    assert np.array_equal(n3, n4) and np.array_equal(t3, t4)


def test_binding_classes_expose_the_abi():
    for name in ("iterate", "resolve", "status", "views", "adjoint", "destroy"):
        assert callable(getattr(api.Sppm, name, None)), name
    for name in ("iterate", "resolve", "status", "info", "views", "destroy"):
        assert callable(getattr(api.Batch, name, None)), name
    for fn in ("build_bvh", "build_bvh_host", "trace_rays", "sppm_create", "render", "render_batch",
               "sppm_render_diff"):
        assert callable(getattr(api, fn, None)), fn
