"""GPU parity of pm_trace_rays against the oracle's brute-force closest hit.

Hit index must match bit-exactly; t must agree to 1e-5 relative (the same
float32 watertight triangle test on both sides makes it exact in practice,
which is asserted as well).
"""
import sys

import numpy as np
import pytest

from paper_1505_06022_amd import api, scenes

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _gpu_trace(torch, bvh, rays, **kw):
    r = torch.from_numpy(np.ascontiguousarray(rays)).cuda()
    h, t = api.trace_rays(bvh, r, **kw)
    torch.cuda.synchronize()
    return h.cpu().numpy(), t.cpu().numpy()


def _compare(h, t, h_ref, t_ref):
    assert np.array_equal(h, h_ref), f"{np.count_nonzero(h != h_ref)} hit mismatches"
    hit = h_ref >= 0
    assert np.all(np.isinf(t[~hit]))
    rel = np.abs(t[hit] - t_ref[hit]) / np.maximum(np.abs(t_ref[hit]), 1e-30)
    assert rel.max(initial=0) <= 1e-5
    assert np.array_equal(t[hit], t_ref[hit])


def test_box_scene_all_rays(torch_cuda, oracle_lib):
    _log("case: box scene, pinhole + random rays")
    sc = scenes.box_scene()
    bvh = api.build_bvh(sc.verts, sc.tri_mat)
    rays = np.concatenate([scenes.pinhole_rays(sc.camera), scenes.random_rays(5000, 1)])
    h_ref, t_ref = oracle_lib.trace_brute_force(sc.verts, rays)
    h, t = _gpu_trace(torch_cuda, bvh, rays)
    _compare(h, t, h_ref, t_ref)
    assert (h >= 0).mean() > 0.8    # random rays leave through the open front


@pytest.mark.parametrize("n_tri,n_rays,seed", [(1, 1, 0), (7, 63, 1), (64, 65, 2), (1000, 257, 3),
                                               (20000, 4097, 4), (3, 0, 5)])
def test_random_scenes_ragged_sizes(torch_cuda, oracle_lib, n_tri, n_rays, seed):
    _log(f"case: soup n_tri={n_tri} n_rays={n_rays} seed={seed}")
    sc = scenes.small_soup(n_tri, seed, spread=0.4 / max(1.0, np.cbrt(n_tri)))
    sc.verts[::11, 2] = sc.verts[::11, 0]   # degenerate triangles
    bvh = api.build_bvh(sc.verts, sc.tri_mat)
    rays = scenes.random_rays(max(n_rays, 1), seed)[:n_rays]
    if n_rays:
        rays[::5, 4:7] = np.array([0, 1, 0], np.float32)  # axis-parallel
        rays[1::7, 3] = 0.05                               # non-zero tmin
        rays[2::9, 7] = 0.3                                # finite tmax
    h_ref, t_ref = oracle_lib.trace_brute_force(sc.verts, rays)
    h, t = _gpu_trace(torch_cuda, bvh, rays)
    _compare(h, t, h_ref, t_ref)


@pytest.mark.parametrize("n_rays,one_bucket", [(4096, False), (4097, False), (262145, False), (50000, True)])
def test_bucketing_chunk_boundaries_and_one_bucket(torch_cuda, oracle_lib, n_rays, one_bucket):
    """The coarse bucketing counts the rays in up to 64 chunks of at least 4096 (one histogram in LDS per chunk):
    one chunk, a second chunk of one ray, 64 chunks with a short last one, and rays that all share one bucket
    (one origin, directions around +y).  Bucketed walks equal the per-ray walk, and sampled rays the brute force."""
    _log(f"case: bucketing n_rays={n_rays} one_bucket={one_bucket}")
    sc = scenes.small_soup(20000, 11, spread=0.03)
    bvh = api.build_bvh(sc.verts, sc.tri_mat)
    rays = scenes.random_rays(n_rays, 11)
    if one_bucket:
        rng = np.random.default_rng(11)
        d = np.stack([rng.uniform(-0.5, 0.5, n_rays), np.ones(n_rays), rng.uniform(-0.5, 0.5, n_rays)], 1)
        rays[:, 0:3] = np.array([0.5, 0.05, 0.5], np.float32)
        rays[:, 4:7] = d / np.linalg.norm(d, axis=1, keepdims=True)
    h, t = _gpu_trace(torch_cuda, bvh, rays, kernel=1)
    for kw in (dict(reorder=1), dict(kernel=4, refill=32, reorder=1, block=64)):
        hb, tb = _gpu_trace(torch_cuda, bvh, rays, **kw)
        assert np.array_equal(h, hb) and np.array_equal(t, tb)
    pick = np.random.default_rng(12).choice(n_rays, min(n_rays, 2048), replace=False)
    h_ref, t_ref = oracle_lib.trace_brute_force(sc.verts, rays[pick])
    _compare(h[pick], t[pick], h_ref, t_ref)


def test_every_link_set_and_stats_mode_agree(torch_cuda, oracle_lib):
    _log("case: forced link sets 0..5 and counters")
    sc = scenes.small_soup(3000, 7, spread=0.03)
    bvh = api.build_bvh(sc.verts, sc.tri_mat)
    rays = np.concatenate([scenes.random_rays(3000, 7), scenes.pinhole_rays(sc.camera)])
    h_ref, t_ref = oracle_lib.trace_brute_force(sc.verts, rays)
    for s in range(6):
        h, t = _gpu_trace(torch_cuda, bvh, rays, link_set=s)
        _compare(h, t, h_ref, t_ref)
    cnt = torch_cuda.zeros((len(rays), 2), dtype=torch_cuda.int32, device="cuda")
    h, t = _gpu_trace(torch_cuda, bvh, rays, counters=cnt)
    _compare(h, t, h_ref, t_ref)
    c = cnt.cpu().numpy()
    assert np.all(c[:, 0] >= 1) and np.all(c[:, 1] >= (h >= 0))


@pytest.mark.parametrize("kernel,refill,reorder,block", [
    (1, 0, False, 0), (2, 1, False, 0), (2, 16, False, 0), (2, 64, False, 0), (1, 0, 1, 0), (1, 0, 2, 0),
    (3, 0, 0, 0), (4, 0, 0, 0), (4, 7, 0, 0), (4, 63, 0, 0), (4, 0, 1, 0), (4, 16, 2, 0), (3, 0, 1, 0),
    (1, 0, 0, 64), (1, 0, 1, 128), (4, 16, 1, 64), (3, 0, 0, 128), (5, 0, 0, 0), (5, 0, 1, 64),
    (5, 0, 2, 128), (2, 16, 1, 0), (2, 1, 2, 0), (6, 0, 0, 0), (6, 0, 1, 64), (6, 0, 0, 128)])
def test_traversal_kernels_agree(torch_cuda, oracle_lib, kernel, refill, reorder, block):
    _log(f"case: traversal kernel={kernel} refill={refill} reorder={reorder} block={block}")
    sc = scenes.small_soup(5000, 11, spread=0.02)
    bvh = api.build_bvh(sc.verts, sc.tri_mat)
    rays = np.concatenate([scenes.random_rays(7001, 11), scenes.pinhole_rays(sc.camera)])
    h_ref, t_ref = oracle_lib.trace_brute_force(sc.verts, rays)
    h, t = _gpu_trace(torch_cuda, bvh, rays, kernel=kernel, refill=refill, reorder=reorder, block=block)
    _compare(h, t, h_ref, t_ref)
    cnt = torch_cuda.zeros((len(rays), 2), dtype=torch_cuda.int32, device="cuda")
    h, t = _gpu_trace(torch_cuda, bvh, rays, kernel=kernel, refill=refill, counters=cnt, reorder=reorder,
                      block=block)
    _compare(h, t, h_ref, t_ref)


@pytest.mark.parametrize("late,reorder,block,slice_", [(32, 1, 64, 0), (32, 0, 256, 0), (0, 2, 128, 100),
                                                        (63, 1, 64, 1000), (5, 1, 64, 7), (16, 0, 64, 64),
                                                        (32, 1, 256, 100000)])
def test_slice_kernel_agrees(torch_cuda, oracle_lib, late, reorder, block, slice_):
    """The postponed walk over per-wavefront slices with lane refill: every
    slice size (automatic, ragged, shorter than a wavefront, longer than the
    batch), threshold and bucketing gives the brute-force closest hits, also
    in statistics mode."""
    _log(f"case: slice kernel late={late} reorder={reorder} block={block} slice={slice_}")
    sc = scenes.small_soup(5000, 11, spread=0.02)
    bvh = api.build_bvh(sc.verts, sc.tri_mat)
    rays = np.concatenate([scenes.random_rays(7001, 11), scenes.pinhole_rays(sc.camera)])
    h_ref, t_ref = oracle_lib.trace_brute_force(sc.verts, rays)
    kw = dict(kernel=api.TRACE_SLICES, refill=late, reorder=reorder, block=block, slice_rays=slice_)
    h, t = _gpu_trace(torch_cuda, bvh, rays, **kw)
    _compare(h, t, h_ref, t_ref)
    cnt = torch_cuda.zeros((len(rays), 2), dtype=torch_cuda.int32, device="cuda")
    h, t = _gpu_trace(torch_cuda, bvh, rays, counters=cnt, **kw)
    _compare(h, t, h_ref, t_ref)
    c = cnt.cpu().numpy()
    assert np.all(c[:, 0] >= 1) and np.all(c[:, 1] >= (h >= 0))


def test_slices_and_packets_in_one_multi_call_equal_single_calls(torch_cuda, oracle_lib):
    """Two batches, the bucketed slice walk and packets over image tiles, in
    one pm_trace_rays_multi call: the same results as two single calls and
    as brute force (automatic and explicit slice sizes)."""
    _log("case: multi call slices + packets, soup 2^14")
    sc = scenes.soup_scene(1 << 14, 4)
    bvh = api.build_bvh(sc.verts, sc.tri_mat)
    cam = scenes.pinhole_rays(scenes.Camera(pos=(0.5, 0.5, -1.5), look=(0.5, 0.5, 0.5), up=(0, 1, 0),
                                            tan_half_fov=0.4, width=96, height=40))
    inc = scenes.random_rays(5000, 9)
    rc, ri = (torch_cuda.from_numpy(np.ascontiguousarray(x)).cuda() for x in (cam, inc))
    kc = dict(kernel=api.TRACE_PACKET, block=64, tile_width=96)
    h_ref, t_ref = oracle_lib.trace_brute_force(sc.verts, inc)
    for slice_ in (0, 130):
        ki = dict(kernel=api.TRACE_SLICES, refill=32, reorder=1, block=64, slice_rays=slice_)
        single = [api.trace_rays(bvh, rc, **kc), api.trace_rays(bvh, ri, **ki)]
        two = api.trace_rays_multi(bvh, [dict(rays=rc, **kc), dict(rays=ri, **ki)])
        for (h, t), (hr, tr) in zip(two, single):
            assert np.array_equal(h.cpu().numpy(), hr.cpu().numpy()), slice_
            assert np.array_equal(t.cpu().numpy(), tr.cpu().numpy()), slice_
        _compare(two[1][0].cpu().numpy(), two[1][1].cpu().numpy(), h_ref, t_ref)


# (builder, split_alpha): the host SAH build, the GPU linear BVH, and the host
# SAH build with spatial splits (triangles in several leaves, clipped boxes)
BUILDS = [(api.BUILD_HOST_SAH, 0.0), (api.BUILD_GPU_LBVH, 0.0), (api.BUILD_HOST_SAH, 1e-5)]


@pytest.mark.parametrize("alpha", [1e-3, 1e-5])
def test_spatial_split_bvh_every_kernel(torch_cuda, oracle_lib, alpha):
    """A BVH with spatial splits (triangles referenced by several leaves, each
    with the box of its clipped part): every traversal kernel, with
    bucketing, packets over image tiles, slices, forced link sets, statistics
    and the two-batch call, equals brute force; hits are original indices."""
    _log(f"case: spatial-split BVH alpha={alpha}")
    sc = scenes.small_soup(5000, 13, spread=0.04)
    bvh = api.build_bvh(sc.verts, sc.tri_mat, split_alpha=alpha)
    inf = bvh.info()
    assert inf["n_refs"] > inf["n_tri"] == 5000
    nodes, tris = bvh.download()
    assert tris.shape == (inf["n_refs"], 12) and np.array_equal(np.unique(tris[:, 9]), np.arange(5000))
    hn, ht, hinf = api.build_bvh_host(sc.verts, sc.tri_mat, split_alpha=alpha)   # the same BVH
    assert np.array_equal(nodes, hn) and np.array_equal(tris, ht) and hinf["n_refs"] == inf["n_refs"]
    inc = scenes.random_rays(7001, 13)
    cam = scenes.pinhole_rays(sc.camera)
    rays = np.concatenate([inc, cam])
    h_ref, t_ref = oracle_lib.trace_brute_force(sc.verts, rays)
    for kw in (dict(kernel=1), dict(kernel=2, refill=16), dict(kernel=3, reorder=1), dict(kernel=4, refill=32,
               reorder=1, block=64), dict(kernel=5, reorder=2), dict(kernel=6),
               dict(kernel=api.TRACE_SLICES, refill=32, reorder=1, block=64, slice_rays=100)):
        h, t = _gpu_trace(torch_cuda, bvh, rays, **kw)
        _compare(h, t, h_ref, t_ref)
    for s_ in range(6):
        h, t = _gpu_trace(torch_cuda, bvh, rays, link_set=s_, kernel=4, refill=32)
        _compare(h, t, h_ref, t_ref)
    cnt = torch_cuda.zeros((len(rays), 2), dtype=torch_cuda.int32, device="cuda")
    h, t = _gpu_trace(torch_cuda, bvh, rays, counters=cnt, kernel=4, refill=32, reorder=1)
    _compare(h, t, h_ref, t_ref)
    W, H = sc.camera.width, sc.camera.height
    h, t = _gpu_trace(torch_cuda, bvh, cam, kernel=6, block=64, tile_width=W)
    _compare(h, t, h_ref[len(inc):], t_ref[len(inc):])
    ri, rc = (torch_cuda.from_numpy(np.ascontiguousarray(x)).cuda() for x in (inc, cam))
    (hi_, ti_), (hc_, tc_) = api.trace_rays_multi(bvh, [dict(rays=ri, kernel=4, refill=32, reorder=1, block=64),
                                                        dict(rays=rc, kernel=6, block=64, tile_width=W)])
    _compare(hi_.cpu().numpy(), ti_.cpu().numpy(), h_ref[:len(inc)], t_ref[:len(inc)])
    _compare(hc_.cpu().numpy(), tc_.cpu().numpy(), h_ref[len(inc):], t_ref[len(inc):])
    bvh.destroy()


@pytest.mark.parametrize("builder,alpha", BUILDS)
@pytest.mark.parametrize("kind", ["soup", "box"])
def test_grazing_and_far_origin_rays(torch_cuda, oracle_lib, builder, alpha, kind):
    """Rays that stress the box test's conservativeness: grazing angles
    1e-1..1e-6 rad at interior points and at edges/vertices of the triangle
    they aim at, and origins 10^2..10^5 extents away; every traversal kernel,
    every build, against brute force."""
    _log(f"case: grazing/far-origin rays builder={builder} alpha={alpha} scene={kind}")
    verts = (scenes.small_soup(4096, 11, spread=0.03).verts if kind == "soup"
             else scenes.box_scene(8, 8).verts)
    angles = [1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6]
    rays = np.concatenate([scenes.grazing_rays(verts, 3000, angles, seed=21, on_edges=False),
                           scenes.grazing_rays(verts, 3000, angles, seed=22, on_edges=True),
                           scenes.far_origin_rays(verts, 2000, seed=31)])
    h_ref, t_ref = oracle_lib.trace_brute_force(verts, rays)
    assert (h_ref >= 0).mean() > 0.5
    bvh = api.build_bvh(verts, builder=builder, split_alpha=alpha)
    for kernel in (1, 2, 3, 4, 5, 6):
        h, t = _gpu_trace(torch_cuda, bvh, rays, kernel=kernel)
        _compare(h, t, h_ref, t_ref)


def _closed_box(lo, hi):
    """The 12 triangles of the closed box [lo, hi]^3 (two per face)."""
    c = np.array([[x, y, z] for x in (lo, hi) for y in (lo, hi) for z in (lo, hi)], np.float64)
    quads = [(0, 1, 3, 2), (4, 6, 7, 5), (0, 4, 5, 1), (2, 3, 7, 6), (0, 2, 6, 4), (1, 5, 7, 3)]
    return np.asarray([[c[a], c[b], c[d]] for a, b, cc, d in quads for b, d in ((b, cc), (cc, d))])


@pytest.mark.parametrize("builder,alpha", BUILDS)
@pytest.mark.parametrize("mesh", ["sphere", "sphere_in_box"])
def test_closed_mesh_watertight_on_device(torch_cuda, oracle_lib, builder, alpha, mesh):
    """Rays aimed exactly at the shared vertices and at points of the shared
    edges of closed meshes: an icosphere (level 3, 1,280 triangles) from inside
    it, and that sphere (radius 0.5) inside a closed box of 12 triangles, from
    points between the two, aimed at both meshes' edges and vertices (with
    spatial splits the box's triangles are clipped into several leaves).  Every
    ray hits, with every traversal kernel, and equals brute force."""
    _log(f"case: watertight {mesh}, builder={builder} alpha={alpha}")
    rng = np.random.default_rng(12)
    c0 = np.array([0.3, -1.2, 0.8])
    if mesh == "sphere":
        verts = (scenes._icosphere(3) * 2.5 + c0).astype(np.float32)
    else:
        verts = np.concatenate([scenes._icosphere(3) * 0.5, _closed_box(-3.0, 3.0)]) + c0
        verts = verts.astype(np.float32)
    pts = np.unique(verts.reshape(-1, 3), axis=0)
    edges = [f[i].astype(np.float64) + lam * (f[(i + 1) % 3].astype(np.float64) - f[i].astype(np.float64))
             for f in verts for i in range(3) for lam in (0.5, rng.random())]
    targets = np.concatenate([pts, np.asarray(edges)]).astype(np.float32)
    if mesh == "sphere":
        o = c0 + 1.2 * rng.uniform(-1, 1, (len(targets), 3)) / np.sqrt(3)
    else:   # between the sphere and the box
        o = rng.uniform(-2.5, 2.5, (len(targets), 3))
        o = c0 + o * np.maximum(1.0, 0.8 / np.linalg.norm(o, axis=1))[:, None]
    o = o.astype(np.float32)
    rays = np.zeros((len(targets), 8), np.float32)
    rays[:, 0:3], rays[:, 4:7], rays[:, 7] = o, targets - o, np.inf
    h_ref, t_ref = oracle_lib.trace_brute_force(verts, rays)
    assert (h_ref >= 0).all()
    bvh = api.build_bvh(verts, builder=builder, split_alpha=alpha)
    if alpha > 0 and mesh == "sphere_in_box":
        assert bvh.info()["n_refs"] > len(verts)
    for kernel in (1, 2, 3, 4, 5, 6, 7):
        h, t = _gpu_trace(torch_cuda, bvh, rays, kernel=kernel)
        _compare(h, t, h_ref, t_ref)
        assert (h >= 0).all(), kernel


@pytest.mark.parametrize("kernel,block", [(1, 0), (3, 64), (4, 128), (6, 0), (6, 64)])
def test_image_tiles_and_packets(torch_cuda, oracle_lib, kernel, block):
    """Camera rays taken in 8x8 pixel tiles per wave (a ragged 37x23 image and
    a 64x64 one), each kernel, against brute force; packets of random rays
    (mixed link sets) take the per-ray walk."""
    _log(f"case: image tiles kernel={kernel} block={block}")
    sc = scenes.small_soup(3000, 12, spread=0.03)
    bvh = api.build_bvh(sc.verts, sc.tri_mat)
    for w, h in ((37, 23), (64, 64)):
        cam = scenes.Camera(pos=(0.5, 0.5, -1.5), look=(0.5, 0.5, 0.5), up=(0.0, 1.0, 0.0), tan_half_fov=0.4,
                            width=w, height=h)
        rays = scenes.pinhole_rays(cam)
        h_ref, t_ref = oracle_lib.trace_brute_force(sc.verts, rays)
        hh, tt = _gpu_trace(torch_cuda, bvh, rays, kernel=kernel, block=block, tile_width=w)
        _compare(hh, tt, h_ref, t_ref)
        cnt = torch_cuda.zeros((len(rays), 2), dtype=torch_cuda.int32, device="cuda")
        hh, tt = _gpu_trace(torch_cuda, bvh, rays, kernel=kernel, block=block, tile_width=w, counters=cnt)
        _compare(hh, tt, h_ref, t_ref)
        assert cnt.cpu().numpy()[:, 0].min() >= 1
    rays = scenes.random_rays(4100, 12)
    h_ref, t_ref = oracle_lib.trace_brute_force(sc.verts, rays)
    hh, tt = _gpu_trace(torch_cuda, bvh, rays, kernel=kernel, block=block, tile_width=41)
    _compare(hh, tt, h_ref, t_ref)
    bvh.destroy()


def test_soup_full_size_sampled_rays(torch_cuda, oracle_lib):
    """1M-triangle soup, all 4.17M rays traced on the GPU; a seeded sample of
    4096 coherent + 4096 incoherent rays checked against brute force over all
    triangles, and 131072 more against the oracle's own BVH."""
    _log("case: soup 2^20 triangles, 1920x1080 + 2^21 rays")
    sc, coh, inc = scenes.soup_workload()
    bvh = api.build_bvh(sc.verts, sc.tri_mat)
    rays = np.concatenate([coh, inc])
    h, t = _gpu_trace(torch_cuda, bvh, rays)
    h1, t1 = _gpu_trace(torch_cuda, bvh, rays, kernel=1)     # one ray per lane: identical
    assert np.array_equal(h, h1) and np.array_equal(t, t1)
    h3, t3 = _gpu_trace(torch_cuda, bvh, rays, kernel=3)     # paired node visits: identical
    assert np.array_equal(h, h3) and np.array_equal(t, t3)
    for late in (0, 8):                                       # postponed leaf tests: identical
        h4, t4 = _gpu_trace(torch_cuda, bvh, rays, kernel=4, refill=late)
        assert np.array_equal(h, h4) and np.array_equal(t, t4)
    h5, t5 = _gpu_trace(torch_cuda, bvh, rays, kernel=5)     # two rays per lane: identical
    assert np.array_equal(h, h5) and np.array_equal(t, t5)
    nc = len(coh)                                             # camera rays as packets of 8x8 tiles: identical
    h6, t6 = _gpu_trace(torch_cuda, bvh, coh, kernel=6, block=64, tile_width=1920)
    assert np.array_equal(h[:nc], h6) and np.array_equal(t[:nc], t6)
    h6, t6 = _gpu_trace(torch_cuda, bvh, rays, kernel=6)
    assert np.array_equal(h, h6) and np.array_equal(t, t6)
    # the incoherent batch as the bench times it: bucketed, postponed (late 32), 64-thread workgroups
    hb, tb = _gpu_trace(torch_cuda, bvh, inc, kernel=4, refill=32, reorder=1, block=64)
    assert np.array_equal(h[nc:], hb) and np.array_equal(t[nc:], tb)
    # the bench's timed step: both batches side by side in one pm_trace_rays_multi call
    ri, rc = (torch_cuda.from_numpy(np.ascontiguousarray(x)).cuda() for x in (inc, coh))
    (hi_, ti_), (hc_, tc_) = api.trace_rays_multi(bvh, [dict(rays=ri, kernel=4, refill=32, reorder=1, block=64),
                                                        dict(rays=rc, kernel=6, block=64, tile_width=1920)])
    assert np.array_equal(h[nc:], hi_.cpu().numpy()) and np.array_equal(t[nc:], ti_.cpu().numpy())
    assert np.array_equal(h[:nc], hc_.cpu().numpy()) and np.array_equal(t[:nc], tc_.cpu().numpy())
    # the bench's BVH: spatial splits; its timed call gives the same hits
    bs = api.build_bvh(sc.verts, sc.tri_mat, split_alpha=scenes.SOUP_SPLIT_ALPHA, trav_cost=scenes.SOUP_TRAV_COST)
    assert bs.info()["n_refs"] > bs.info()["n_tri"]
    (hi_, ti_), (hc_, tc_) = api.trace_rays_multi(bs, [dict(rays=ri, kernel=4, refill=32, reorder=1, block=64),
                                                       dict(rays=rc, kernel=6, block=64, tile_width=1920)])
    assert np.array_equal(h[nc:], hi_.cpu().numpy()) and np.array_equal(t[nc:], ti_.cpu().numpy())
    assert np.array_equal(h[:nc], hc_.cpu().numpy()) and np.array_equal(t[:nc], tc_.cpu().numpy())
    hs, ts = _gpu_trace(torch_cuda, bs, rays, kernel=1)
    assert np.array_equal(h, hs) and np.array_equal(t, ts)
    bs.destroy()
    del ri, rc, hi_, ti_, hc_, tc_
    h5, t5 = _gpu_trace(torch_cuda, bvh, rays[:-1], kernel=5, reorder=1, block=64)   # odd count
    assert np.array_equal(h[:-1], h5) and np.array_equal(t[:-1], t5)
    for level in (1, 2):                                      # reordered: identical
        h2, t2 = _gpu_trace(torch_cuda, bvh, rays, reorder=level)
        assert np.array_equal(h, h2) and np.array_equal(t, t2)
        h2, t2 = _gpu_trace(torch_cuda, bvh, rays, reorder=level, kernel=4)
        assert np.array_equal(h, h2) and np.array_equal(t, t2)
    rng = np.random.default_rng(123)
    pick = np.concatenate([rng.choice(len(coh), 4096, replace=False),
                           len(coh) + rng.choice(len(inc), 4096, replace=False)])
    h_ref, t_ref = oracle_lib.trace_brute_force(sc.verts, rays[pick])
    _compare(h[pick], t[pick], h_ref, t_ref)
    pick2 = rng.choice(len(rays), 131072, replace=False)
    osc = oracle_lib.OracleScene(sc, use_bvh=True)
    h2, t2 = osc.trace(rays[pick2])
    _compare(h[pick2], t[pick2], h2, t2)
    assert (h[:len(coh)] >= 0).mean() > 0.3    # the 16:9 view extends past the cube


def test_trace_option_errors(torch_cuda):
    """Invalid options are rejected by the host before any launch."""
    _log("case: trace option validation")
    sc = scenes.small_soup(64, 1)
    bvh = api.build_bvh(sc.verts, sc.tri_mat)
    r = torch_cuda.from_numpy(scenes.random_rays(100, 1)).cuda()
    for kw in (dict(block=100), dict(block=512), dict(kernel=8), dict(kernel=-1), dict(kernel=4, refill=64),
               dict(kernel=7, refill=64), dict(kernel=7, slice_rays=-1), dict(kernel=7, slice_rays=(1 << 24) + 1),
               dict(tile_width=10, kernel=7), dict(reorder=3), dict(tile_width=7), dict(tile_width=-1),
               dict(tile_width=10, reorder=1), dict(tile_width=10, kernel=2), dict(link_set=6)):
        with pytest.raises(api.PMError) as e:
            api.trace_rays(bvh, r, **kw)
        assert e.value.code == api.PM_ERR_ARG, kw
    bvh.destroy()


def test_probe_chase_matches_host(torch_cuda):
    """The memory microbenchmark walks the chains its header defines (host model, several tiles and a ragged tail)."""
    _log("case: probe chase 2^10 rows, 1000 lanes, 37 steps")
    rng = np.random.default_rng(5)
    rows = rng.integers(-2**31, 2**31, size=(1 << 10, 4), dtype=np.int64).astype(np.int32)
    n_lanes, steps = 1000, 37
    got = api.probe_chase(torch_cuda.from_numpy(rows).cuda(), steps, n_lanes).cpu().numpy().view(np.uint32)
    u = rows.view(np.uint32)
    mask = np.uint32((1 << 10) - 1)
    lane = np.arange(n_lanes, dtype=np.uint64)
    r = ((lane * 0x9E3779B1) & 0xFFFFFFFF).astype(np.uint32) & mask
    salt = ((lane * 0x85EBCA77) & 0xFFFFFFFF).astype(np.uint32)
    acc = np.zeros(n_lanes, dtype=np.uint32)
    for _ in range(steps):
        q = u[r]
        acc ^= (q[:, 0] ^ q[:, 1]) ^ (q[:, 2] ^ q[:, 3])
        r = (q[:, 0] ^ salt) & mask
    assert np.array_equal(got, acc)


def test_multi_batch_equals_single_calls(torch_cuda):
    """pm_trace_rays_multi: batches traced concurrently give exactly the single-call results (three batches, two calls)."""
    _log("case: multi-batch trace (packets + bucketed postponed + per-ray with counters), soup 2^14")
    sc = scenes.soup_scene(1 << 14, 4)
    bvh = api.build_bvh(sc.verts, sc.tri_mat)
    cam = scenes.pinhole_rays(scenes.Camera(pos=(0.5, 0.5, -1.5), look=(0.5, 0.5, 0.5), up=(0, 1, 0), tan_half_fov=0.4,
                                            width=96, height=40))
    inc = scenes.random_rays(5000, 9)
    inc2 = scenes.random_rays(777, 10)
    rc, ri, ri2 = (torch_cuda.from_numpy(np.ascontiguousarray(x)).cuda() for x in (cam, inc, inc2))
    kc = dict(kernel=api.TRACE_PACKET, block=64, tile_width=96)
    ki = dict(kernel=api.TRACE_POSTPONED, refill=32, reorder=1, block=64)
    ref = [api.trace_rays(bvh, rc, **kc), api.trace_rays(bvh, ri, **ki)]
    cnt_ref = torch_cuda.zeros((len(inc2), 2), dtype=torch_cuda.int32, device="cuda")
    ref.append(api.trace_rays(bvh, ri2, counters=cnt_ref))
    ref = [(h.cpu().numpy(), t.cpu().numpy()) for h, t in ref]
    for call in range(2):
        cnt = torch_cuda.zeros((len(inc2), 2), dtype=torch_cuda.int32, device="cuda")
        got = api.trace_rays_multi(bvh, [dict(rays=ri, **ki), dict(rays=rc, **kc), dict(rays=ri2, counters=cnt)])
        got = [got[1], got[0], got[2]]
        for (h, t), (hr, tr) in zip(got, ref):
            assert np.array_equal(h.cpu().numpy(), hr), call
            assert np.array_equal(t.cpu().numpy(), tr), call
        assert torch_cuda.equal(cnt, cnt_ref), call
        # two batches, bucketed postponed walk + packets over image tiles: one fused launch
        two = api.trace_rays_multi(bvh, [dict(rays=rc, **kc), dict(rays=ri, **ki)])
        for (h, t), (hr, tr) in zip(two, ref[:2]):
            assert np.array_equal(h.cpu().numpy(), hr) and np.array_equal(t.cpu().numpy(), tr), call
    # the fused launch in statistics mode: the same hits, and per-ray counts from each walk
    cc = torch_cuda.zeros((len(cam), 2), dtype=torch_cuda.int32, device="cuda")
    ci = torch_cuda.zeros((len(inc), 2), dtype=torch_cuda.int32, device="cuda")
    two = api.trace_rays_multi(bvh, [dict(rays=ri, counters=ci, **ki), dict(rays=rc, counters=cc, **kc)])
    for (h, t), (hr, tr) in zip(two, [ref[1], ref[0]]):
        assert np.array_equal(h.cpu().numpy(), hr) and np.array_equal(t.cpu().numpy(), tr)
    cc1 = torch_cuda.zeros_like(cc)
    ci1 = torch_cuda.zeros_like(ci)
    api.trace_rays(bvh, rc, counters=cc1, **kc)
    api.trace_rays(bvh, ri, counters=ci1, **ki)
    assert torch_cuda.equal(cc, cc1)               # packets: the same walk either way
    assert int(ci[:, 0].min()) >= 1 and int(ci1[:, 0].min()) >= 1
    assert (ref[0][0] >= 0).any() and (ref[1][0] >= 0).any()
    bvh.destroy()



def test_probe_stream_copy_and_read(torch_cuda):
    """pm_probe_stream: the copy reproduces the source exactly; the read mode's
    XOR of every word equals the host's; bad arguments are refused."""
    _log("case: stream probe")
    torch = torch_cuda
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    for n_words in (16, 4096 + 48, (1 << 22) + 16 * 7):
        src = torch.randint(-2**31, 2**31 - 1, (n_words,), dtype=torch.int32, device="cuda", generator=g)
        dst = torch.zeros_like(src)
        api.probe_stream(src, dst)
        out = torch.zeros(1, dtype=torch.int32, device="cuda")
        api.probe_stream(src, out=out)
        torch.cuda.synchronize()
        assert torch.equal(dst, src)
        h = src.cpu().numpy().view(np.uint32)
        assert int(out.cpu().numpy().view(np.uint32)[0]) == int(np.bitwise_xor.reduce(h))
    with pytest.raises(api.PMError):
        api.probe_stream(src[:3], dst)            # 12 bytes: not a multiple of 64
