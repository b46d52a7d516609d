"""GPU parity of the SPPM iteration against the oracle, stage by stage.

The GPU path and the oracle evaluate the same float32/float64 operations in
the same order and sum flux in integer fixed point, so hit points, stored
photons (as a set keyed by path and bounce), per-pixel counts and fluxes and
the per-pixel state match exactly; the image is also checked against the
stated per-pixel relative tolerance 1e-4.
"""
import math
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


def _gpu_stage(torch, s):
    torch.cuda.synchronize()
    v = s.views()
    out = {k: (t.cpu().numpy() if hasattr(t, "cpu") else t) for k, t in v.items()}
    n = int(out["photon_count"][0])
    out["n_photons"] = n
    ph = out["photons"][:min(n, len(out["photons"]))]
    meta = ph[:, 7].view(np.uint32)
    order = np.argsort(meta, kind="stable")
    out["ph_sorted"] = ph[order]
    out["ph_path"] = (meta[order] >> 5).astype(np.uint32)
    out["ph_bounce"] = (meta[order] & 31).astype(np.uint32)
    return out


def _check_hit_points(g, hp):
    valid_g = g["hp_nrm"][:, 3].view(np.int32) >= 0
    assert np.array_equal(valid_g, hp.valid > 0)
    v = valid_g
    assert np.array_equal(g["hp_pos"][v, :3], hp.x[v])
    assert np.array_equal(g["hp_nrm"][v, :3], hp.n[v])
    assert np.array_equal(g["hp_pos"][v, 3], hp.wk[v])
    assert np.array_equal(g["hp_nrm"][v, 3].view(np.int32), hp.mat[v])


def _check_photons(g, ph):
    assert g["n_photons"] == ph.n
    d = ph.view()
    assert np.array_equal(g["ph_path"], d["path"])
    assert np.array_equal(g["ph_bounce"], d["bounce"])
    s = g["ph_sorted"]
    assert np.array_equal(s[:, 0:3], d["x"])
    assert np.array_equal(s[:, 3], d["phi"])
    assert np.array_equal(s[:, 4:7], d["w"])


def _run_parity(torch, oracle_lib, sc, Np, K, r0, seed, alpha=0.7, stage_iters=1, **kw):
    osc = oracle_lib.OracleScene(sc)
    params = api.sppm_params(Np, alpha=alpha, r0=r0, seed=seed, **kw)
    s = api.Sppm(sc, params)
    P = osc.P
    N, R2, tau, D = np.zeros(P), np.full(P, r0 * r0), np.zeros(P), np.zeros(P)
    for k in range(K):
        s.iterate(1)
        hp = oracle_lib.eye_pass(osc, seed, k)
        ph = oracle_lib.photon_pass(osc, seed, k, Np)
        M, Phi = oracle_lib.gather(hp, ph, R2)
        if k < stage_iters:
            g = _gpu_stage(torch, s)
            _check_hit_points(g, hp)
            _check_photons(g, ph)
            assert np.array_equal(g["M"].view(np.uint32), M)
            assert np.array_equal(g["Phi"].view(np.uint64), Phi)
        oracle_lib.update(hp.valid, M, Phi, alpha, N, R2, tau)
        D += hp.d_add
    img = s.resolve().cpu().numpy().ravel()
    s.status()
    g = _gpu_stage(torch, s)
    assert np.array_equal(g["N"], N)
    assert np.array_equal(g["R2"], R2)
    assert np.array_equal(g["tau"], tau)
    assert np.array_equal(g["D"], D)
    ref = oracle_lib.resolve(R2, tau, D, K)
    nz = ref != 0
    rel = np.abs(img[nz] - ref[nz]) / np.abs(ref[nz])
    assert rel.max(initial=0) <= 1e-4
    assert np.array_equal(img, ref)
    # and the one-call oracle run agrees with this stepwise one
    full = oracle_lib.sppm_run(osc, seed, Np, K, alpha=alpha, r0=r0)
    assert np.array_equal(full.image, ref)
    s.destroy()
    return img


def test_box_scene_parity(torch_cuda, oracle_lib):
    """Room with two boxes, 64x64, 2 iterations of 2^14 photons, r0 = 0.05 diag."""
    _log("case: box scene 64x64, 2 x 2^14 photons")
    sc = scenes.box_scene(64, 64)
    img = _run_parity(torch_cuda, oracle_lib, sc, 1 << 14, 2, 0.05 * math.sqrt(3.0), seed=1, stage_iters=2)
    assert (img > 0).mean() > 0.5


def test_specular_scene_parity(torch_cuda, oracle_lib):
    """Reduced procedural scene with mirror and glass spheres, ragged image size."""
    _log("case: reduced procedural scene 97x61")
    sc = scenes.procedural_scene(width=97, height=61, hf_cells=20, sphere_level=2, glass_level=3, seed=3)
    diag = float(np.linalg.norm(sc.verts.reshape(-1, 3).max(0) - sc.verts.reshape(-1, 3).min(0)))
    _run_parity(torch_cuda, oracle_lib, sc, 1 << 15, 3, 0.05 * diag * 64 / 97, seed=3)


@pytest.mark.parametrize("photon_kernel,refill", [(1, 0), (2, 1), (2, 8), (2, 64), (4, 0), (4, 1), (4, 16), (4, 64),
                                                  (5, 0), (6, 0), (6, 1), (6, 64)])
def test_photon_kernels_parity(torch_cuda, oracle_lib, photon_kernel, refill):
    """One path per lane, lanes regenerating paths, and lanes regenerating rays
    give the same photons and images."""
    _log(f"case: photon kernel {photon_kernel} refill {refill}")
    sc = scenes.procedural_scene(width=61, height=37, hf_cells=12, sphere_level=2, glass_level=2, seed=8)
    _run_parity(torch_cuda, oracle_lib, sc, 3 * (1 << 12) + 5, 2, 0.02, seed=8, stage_iters=2,
                photon_kernel=photon_kernel, refill=refill)


@pytest.mark.parametrize("pass_threads,passes", [(0, 0), (100, 3), (1 << 16, 1), (4096, 64), (1 << 14, 32)])
def test_one_bounce_per_pass_parity(torch_cuda, oracle_lib, pass_threads, passes):
    """The paper's schedule as written (one bounce per thread per launch, a new
    path in the pass after one ends) stores the same photons as the other
    schedules, whatever the thread count and however many paths the passes
    leave to the final drain."""
    _log(f"case: one bounce per pass, threads {pass_threads} passes {passes}")
    sc = scenes.procedural_scene(width=61, height=37, hf_cells=12, sphere_level=2, glass_level=2, seed=8)
    Np = 3 * (1 << 12) + 5
    _run_parity(torch_cuda, oracle_lib, sc, Np, 2, 0.02, seed=8, stage_iters=2,
                photon_kernel=api.PHOTON_PASSES, pass_threads=pass_threads, passes=passes)
    # photon_count[3]: paths the passes left unfinished or unstarted
    s = api.Sppm(sc, api.sppm_params(Np, r0=0.02, seed=8, photon_kernel=api.PHOTON_PASSES,
                                     pass_threads=pass_threads, passes=passes))
    s.iterate(1)
    torch_cuda.cuda.synchronize()
    left = int(s.views()["photon_count"][3])
    if pass_threads >= Np and passes >= 32:
        assert left == 0      # every path starts in the first pass and has at most 32 bounces
    elif pass_threads == 100:
        assert left >= Np - 3 * 100
    assert 0 <= left <= Np
    s.destroy()


def test_fine_grid_with_hash_collisions_parity(torch_cuda, oracle_lib):
    """The exact gather's fine cells (edge R_max (1 + 2^-5), up to 3x3x3 cells
    per hit point) on the smallest table (2^12 buckets) and a large radius:
    about 20^3 cells share 4096 buckets, so the cells around a hit point often
    collide, and a bucket reached twice must be counted once."""
    _log("case: fine grid, 2^12 buckets, r0 = 0.05")
    sc = scenes.procedural_scene(width=61, height=37, hf_cells=12, sphere_level=2, glass_level=2, seed=8)
    _run_parity(torch_cuda, oracle_lib, sc, 1000, 3, 0.05, seed=12, stage_iters=3)


def test_dense_discs_wave_gather_parity(torch_cuda, oracle_lib):
    """Radii large enough that most hit points' buckets hold hundreds to
    thousands of photons, so the gather scans them with the whole wavefront
    and adds the lanes' partial counts and fixed-point sums: M and flux must
    still equal the oracle's exactly."""
    _log("case: box scene 32x32, 2^15 photons, r0 = 0.2")
    sc = scenes.box_scene(32, 32)
    _run_parity(torch_cuda, oracle_lib, sc, 1 << 15, 2, 0.2, seed=14, stage_iters=2)
    # both ways of scanning were taken: a hit point's buckets hold at least its
    # M photons, and the wave scans them together from 256 photons on
    osc = oracle_lib.OracleScene(sc)
    hp = oracle_lib.eye_pass(osc, 14, 0)
    M, _ = oracle_lib.gather(hp, oracle_lib.photon_pass(osc, 14, 0, 1 << 15), np.full(osc.P, 0.04))
    v = hp.valid > 0
    assert (M[v] >= 256).mean() > 0.5 and (M[v] < 64).any()


@pytest.mark.parametrize("single_link_set", [1, 4, 6])
def test_single_link_set_parity(torch_cuda, oracle_lib, single_link_set):
    """Every ray walking one link set (a single threaded BVH) changes nothing
    but speed: stage-by-stage parity with the oracle still holds."""
    _log(f"case: single link set {single_link_set - 1}")
    sc = scenes.procedural_scene(width=61, height=37, hf_cells=12, sphere_level=2, glass_level=2, seed=8)
    _run_parity(torch_cuda, oracle_lib, sc, 1 << 12, 2, 0.02, seed=9, stage_iters=2,
                single_link_set=single_link_set)


@pytest.mark.parametrize("case", ["two_lights", "mirror_floor", "mirror_corridor", "specular_furnace",
                                  "polygon_light_mirror"])
def test_pin_scene_parity(torch_cuda, oracle_lib, case):
    """The scenes that pin the oracle's emission and specular transport
    (unequal lights, a planar mirror, a mirror corridor up to the eye depth
    cap, a furnace with a mirror box and a glass sphere, a mirror over a floor
    with no Russian-roulette survival): the GPU's stages equal the oracle's."""
    _log(f"case: pin scene {case}")
    if case == "two_lights":
        sc, Np, r0 = scenes.two_light_scene(Le=(1.0, 12.0), half=(0.1, 0.05), width=24, height=16), 1 << 13, 0.05
    elif case == "mirror_floor":
        sc, Np, r0 = scenes.mirror_floor_scene(), 1 << 13, 0.05
    elif case == "mirror_corridor":
        sc, Np, r0 = scenes.mirror_corridor_scene(), 1 << 12, 0.1
    elif case == "specular_furnace":
        sc, Np, r0 = scenes.specular_furnace_scene(width=24, height=20), 1 << 13, 0.05
    else:
        sc, Np, r0 = scenes.polygon_light_mirror_scene(), 1 << 13, 0.04
    img = _run_parity(torch_cuda, oracle_lib, sc, Np, 2, r0, seed=6, stage_iters=2)
    assert (img > 0).any()


def test_degenerate_cases(torch_cuda, oracle_lib):
    _log("case: single photon, no emitter, tiny image")
    sc = scenes.box_scene(5, 3)
    _run_parity(torch_cuda, oracle_lib, sc, 1, 2, 0.1, seed=4, stage_iters=2)
    dark = scenes.box_scene(7, 5)
    dark.mat_Le[:] = 0
    img = _run_parity(torch_cuda, oracle_lib, dark, 64, 1, 0.1, seed=5)
    assert np.all(img == 0)


def test_determinism_across_schedules(torch_cuda):
    """Integer counts and fixed-point sums make the result independent of
    thread order: repeated runs and every photon schedule give bit-identical
    per-pixel state and images (no oracle involved)."""
    _log("case: determinism across runs and photon schedules")
    sc = scenes.procedural_scene(width=61, height=37, hf_cells=12, sphere_level=2, glass_level=2, seed=8)
    out = []
    for kw in (dict(), dict(), dict(photon_kernel=1), dict(photon_kernel=2, refill=1), dict(photon_kernel=3),
               dict(photon_kernel=3, pass_threads=333, passes=2), dict(photon_kernel=4), dict(photon_kernel=4, refill=5),
               dict(photon_kernel=5), dict(photon_kernel=6), dict(photon_kernel=6, refill=3)):
        s = api.Sppm(sc, api.sppm_params(1 << 13, r0=0.03, seed=21, **kw))
        s.iterate(3)
        img = s.resolve().cpu().numpy()
        torch_cuda.cuda.synchronize()
        v = s.views()
        out.append([img] + [v[k].cpu().numpy().copy() for k in ("N", "R2", "tau", "D", "M", "Phi")])
        s.destroy()
    for o in out[1:]:
        for a, b in zip(out[0], o):
            assert np.array_equal(a, b)


def test_flux_fixed_point_overflow_is_reported(torch_cuda):
    """A light so bright that each flux term at 2^52 fixed point passes 2^64:
    the range query flags it and pm_sppm_status reports PM_ERR_OVERFLOW
    naming fixed_shift; the same scene at 2^20 is clean."""
    _log("case: flux fixed-point overflow")
    import dataclasses
    sc = scenes.box_scene(16, 16)
    sc = dataclasses.replace(sc, mat_Le=np.where(sc.mat_Le > 0, np.float32(1e12), sc.mat_Le).astype(np.float32))
    for shift, bad in ((52, True), (20, False)):
        s = api.Sppm(sc, api.sppm_params(1 << 12, r0=0.1, fixed_shift=shift))
        s.iterate(1)
        if bad:
            with pytest.raises(api.PMError) as e:
                s.status()
            assert e.value.code == api.PM_ERR_OVERFLOW and "fixed_shift" in str(e.value)
        else:
            s.status()
        s.destroy()


def test_photon_store_overflow_is_reported(torch_cuda):
    _log("case: photon store overflow")
    sc = scenes.furnace_scene(rho=0.9, width=8, height=8)
    s = api.Sppm(sc, api.sppm_params(256, r0=0.05, store_factor=1))
    s.iterate(1)
    with pytest.raises(api.PMError) as e:
        s.status()
    assert e.value.code == api.PM_ERR_OVERFLOW
    s.destroy()


def test_render_one_call_matches_oracle(torch_cuda, oracle_lib):
    _log("case: pm_render white furnace")
    sc = scenes.furnace_scene(rho=0.5, Le=1.0, width=16, height=16)
    img = api.render(sc, api.sppm_params(1 << 15, r0=0.05, seed=7), 4).cpu().numpy().ravel()
    ref = oracle_lib.sppm_run(oracle_lib.OracleScene(sc), 7, 1 << 15, 4, r0=0.05).image
    assert np.array_equal(img, ref)
    assert abs(img.mean() / 2.0 - 1) < 0.015


def test_full_size_procedural_iteration(torch_cuda, oracle_lib):
    """250k-triangle scene at 1280x720 with 2^20 photons: one full iteration
    on the GPU compared with one full oracle iteration (oracle BVH)."""
    _log("case: procedural 250k triangles, 1280x720, 2^20 photons")
    sc = scenes.procedural_scene()
    diag = float(np.linalg.norm(sc.verts.reshape(-1, 3).max(0) - sc.verts.reshape(-1, 3).min(0)))
    r0 = 0.05 * diag * 64 / 1280
    Np, seed = 1 << 20, 3
    _run_parity(torch_cuda, oracle_lib, sc, Np, 1, r0, seed=seed)


def test_full_size_procedural_eight_iterations(torch_cuda, oracle_lib):
    """The full SPPM workload's scene at full size (1280x720, 2^20 photons)
    for 8 consecutive iterations, so the update runs with N > 0 and shrinking
    radii: per-iteration M and flux, the stored photons of the first and last
    iterations, and the final N, R^2, tau, D and image equal the oracle's."""
    _log("case: procedural 250k triangles, 1280x720, 2^20 photons, 8 iterations")
    sc = scenes.procedural_scene()
    diag = float(np.linalg.norm(sc.verts.reshape(-1, 3).max(0) - sc.verts.reshape(-1, 3).min(0)))
    r0 = 0.05 * diag * 64 / 1280
    Np, seed, K, alpha = 1 << 20, 3, 8, 0.7
    osc = oracle_lib.OracleScene(sc)
    s = api.Sppm(sc, api.sppm_params(Np, alpha=alpha, r0=r0, seed=seed))
    P = osc.P
    N, R2, tau, D = np.zeros(P), np.full(P, r0 * r0), np.zeros(P), np.zeros(P)
    for k in range(K):
        s.iterate(1)
        hp = oracle_lib.eye_pass(osc, seed, k)
        ph = oracle_lib.photon_pass(osc, seed, k, Np)
        M, Phi = oracle_lib.gather(hp, ph, R2)
        torch_cuda.cuda.synchronize()
        v = s.views()
        if k in (0, K - 1):
            g = _gpu_stage(torch_cuda, s)
            _check_hit_points(g, hp)
            _check_photons(g, ph)
        assert np.array_equal(v["M"].cpu().numpy().view(np.uint32), M), k
        assert np.array_equal(v["Phi"].cpu().numpy().view(np.uint64), Phi), k
        oracle_lib.update(hp.valid, M, Phi, alpha, N, R2, tau)
        D += hp.d_add
        _log(f"  iteration {k} equal; {int((hp.valid > 0).sum())} hit points, {ph.n} photons")
    img = s.resolve().cpu().numpy().ravel()
    s.status()
    v = s.views()
    for name, ref in (("N", N), ("R2", R2), ("tau", tau), ("D", D)):
        assert np.array_equal(v[name].cpu().numpy(), ref), name
    # about 47% of the pixels hold a hit point; nearly all of those have shrunk
    assert np.all(R2 <= r0 * r0) and (R2 < r0 * r0).mean() > 0.4 and N.max() > 0
    ref = oracle_lib.resolve(R2, tau, D, K)
    assert np.array_equal(img, ref)
    s.destroy()


def test_checkpoint_resume_is_bit_identical(torch_cuda):
    """K iterations straight equal k iterations, a checkpoint, a fresh handle
    loaded from it and K - k more (counter-keyed streams make resume exact);
    a checkpoint is refused by a handle with other parameters."""
    _log("case: checkpoint and resume, reduced procedural scene")
    sc = scenes.procedural_scene(width=61, height=37, hf_cells=12, sphere_level=2, glass_level=2, seed=8)
    prm = api.sppm_params(1 << 13, r0=0.02, seed=21, record_iterations=4)
    a = api.Sppm(sc, prm)
    a.iterate(4)
    ref = a.resolve().cpu().numpy()
    ref_state = {k: v.cpu().numpy() for k, v in a.views().items() if k in ("N", "R2", "tau", "D")}
    g = torch_cuda.ones((sc.camera.height, sc.camera.width), device="cuda")
    ref_grad = a.adjoint(g, sc.albedo_params).cpu().numpy()
    a.destroy()

    b = api.Sppm(sc, prm)
    b.iterate(2)
    ck = b.save()
    b.destroy()
    c = api.Sppm(sc, prm)
    c.load(ck)
    assert c.views()["iterations"] == 2
    c.iterate(2)
    img = c.resolve().cpu().numpy()
    assert np.array_equal(img, ref)
    v = c.views()
    for k in ("N", "R2", "tau", "D"):
        assert np.array_equal(v[k].cpu().numpy(), ref_state[k]), k
    # the adjoint's sums are integer sums: the resumed gradient is bit-identical
    assert np.array_equal(c.adjoint(g, sc.albedo_params).cpu().numpy(), ref_grad)
    c.destroy()

    # another seed, a truncated buffer and a foreign buffer are all refused
    d = api.Sppm(sc, api.sppm_params(1 << 13, r0=0.02, seed=22, record_iterations=4))
    for bad in (ck, ck[:100], b"x" * len(ck)):
        with pytest.raises(api.PMError) as e:
            d.load(bad)
        assert e.value.code == api.PM_ERR_ARG
    d.destroy()
    e2 = api.Sppm(sc, prm)
    with pytest.raises(api.PMError):
        e2.load(ck[:len(ck) - 8])
    assert e2.views()["iterations"] == 0
    e2.destroy()


def _run_stochastic_parity(torch, oracle_lib, sc, Np, K, r0, seed, alpha=0.7, **kw):
    """Stochastic spatial hashing: per-iteration M and Phi, the final state and
    the image equal the oracle's estimate bit for bit (the survivor of each
    entry is the smallest key, whatever the order of the atomics)."""
    osc = oracle_lib.OracleScene(sc)
    lo = oracle_lib.scene_lo(sc)
    s = api.Sppm(sc, api.sppm_params(Np, alpha=alpha, r0=r0, seed=seed, gather_mode=1, **kw))
    P = osc.P
    N, R2, tau, D = np.zeros(P), np.full(P, r0 * r0), np.zeros(P), np.zeros(P)
    for k in range(K):
        s.iterate(1)
        hp = oracle_lib.eye_pass(osc, seed, k)
        ph = oracle_lib.photon_pass(osc, seed, k, Np)
        M, Phi = oracle_lib.gather_stochastic(hp, ph, R2, lo, Np, seed, k)
        g = _gpu_stage(torch, s)
        assert g["n_photons"] == ph.n
        assert np.array_equal(g["M"].view(np.uint32), M)
        assert np.array_equal(g["Phi"].view(np.uint64), Phi)
        oracle_lib.update(hp.valid, M, Phi, alpha, N, R2, tau)
        D += hp.d_add
    img = s.resolve().cpu().numpy().ravel()
    s.status()
    g = _gpu_stage(torch, s)
    for name, ref in (("N", N), ("R2", R2), ("tau", tau), ("D", D)):
        assert np.array_equal(g[name], ref), name
    ref = oracle_lib.resolve(R2, tau, D, K)
    assert np.array_equal(img, ref)
    full = oracle_lib.sppm_run(osc, seed, Np, K, alpha=alpha, r0=r0, gather_method=2)
    assert np.array_equal(full.image, ref)
    s.destroy()
    return img


@pytest.mark.parametrize("case", ["box", "specular", "tiny"])
def test_stochastic_hashing_parity(torch_cuda, oracle_lib, case):
    _log(f"case: stochastic spatial hashing, {case}")
    if case == "box":
        _run_stochastic_parity(torch_cuda, oracle_lib, scenes.box_scene(64, 64), 1 << 14, 3, 0.05 * math.sqrt(3.0), 1)
    elif case == "specular":
        sc = scenes.procedural_scene(width=97, height=61, hf_cells=20, sphere_level=2, glass_level=3, seed=3)
        _run_stochastic_parity(torch_cuda, oracle_lib, sc, 3 * (1 << 12) + 7, 2, 0.02, 5, photon_kernel=1)
    else:
        _run_stochastic_parity(torch_cuda, oracle_lib, scenes.box_scene(5, 3), 1, 2, 0.1, 4)


def test_stochastic_hashing_full_size_iteration(torch_cuda, oracle_lib):
    """250k triangles, 1280x720, 2^20 photons: one stochastic-hashing iteration
    equals the oracle's."""
    _log("case: stochastic spatial hashing, procedural 250k triangles, 2^20 photons")
    sc = scenes.procedural_scene()
    diag = float(np.linalg.norm(sc.verts.reshape(-1, 3).max(0) - sc.verts.reshape(-1, 3).min(0)))
    _run_stochastic_parity(torch_cuda, oracle_lib, sc, 1 << 20, 1, 0.05 * diag * 64 / 1280, 3)


def test_stochastic_hashing_is_refused_where_unsupported(torch_cuda):
    _log("case: stochastic hashing in a batch")
    sc = scenes.box_scene(8, 8)
    with pytest.raises(api.PMError) as e:
        api.Batch([sc, sc], [api.sppm_params(256, r0=0.1), api.sppm_params(256, r0=0.1, gather_mode=1)])
    assert e.value.code == api.PM_ERR_ARG
    _log("case: one-bounce-per-pass photons in a batch")
    with pytest.raises(api.PMError) as e:
        api.Batch([sc, sc], [api.sppm_params(256, r0=0.1), api.sppm_params(256, r0=0.1, photon_kernel=3)])
    assert e.value.code == api.PM_ERR_ARG


def test_profile_counts_and_times(torch_cuda, oracle_lib):
    """PM_PROFILE_COUNT and PM_PROFILE_TIME leave results unchanged; the
    counts of paths, stored photons, hit points and accepted photons equal
    the oracle's, and the other counts and the stage times are consistent."""
    _log("case: profiling counts and stage times")
    sc = scenes.procedural_scene(width=97, height=61, hf_cells=20, sphere_level=2, glass_level=3, seed=3)
    Np, K, r0, seed = 1 << 14, 3, 0.02, 5
    out = {}
    for prof, pk in ((0, 0), (api.PROFILE_COUNT, 0), (api.PROFILE_TIME, 0), (api.PROFILE_COUNT | api.PROFILE_TIME, 0),
                     (api.PROFILE_COUNT | 8, 4), (api.PROFILE_COUNT | 16, 5), (api.PROFILE_COUNT | 32, 2),
                     (api.PROFILE_TIME | 64, 2)):
        s = api.Sppm(sc, api.sppm_params(Np, r0=r0, seed=seed, profile=prof & 3, photon_kernel=pk))
        s.iterate(K)
        img = s.resolve().cpu().numpy()
        s.status()
        out[prof] = (img, {k: v.cpu().numpy() for k, v in s.views().items() if k in ("N", "R2", "tau", "D")},
                     s.stats())
        s.destroy()
    for prof in out:
        assert np.array_equal(out[prof][0], out[0][0])
        for k in ("N", "R2", "tau", "D"):
            assert np.array_equal(out[prof][1][k], out[0][1][k])
    st = out[api.PROFILE_COUNT | api.PROFILE_TIME][2]
    osc = oracle_lib.OracleScene(sc)
    P = osc.P
    R2 = np.full(P, r0 * r0)
    N, tau = np.zeros(P), np.zeros(P)
    stored = hits = accepted = 0
    for k in range(K):
        hp = oracle_lib.eye_pass(osc, seed, k)
        ph = oracle_lib.photon_pass(osc, seed, k, Np)
        M, Phi = oracle_lib.gather(hp, ph, R2)
        stored += ph.n
        hits += int((hp.valid > 0).sum())
        accepted += int(M.astype(np.int64).sum())
        oracle_lib.update(hp.valid, M, Phi, 0.7, N, R2, tau)
    assert st["counted_iterations"] == K and st["timed_iterations"] == K
    assert st["eye_paths"] == K * P and st["photon_paths"] == K * Np
    assert st["photons_stored"] == stored and st["gather_hit_points"] == hits and st["gather_accepted"] == accepted
    assert st["eye_rays"] >= st["eye_paths"] and st["photon_rays"] >= stored
    assert st["eye_box_tests"] >= st["eye_rays"] and st["photon_box_tests"] >= st["photon_rays"]
    assert st["gather_examined"] >= accepted and st["gather_buckets"] >= hits
    for k in ("ms_eye", "ms_photon", "ms_grid", "ms_gather", "ms_update"):
        assert 0 < st[k] < st["ms_iteration"], k
    assert out[api.PROFILE_TIME][2]["eye_paths"] == 0      # counting was off there
    # the ray-granularity, LDS-queue and single-launch regeneration kernels walk the same rays and store the
    # same photons as the default two-phase pass
    for key in (api.PROFILE_COUNT | 8, api.PROFILE_COUNT | 16, api.PROFILE_COUNT | 32):
        st4 = out[key][2]
        for k in ("photon_paths", "photon_rays", "photons_stored", "photon_box_tests", "photon_tri_tests"):
            assert st4[k] == out[api.PROFILE_COUNT][2][k], (key, k)
    with pytest.raises(api.PMError):
        api.Sppm(sc, api.sppm_params(Np, r0=r0, gather_mode=1, profile=api.PROFILE_COUNT))
    with pytest.raises(api.PMError):
        api.Batch([sc, sc], [api.sppm_params(256, r0=0.1, profile=api.PROFILE_TIME)] * 2)


def test_spatial_split_bvh_gives_the_same_render_and_gradient(torch_cuda):
    """A BVH with spatial splits (triangles referenced by several leaves) under
    the SPPM passes: every photon schedule, the images and state, and the
    adjoint's gradient (through torch.autograd) equal those of the plain SAH
    BVH bit for bit, since each walk returns the same closest hit."""
    _log("case: SPPM on a spatial-split BVH (250k-triangle scene, 64x36)")
    torch = torch_cuda
    sc = scenes.procedural_scene(width=64, height=36)
    plain = api.build_bvh(sc.verts, sc.tri_mat)
    split = api.build_bvh(sc.verts, sc.tri_mat, split_alpha=1e-4)
    assert split.info()["n_refs"] > split.info()["n_tri"] == plain.info()["n_refs"]
    for kw in (dict(), dict(photon_kernel=1), dict(photon_kernel=2), dict(photon_kernel=3, pass_threads=4096, passes=4),
               dict(photon_kernel=4), dict(photon_kernel=5)):
        out = []
        for bvh in (plain, split):
            s = api.Sppm(sc, api.sppm_params(1 << 14, r0=0.03, seed=5, **kw), bvh=bvh)
            s.iterate(3)
            img = s.resolve().cpu().numpy()
            torch.cuda.synchronize()
            v = s.views()
            out.append([img] + [v[k].cpu().numpy().copy() for k in ("N", "R2", "tau", "D", "M", "Phi")])
            s.destroy()
        for a, b in zip(*out):
            assert np.array_equal(a, b), kw
    pm = sc.albedo_params
    params = api.sppm_params(1 << 14, r0=0.03, seed=6)
    target = api.render(sc, params, 2, bvh=plain).double() * 0.9
    grads = []
    for bvh in (plain, split):
        rho = torch.tensor(sc.mat_rho[pm], dtype=torch.float64, requires_grad=True)
        Le = torch.tensor(10.0, dtype=torch.float64, requires_grad=True)
        img = api.sppm_render_diff(rho, Le, sc, pm, params, 2, bvh=bvh)
        ((img.double() - target) ** 2).mean().backward()
        grads.append(np.append(rho.grad.cpu().numpy(), Le.grad.item()))
    assert np.array_equal(grads[0], grads[1]) and np.abs(grads[0]).max() > 0
    plain.destroy()
    split.destroy()
