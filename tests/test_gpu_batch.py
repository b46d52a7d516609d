"""Batched rendering (pm_batch_*): one persistent launch per stage for all
scenes, hipGraph replay and autotuning.  Results must equal per-scene renders
bit for bit (fixed-point flux makes them independent of scheduling), and the
small scenes must equal the oracle."""
import math
import os
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


def _mixed():
    out = []
    out.append((scenes.box_scene(64, 64), 1 << 14, 0.05 * math.sqrt(3.0), 1))
    out.append((scenes.box_scene(33, 17), 1 << 10, 0.1, 2))
    out.append((scenes.furnace_scene(rho=0.5, width=16, height=16), 1 << 13, 0.05, 3))
    sc = scenes.procedural_scene(width=97, height=61, hf_cells=20, sphere_level=2, glass_level=3, seed=3)
    out.append((sc, 1 << 15, 0.01, 4))
    sc2 = scenes.procedural_scene(width=40, height=40, hf_cells=8, sphere_level=1, glass_level=1, seed=9)
    out.append((sc2, 1 << 12, 0.02, 5))
    out.append((scenes.box_scene(7, 5), 1, 0.1, 6))
    return out


def _single(torch, sc, Np, r0, seed, K):
    s = api.Sppm(sc, api.sppm_params(Np, r0=r0, seed=seed))
    s.iterate(K)
    img = s.resolve().cpu().numpy()
    v = s.views()
    st = {k: v[k].cpu().numpy() for k in ("N", "R2", "tau", "D")}
    s.destroy()
    return img, st


@pytest.mark.parametrize("chunk,block,graph", [(1024, 256, True), (64, 128, False), (4096, 128, True)])
def test_batch_equals_single_scene_renders(torch_cuda, oracle_lib, chunk, block, graph):
    _log(f"case: batch chunk={chunk} block={block} graph={graph}")
    work = _mixed()
    K = 3
    b = api.Batch([w[0] for w in work], [api.sppm_params(w[1], r0=w[2], seed=w[3]) for w in work],
                  chunk=chunk, block=block, use_graph=graph)
    b.iterate(K)
    imgs = [im.cpu().numpy() for im in b.resolve()]
    b.status()
    info = b.info()
    assert info["chunk"] == chunk and info["block"] == block and info["uses_graph"] == graph
    for i, (sc, Np, r0, seed) in enumerate(work):
        ref_img, ref_st = _single(torch_cuda, sc, Np, r0, seed, K)
        assert np.array_equal(imgs[i], ref_img), i
        v = b.views(i)
        for k in ("N", "R2", "tau", "D"):
            assert np.array_equal(v[k].cpu().numpy(), ref_st[k]), (i, k)
    # the small scenes against the oracle directly
    for i in (1, 2, 5):
        sc, Np, r0, seed = work[i]
        ref = oracle_lib.sppm_run(oracle_lib.OracleScene(sc), seed, Np, K, r0=r0).image
        assert np.array_equal(imgs[i].ravel(), ref)
    b.destroy()


def test_autotune_and_cache(torch_cuda, tmp_path):
    _log("case: batch autotune + cache")
    os.environ["PM_AUTOTUNE_CACHE"] = str(tmp_path / "tune.txt")
    try:
        work = _mixed()
        prm = [api.sppm_params(w[1], r0=w[2], seed=w[3]) for w in work]
        b = api.Batch([w[0] for w in work], prm, autotune=True)
        info = b.info()
        assert len(info["candidates"]) == 8 and not info["tuned_from_cache"]
        best = min(info["candidates"], key=lambda c: c[2])
        assert (info["chunk"], info["block"]) == (best[0], best[1])
        assert info["iterations"] == 0          # the state was reset after tuning
        b.iterate(2)
        imgs = [im.cpu().numpy() for im in b.resolve()]
        b.destroy()
        b2 = api.Batch([w[0] for w in work], prm, autotune=True)
        info2 = b2.info()
        assert info2["tuned_from_cache"] and (info2["chunk"], info2["block"]) == (info["chunk"], info["block"])
        b2.destroy()
        ref = api.render_batch([w[0] for w in work], prm, 2, chunk=512, block=256)
        for a, r in zip(imgs, ref):
            assert np.array_equal(a, r.cpu().numpy())
    finally:
        del os.environ["PM_AUTOTUNE_CACHE"]


def test_batch_overflow_reported(torch_cuda):
    _log("case: batch overflow")
    work = [(scenes.box_scene(8, 8), api.sppm_params(256, r0=0.1)),
            (scenes.furnace_scene(rho=0.9, width=8, height=8), api.sppm_params(256, r0=0.05, store_factor=1))]
    b = api.Batch([w[0] for w in work], [w[1] for w in work], chunk=128)
    b.iterate(1)
    with pytest.raises(api.PMError) as e:
        b.status()
    assert e.value.code == api.PM_ERR_OVERFLOW
    b.destroy()


def test_batched_workload_sample_matches_single(torch_cuda):
    """A few scenes of the 32-scene uneven workload, batched vs alone."""
    _log("case: batched workload sample")
    work = scenes.batch_workload()[:6]
    prm = [api.sppm_params(Np, r0=r0, seed=11 + i) for i, (_, Np, r0) in enumerate(work)]
    imgs = api.render_batch([w[0] for w in work], prm, 2, chunk=2048, block=256)
    for i, (sc, Np, r0) in enumerate(work):
        ref, _ = _single(torch_cuda, sc, Np, r0, 11 + i, 2)
        assert np.array_equal(imgs[i].cpu().numpy(), ref)


def test_full_batched_workload_autotuned_equals_single_and_oracle(torch_cuda, oracle_lib, tmp_path):
    """The batched workload as the benchmark runs it: all 32 uneven scenes,
    16 iterations, chunk and block picked by the autotuner, one graph per
    iteration.  Every scene's image and state equal its own single-handle
    render bit for bit, and the three scenes with the fewest photons also
    equal the oracle."""
    _log("case: batched workload, 32 scenes, K = 16, autotuned")
    os.environ["PM_AUTOTUNE_CACHE"] = str(tmp_path / "tune.txt")
    try:
        work = scenes.batch_workload()
        assert len(work) == 32
        K = 16
        prm = [api.sppm_params(Np, alpha=0.7, r0=r0, seed=100 + i) for i, (_, Np, r0) in enumerate(work)]
        b = api.Batch([w[0] for w in work], prm, autotune=True)
        info = b.info()
        _log(f"  autotuned chunk {info['chunk']} block {info['block']}")
        b.iterate(K)
        imgs = [im.cpu().numpy() for im in b.resolve()]
        b.status()
        states = [{k: v.cpu().numpy() for k, v in b.views(i).items() if k in ("N", "R2", "tau", "D")}
                  for i in range(len(work))]
        b.destroy()
    finally:
        del os.environ["PM_AUTOTUNE_CACHE"]
    for i, (sc, Np, r0) in enumerate(work):
        s = api.Sppm(sc, prm[i])
        s.iterate(K)
        ref = s.resolve().cpu().numpy()
        s.status()
        v = s.views()
        assert np.array_equal(imgs[i], ref), i
        for k in ("N", "R2", "tau", "D"):
            assert np.array_equal(states[i][k], v[k].cpu().numpy()), (i, k)
        s.destroy()
    _log("  32 scenes equal their single renders; oracle on the three smallest")
    smallest = sorted(range(len(work)), key=lambda i: (work[i][1], work[i][0].n_tri))[:3]
    for i in smallest:
        sc, Np, r0 = work[i]
        ref = oracle_lib.sppm_run(oracle_lib.OracleScene(sc), 100 + i, Np, K, alpha=0.7, r0=r0).image
        assert np.array_equal(imgs[i].ravel(), ref), i
