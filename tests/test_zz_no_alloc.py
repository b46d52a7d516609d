"""pm_trace_rays_noalloc: the bucketed trace on the library's static
per-device scratch, for callers that cannot allocate.  Its results must equal
pm_trace_rays_ex's with the same options bit for bit (hit index and t), on
two calls in a row whose second call is smaller (the scratch keeps the first
call's contents), and it must allocate no device memory.
"""
import ctypes
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


def _free_bytes():
    hip = ctypes.CDLL("libamdhip64.so")
    free, total = ctypes.c_size_t(), ctypes.c_size_t()
    assert hip.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    return free.value


def _both(torch, bvh, rays, **kw):
    """(hit, t) of the allocation-free call and of pm_trace_rays_ex, same options."""
    n = rays.shape[0]
    h0 = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    t0 = torch.full((n,), -7.0, dtype=torch.float32, device="cuda")
    api.trace_rays_noalloc(bvh, rays, h0, t0, **kw)
    h1, t1 = api.trace_rays(bvh, rays, **kw)
    torch.cuda.synchronize()
    return h0.cpu().numpy(), t0.cpu().numpy(), h1.cpu().numpy(), t1.cpu().numpy()


@pytest.mark.parametrize("reorder,kernel,refill", [(1, 0, 0), (2, api.TRACE_POSTPONED, 32),
                                                   (1, api.TRACE_PAIRED, 0), (1, api.TRACE_SLICES, 32)])
def test_noalloc_equals_bucketed_trace_two_calls(torch_cuda, reorder, kernel, refill):
    torch = torch_cuda
    _log(f"case: noalloc trace, soup 2^16, reorder {reorder} kernel {kernel}")
    sc = scenes.small_soup(1 << 16, seed=4, spread=0.01)
    bvh = api.build_bvh(sc.verts, sc.tri_mat)
    for n in (200_003, 61_441):    # the second call is smaller than the first
        rays = torch.from_numpy(scenes.random_rays(n, seed=n)).cuda()
        h0, t0, h1, t1 = _both(torch, bvh, rays, reorder=reorder, kernel=kernel, refill=refill, block=64)
        assert np.array_equal(h0, h1) and np.array_equal(t0.view(np.uint32), t1.view(np.uint32))
        assert (h0 >= 0).mean() > 0.2
    bvh.destroy()


def test_noalloc_full_size_soup_and_limits(torch_cuda):
    """The traversal workload's incoherent batch (2^21 rays on 2^20 triangles),
    then a smaller camera batch; the device's free memory does not change over
    calls after the first; n above the maximum and reorder 0 / tile_width are
    refused before any work."""
    torch = torch_cuda
    _log("case: noalloc trace, soup 2^20, 2^21 incoherent rays then 1920x1080 camera rays")
    sc, cam, inc = scenes.soup_workload()
    bvh = api.build_bvh(sc.verts, sc.tri_mat)
    inc_d = torch.from_numpy(inc).cuda()
    cam_d = torch.from_numpy(cam).cuda()
    h0, t0, h1, t1 = _both(torch, bvh, inc_d, reorder=2, kernel=api.TRACE_POSTPONED, refill=32, block=64)
    assert np.array_equal(h0, h1) and np.array_equal(t0.view(np.uint32), t1.view(np.uint32))
    h0, t0, h1, t1 = _both(torch, bvh, cam_d, reorder=1)
    assert np.array_equal(h0, h1) and np.array_equal(t0.view(np.uint32), t1.view(np.uint32))
    # no allocation: outputs are preallocated, so free memory is unchanged
    hit = torch.empty(inc.shape[0], dtype=torch.int32, device="cuda")
    t = torch.empty(inc.shape[0], dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    before = _free_bytes()
    for rays in (inc_d, cam_d, inc_d):
        api.trace_rays_noalloc(bvh, rays, hit, t, reorder=2, kernel=api.TRACE_POSTPONED, refill=32)
    torch.cuda.synchronize()
    assert _free_bytes() == before
    # refusals
    big = torch.empty((api.NOALLOC_MAX_RAYS + 1, 8), dtype=torch.float32, device="cuda")
    hb = torch.empty(api.NOALLOC_MAX_RAYS + 1, dtype=torch.int32, device="cuda")
    tb = torch.empty(api.NOALLOC_MAX_RAYS + 1, dtype=torch.float32, device="cuda")
    with pytest.raises(api.PMError) as e:
        api.trace_rays_noalloc(bvh, big, hb, tb)
    assert e.value.code == api.PM_ERR_ARG and "PM_NOALLOC_MAX_RAYS" in str(e.value)
    with pytest.raises(api.PMError):
        api.trace_rays_noalloc(bvh, inc_d, hit, t, reorder=3)
    h0 = torch.empty(0, dtype=torch.int32, device="cuda")
    api.trace_rays_noalloc(bvh, inc_d[:0], h0, torch.empty(0, dtype=torch.float32, device="cuda"))
    bvh.destroy()
