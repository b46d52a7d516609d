"""GPU adjoint (pm_sppm_adjoint, replay) against the oracle's forward-mode
gradient, against central differences of GPU renders under common random
numbers, and through torch.autograd."""
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


def _diag(sc):
    v = sc.verts.reshape(-1, 3)
    return float(np.linalg.norm(v.max(0) - v.min(0)))


def _gpu_grad(torch, sc, Np, K, r0, seed, g):
    s = api.Sppm(sc, api.sppm_params(Np, r0=r0, seed=seed, record_iterations=K))
    s.iterate(K)
    img = s.resolve()
    grad = s.adjoint(torch.from_numpy(g).cuda(), sc.albedo_params)
    torch.cuda.synchronize()
    out = grad.cpu().numpy(), img.cpu().numpy().ravel()
    s.destroy()
    return out


def _check_close(gpu, ref, rel=1e-4):
    scale = np.abs(ref).max()
    err = np.abs(gpu - ref)
    assert np.all(err <= rel * np.abs(ref) + 1e-9 * scale), (gpu, ref)


@pytest.mark.parametrize("case", ["box", "specular"])
def test_adjoint_matches_oracle_forward_mode(torch_cuda, oracle_lib, case):
    _log(f"case: adjoint vs oracle, {case}")
    if case == "box":
        sc, Np, K, seed = scenes.box_scene(32, 32), 1 << 13, 3, 1
        r0 = 0.05 * math.sqrt(3.0)
    else:
        sc = scenes.procedural_scene(width=80, height=45, hf_cells=16, sphere_level=2, glass_level=3, seed=3)
        Np, K, seed = 1 << 14, 3, 3
        r0 = 0.05 * _diag(sc) * 64 / 80
    P = sc.camera.width * sc.camera.height
    g = np.random.default_rng(7).standard_normal(P).astype(np.float32)
    grad, img = _gpu_grad(torch_cuda, sc, Np, K, r0, seed, g)
    ref, ref_img = oracle_lib.sppm_grad(oracle_lib.OracleScene(sc), seed, Np, K, g.astype(np.float64),
                                        sc.albedo_params, r0=r0)
    assert np.array_equal(img, ref_img)
    _check_close(grad, ref)
    assert np.count_nonzero(grad) == len(grad)


def test_adjoint_matches_central_differences(torch_cuda):
    _log("case: adjoint vs GPU central differences")
    sc = scenes.box_scene(32, 32)
    Np, K, seed, r0 = 1 << 13, 2, 5, 0.05 * math.sqrt(3.0)
    P = 32 * 32
    g = np.random.default_rng(3).standard_normal(P).astype(np.float32)
    grad, _ = _gpu_grad(torch_cuda, sc, Np, K, r0, seed, g)

    def radiance(scene):
        s = api.Sppm(scene, api.sppm_params(Np, r0=r0, seed=seed))
        s.iterate(K)
        v = s.views()
        L = (v["tau"] / (math.pi * v["R2"] * K) + v["D"] / K).cpu().numpy()
        s.destroy()
        return L

    h = 1e-3
    for i, m in enumerate(sc.albedo_params):
        rp, rm = sc.mat_rho.copy(), sc.mat_rho.copy()
        rp[m] += h
        rm[m] -= h
        fd = (g * (radiance(sc.with_rho(rp)) - radiance(sc.with_rho(rm)))).sum() / (float(rp[m]) - float(rm[m]))
        assert abs(fd - grad[i]) <= 2e-4 * abs(grad[i]) + 1e-6, (m, fd, grad[i])
    sp, sm = sc.with_Le(1 + h), sc.with_Le(1 - h)
    fd = (g * (radiance(sp) - radiance(sm))).sum() / (float(sp.mat_Le.max()) - float(sm.mat_Le.max()))
    assert abs(fd - grad[-1]) <= 2e-4 * abs(grad[-1])


def test_autograd_function(torch_cuda):
    _log("case: autograd image loss")
    torch = torch_cuda
    sc = scenes.box_scene(24, 24)
    Np, K, r0 = 1 << 12, 2, 0.08
    params = api.sppm_params(Np, r0=r0, seed=2)
    pm = sc.albedo_params
    rho = torch.tensor(sc.mat_rho[pm], dtype=torch.float64, requires_grad=True)
    Le = torch.tensor(10.0, dtype=torch.float64, requires_grad=True)
    rng = np.random.default_rng(4)
    target_sc = sc.with_rho(sc.mat_rho + np.where(np.isin(np.arange(len(sc.mat_rho)), pm),
                                                  rng.uniform(-0.1, 0.1, len(sc.mat_rho)), 0).astype(np.float32))
    target = api.render(target_sc, params, K)
    img = api.sppm_render_diff(rho, Le, sc, pm, params, K)
    loss = ((img.double() - target.double()) ** 2).mean()
    loss.backward()
    g = (2.0 * (img.double() - target.double()) / img.numel()).float()
    s = api.Sppm(sc, api.sppm_params(Np, r0=r0, seed=2, record_iterations=K))
    s.iterate(K)
    direct = s.adjoint(g, pm).cpu().numpy()
    s.destroy()
    # the adjoint's sums are integer sums: autograd and the direct call agree bit for bit
    assert np.array_equal(rho.grad.cpu().numpy(), direct[:-1])
    assert Le.grad.item() == direct[-1]
    assert np.all(np.isfinite(direct)) and np.abs(direct).max() > 0
    # Le as a plain number is a constant: backward still runs, and only the albedos get gradients
    rho2 = torch.tensor(sc.mat_rho[pm], dtype=torch.float64, requires_grad=True)
    img2 = api.sppm_render_diff(rho2, 10.0, sc, pm, params, K)
    ((img2.double() - target.double()) ** 2).mean().backward()
    assert np.array_equal(rho2.grad.cpu().numpy(), direct[:-1])
    # and with only Le requiring a gradient, the albedos get none
    rho3 = torch.tensor(sc.mat_rho[pm], dtype=torch.float64)
    Le3 = torch.tensor(10.0, dtype=torch.float64, requires_grad=True)
    img3 = api.sppm_render_diff(rho3, Le3, sc, pm, params, K)
    ((img3.double() - target.double()) ** 2).mean().backward()
    assert rho3.grad is None and Le3.grad.item() == direct[-1]


def test_adjoint_requires_recording(torch_cuda):
    _log("case: adjoint error paths")
    sc = scenes.box_scene(8, 8)
    s = api.Sppm(sc, api.sppm_params(256, r0=0.1))
    g = torch_cuda.ones(64, device="cuda")
    with pytest.raises(api.PMError) as e:
        s.adjoint(g, sc.albedo_params)
    assert e.value.code == api.PM_ERR_STATE
    s.iterate(1)
    with pytest.raises(api.PMError) as e:
        s.adjoint(g, sc.albedo_params)
    assert e.value.code == api.PM_ERR_STATE
    s.destroy()
    s = api.Sppm(sc, api.sppm_params(256, r0=0.1, record_iterations=1))
    s.iterate(1)
    light = int(np.nonzero(sc.mat_Le)[0][0])
    with pytest.raises(api.PMError) as e:
        s.adjoint(g, [light])           # black emitter: rho = 0 is not a parameter
    assert e.value.code == api.PM_ERR_ARG
    s.destroy()


def test_adjoint_is_bit_reproducible(torch_cuda):
    """Every sum of the adjoint is an integer sum of individually rounded
    terms, so repeated calls, and calls on a second handle, give the same bits
    whatever the order of the atomics and of the photons in their buckets."""
    _log("case: adjoint reproducibility")
    torch = torch_cuda
    sc = scenes.procedural_scene(width=97, height=61, hf_cells=20, sphere_level=2, glass_level=3, seed=3)
    P = sc.camera.width * sc.camera.height
    g = torch.from_numpy(np.random.default_rng(9).standard_normal(P).astype(np.float32)).cuda()
    out = []
    for _ in range(2):
        s = api.Sppm(sc, api.sppm_params(1 << 14, r0=0.02, seed=4, record_iterations=3))
        s.iterate(3)
        out.append(s.adjoint(g, sc.albedo_params).cpu().numpy())
        out.append(s.adjoint(g, sc.albedo_params).cpu().numpy())
        s.destroy()
    for o in out[1:]:
        assert np.array_equal(o, out[0])
    # the floor under the heightfield is neither seen nor reached: its gradient is exactly 0
    assert np.count_nonzero(out[0]) >= len(out[0]) - 2


@pytest.mark.parametrize("K", [1, 2, 5])
def test_overlapped_adjoint_equals_serial(torch_cuda, K):
    """The adjoint overlaps the replayed photon pass of iteration k + 1 with
    the grid, gather and path sums of k (two stores, tables and maxima by
    iteration parity).  A handle that times its stages (PM_PROFILE_TIME) has
    one store and runs the adjoint serially: the gradients are the same bits,
    for one, two (each parity once) and an odd number of iterations, also
    on a second call of the overlapped schedule."""
    _log(f"case: overlapped vs serial adjoint, K={K}")
    torch = torch_cuda
    sc = scenes.procedural_scene(width=97, height=61, hf_cells=20, sphere_level=2, glass_level=3, seed=3)
    P = sc.camera.width * sc.camera.height
    g = torch.from_numpy(np.random.default_rng(10).standard_normal(P).astype(np.float32)).cuda()
    grads = []
    for profile in (0, api.PROFILE_TIME):
        s = api.Sppm(sc, api.sppm_params(1 << 14, r0=0.02, seed=5, record_iterations=K, profile=profile))
        s.iterate(K)
        grads.append(s.adjoint(g, sc.albedo_params).cpu().numpy())
        if profile == 0:
            grads.append(s.adjoint(g, sc.albedo_params).cpu().numpy())
        s.destroy()
    assert np.count_nonzero(grads[0]) > 3
    for o in grads[1:]:
        assert np.array_equal(o, grads[0])


def _many_materials(sc, n_mat=256):
    """The box scene with its materials moved to the top of a 256-entry table:
    the light to 0, the seven diffuse materials to 249..255 (so materials 254
    and 255 carry photons), and unused diffuse fillers in between."""
    import dataclasses
    old = len(sc.mat_type)
    light = int(np.nonzero(sc.mat_Le > 0)[0][0])
    diffuse = [m for m in range(old) if m != light]
    new_id = np.zeros(old, np.int64)
    new_id[light] = 0
    new_id[diffuse] = np.arange(n_mat - len(diffuse), n_mat)
    def table(a, fill):
        t = np.full(n_mat, fill, a.dtype)
        t[new_id] = a
        return t
    return dataclasses.replace(sc, tri_mat=new_id[sc.tri_mat].astype(np.uint32),
                               mat_type=table(sc.mat_type, 0), mat_rho=table(sc.mat_rho, np.float32(0.5)),
                               mat_q=table(sc.mat_q, np.float32(0.5)), mat_Le=table(sc.mat_Le, np.float32(0)),
                               mat_ior=table(sc.mat_ior, np.float32(1)),
                               albedo_params=new_id[diffuse].astype(np.int32))


def test_adjoint_with_256_materials_matches_oracle(torch_cuda, oracle_lib):
    """Material ids up to 255 are ordinary entries of the adjoint's per-path
    material table (its markers lie outside the material range)."""
    _log("case: adjoint, 256 materials")
    sc = _many_materials(scenes.box_scene(32, 32))
    assert {254, 255} <= set(sc.albedo_params.tolist())
    Np, K, seed, r0 = 1 << 13, 3, 1, 0.05 * math.sqrt(3.0)
    g = np.random.default_rng(7).standard_normal(32 * 32).astype(np.float32)
    grad, img = _gpu_grad(torch_cuda, sc, Np, K, r0, seed, g)
    ref, ref_img = oracle_lib.sppm_grad(oracle_lib.OracleScene(sc), seed, Np, K, g.astype(np.float64),
                                        sc.albedo_params, r0=r0)
    assert np.array_equal(img, ref_img)
    _check_close(grad, ref)
    assert np.count_nonzero(grad) == len(grad)


def _perturbed_target(torch, sc, params, K, bvh, seed=11):
    """Target image rendered at albedos perturbed by U[-0.1, 0.1] (same seed, same K)."""
    rng = np.random.default_rng(seed)
    rho = sc.mat_rho.copy()
    pm = sc.albedo_params
    rho[pm] = np.clip(rho[pm] + rng.uniform(-0.1, 0.1, len(pm)).astype(np.float32), 0.01, 0.99)
    return api.render(sc.with_rho(rho), params, K, bvh=bvh)


def test_adjoint_procedural_320x180_against_oracle_and_central_differences(torch_cuda, oracle_lib):
    """The adjoint workload's check size: the 250k-triangle procedural scene at
    320x180 with 2^16 photons and K = 4; 16 albedos and Le; L2 loss against a
    target rendered at albedos perturbed by U[-0.1, 0.1]; gradient through the
    torch.autograd.Function.  It equals the direct adjoint call bit for bit,
    the oracle's forward-mode gradient to 1e-4, and central differences
    (h = 1e-3, common random numbers) of float64 GPU radiance to 2e-4."""
    _log("case: adjoint, procedural 250k triangles, 320x180, 2^16 photons, K = 4")
    torch = torch_cuda
    sc = scenes.procedural_scene(width=320, height=180)
    Np, K, seed = 1 << 16, 4, 3
    r0 = 0.05 * _diag(sc) * 64 / 320
    params = api.sppm_params(Np, r0=r0, seed=seed)
    bvh = api.build_bvh(sc.verts, sc.tri_mat)
    pm = sc.albedo_params
    assert len(pm) == 16
    target = _perturbed_target(torch, sc, params, K, bvh).double()
    light = int(np.nonzero(sc.mat_Le > 0)[0][0])
    rho = torch.tensor(sc.mat_rho[pm].astype(np.float64), requires_grad=True)
    Le = torch.tensor(float(sc.mat_Le[light]), dtype=torch.float64, requires_grad=True)
    img = api.sppm_render_diff(rho, Le, sc, pm, params, K)
    loss = ((img.double() - target) ** 2).mean()
    loss.backward()
    grad = np.concatenate([rho.grad.cpu().numpy(), [Le.grad.item()]])
    img = img.detach()
    g = (2.0 * (img.double() - target) / img.numel()).float()
    _log("  direct adjoint call")
    s = api.Sppm(sc, api.sppm_params(Np, r0=r0, seed=seed, record_iterations=K), bvh=bvh)
    s.iterate(K)
    direct = s.adjoint(g, pm).cpu().numpy()
    s.destroy()
    assert np.array_equal(grad, direct)
    _log("  oracle forward-mode gradient")
    ref, ref_img = oracle_lib.sppm_grad(oracle_lib.OracleScene(sc), seed, Np, K,
                                        g.cpu().numpy().ravel().astype(np.float64), pm, r0=r0)
    assert np.array_equal(img.cpu().numpy().ravel(), ref_img)
    _check_close(grad, ref)
    _log("  central differences")
    T = target.cpu().numpy().ravel()

    def loss64(scene):
        s = api.Sppm(scene, params, bvh=bvh)
        s.iterate(K)
        v = s.views()
        L = (v["tau"] / (math.pi * v["R2"] * K) + v["D"] / K).cpu().numpy()
        s.destroy()
        return ((L - T) ** 2).mean()

    h = 1e-3
    top = np.abs(grad).max()
    for i, m in enumerate(pm):
        rp, rm = sc.mat_rho.copy(), sc.mat_rho.copy()
        rp[m] += h
        rm[m] -= h
        fd = (loss64(sc.with_rho(rp)) - loss64(sc.with_rho(rm))) / (float(rp[m]) - float(rm[m]))
        assert abs(fd - grad[i]) <= 2e-4 * abs(grad[i]) + 1e-6 * top, (m, fd, grad[i])
    sp, sm = sc.with_Le(1 + h), sc.with_Le(1 - h)
    fd = (loss64(sp) - loss64(sm)) / (float(sp.mat_Le[light]) - float(sm.mat_Le[light]))
    assert abs(fd - grad[-1]) <= 2e-4 * abs(grad[-1]) + 1e-6 * top
    bvh.destroy()
