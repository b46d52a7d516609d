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
    assert np.allclose(rho.grad.cpu().numpy(), direct[:-1], rtol=1e-12, atol=0)
    assert np.isclose(Le.grad.item(), direct[-1], rtol=1e-12)
    assert np.all(np.isfinite(direct)) and np.abs(direct).max() > 0


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
