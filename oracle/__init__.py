"""CPU oracle for the photon-mapping hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding)
never imports it, and it imports nothing from the product path: it receives
the same seeded input arrays (from ``paper_1505_06022_amd.scenes``, which
holds no renderer arithmetic) and computes everything itself in plain C
(``pm_oracle.c``), loaded here with ctypes.

Every function here is pinned by a ``-m "not gpu"`` test against something
other than itself.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pm_oracle.c")
_LIB = os.path.join(_HERE, "libpm_oracle.so")

EYE = 1
PHOTON = 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, IEEE semantics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-pthread", "-Wall", "-Wno-unused-function",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


def default_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


class SceneDesc(C.Structure):
    _fields_ = [
        ("verts", C.c_void_p), ("tri_mat", C.c_void_p), ("n_tri", C.c_int64),
        ("mat_type", C.c_void_p), ("mat_rho", C.c_void_p), ("mat_q", C.c_void_p),
        ("mat_Le", C.c_void_p), ("mat_ior", C.c_void_p), ("n_mat", C.c_int32),
        ("cam_pos", C.c_float * 3), ("cam_look", C.c_float * 3), ("cam_up", C.c_float * 3),
        ("tan_half_fov", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
    ]


class RunOpts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("max_eye_depth", C.c_int32),
                ("max_photon_bounces", C.c_int32), ("nthreads", C.c_int32)]


class HitPoints(C.Structure):
    _fields_ = [("valid", C.c_void_p), ("x", C.c_void_p), ("n", C.c_void_p), ("wk", C.c_void_p),
                ("W", C.c_void_p), ("mat", C.c_void_p), ("tri", C.c_void_p), ("d_add", C.c_void_p)]


class Photons(C.Structure):
    _fields_ = [("x", C.c_void_p), ("w", C.c_void_p), ("phi", C.c_void_p), ("path", C.c_void_p),
                ("bounce", C.c_void_p), ("mats", C.c_void_p), ("cap", C.c_int64)]


class SppmParams(C.Structure):
    _fields_ = [("n_photons", C.c_int64), ("alpha", C.c_double), ("r0", C.c_double),
                ("shift", C.c_int32), ("gather_method", C.c_int32), ("photon_cap", C.c_int64)]


class State(C.Structure):
    _fields_ = [("N", C.c_void_p), ("R2", C.c_void_p), ("tau", C.c_void_p), ("D", C.c_void_p),
                ("R2_hist", C.c_void_p), ("M_hist", C.c_void_p), ("n_stored", C.c_void_p)]


def _declare(L):
    P = C.c_void_p
    L.orc_rng_seed.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, P]
    L.orc_splitmix64.argtypes = [C.c_uint64, C.c_int64, P]
    L.orc_xor128.argtypes = [P, C.c_int64, P]
    L.orc_photon_emit.argtypes = [P, C.c_uint64, C.c_uint32, C.c_int64, P, P, P]
    L.orc_rng_step_component.argtypes = [C.c_int, P, P, C.c_int64]
    L.orc_rng_draw.argtypes = [P, P, C.c_int64]
    L.orc_rng_streams.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_int64, C.c_int64, P]
    L.orc_scene_create.argtypes = [C.POINTER(SceneDesc), C.c_int]
    L.orc_scene_create.restype = P
    L.orc_scene_destroy.argtypes = [P]
    L.orc_scene_eps.argtypes = [P]
    L.orc_scene_eps.restype = C.c_float
    L.orc_scene_power.argtypes = [P]
    L.orc_scene_power.restype = C.c_double
    L.orc_trace.argtypes = [P, P, C.c_int64, P, P, C.c_int, C.c_int]
    L.orc_eye_pass.argtypes = [P, C.POINTER(RunOpts), C.c_uint32, C.POINTER(HitPoints)]
    L.orc_eye_pixels.argtypes = [P, C.POINTER(RunOpts), C.c_uint32, P, C.c_int64, C.POINTER(HitPoints)]
    L.orc_photon_flux.argtypes = [P, C.c_int64]
    L.orc_photon_flux.restype = C.c_float
    L.orc_photon_pass.argtypes = [P, C.POINTER(RunOpts), C.c_uint32, C.c_int64, P, C.c_int64, C.POINTER(Photons)]
    L.orc_photon_pass.restype = C.c_int64
    L.orc_gather.argtypes = [C.POINTER(HitPoints), C.c_int64, C.POINTER(Photons), C.c_int64, P, C.c_int, C.c_int,
                             C.c_int, P, P, P]
    L.orc_gather_stochastic.argtypes = [C.POINTER(HitPoints), C.c_int64, C.POINTER(Photons), C.c_int64, P, C.c_int,
                                        P, C.c_int64, C.c_uint64, C.c_uint32, P, P, P]
    L.orc_update.argtypes = [C.c_int64, P, P, P, C.c_double, C.c_int, P, P, P]
    L.orc_resolve.argtypes = [C.c_int64, P, P, P, C.c_int32, P]
    L.orc_sppm_run.argtypes = [P, C.POINTER(RunOpts), C.POINTER(SppmParams), C.c_int32, C.c_int32, C.POINTER(State)]
    L.orc_sppm_run.restype = C.c_int
    L.orc_sppm_grad.argtypes = [P, C.POINTER(RunOpts), C.POINTER(SppmParams), C.c_int32, P, P, C.c_int32, P, P]
    L.orc_sppm_grad.restype = C.c_int
    L.orc_fresnel.argtypes = [C.c_float, C.c_float]
    L.orc_fresnel.restype = C.c_float
    L.orc_onb.argtypes = [P, P, P]
    L.orc_cosine_dirs.argtypes = [P, C.c_uint64, C.c_int64, P]
    L.orc_glass_dirs.argtypes = [P, P, C.c_float, C.c_uint64, C.c_int64, P]


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# --------------------------------------------------------------------------
# RNG
# --------------------------------------------------------------------------
def rng_seed(seed: int, kind: int, k: int, index: int) -> np.ndarray:
    s = np.zeros(4, np.uint32)
    lib().orc_rng_seed(seed, kind, k, index, _p(s))
    return s


def splitmix64(state: int, n: int) -> np.ndarray:
    """n successive splitmix64 outputs starting from ``state``."""
    out = np.zeros(n, np.uint64)
    lib().orc_splitmix64(state, n, _p(out))
    return out


def xor128(seed_words, n: int) -> np.ndarray:
    """n successive outputs of Marsaglia's xor128 from four seed words."""
    sw = np.ascontiguousarray(seed_words, np.uint32)
    out = np.zeros(n, np.uint32)
    lib().orc_xor128(_p(sw), n, _p(out))
    return out


def rng_step_component(j: int, states: np.ndarray) -> np.ndarray:
    states = np.ascontiguousarray(states, np.uint32)
    out = np.empty_like(states)
    lib().orc_rng_step_component(j, _p(states), _p(out), states.size)
    return out


def rng_draw(state: np.ndarray, n: int) -> np.ndarray:
    """Draw n numbers starting from ``state`` (a copy is advanced)."""
    s = np.ascontiguousarray(state, np.uint32).copy()
    out = np.empty(n, np.float32)
    lib().orc_rng_draw(_p(s), _p(out), n)
    return out


def rng_streams(seed: int, kind: int, k: int, index0: int, n_streams: int, n_draws: int) -> np.ndarray:
    out = np.empty((n_streams, n_draws), np.float32)
    lib().orc_rng_streams(seed, kind, k, index0, n_streams, n_draws, _p(out))
    return out


# --------------------------------------------------------------------------
# Scenes and closest hits
# --------------------------------------------------------------------------
class OracleScene:
    """Oracle-side scene; keeps references to the numpy arrays it points to."""

    def __init__(self, scene, use_bvh: bool | None = None):
        self._keep = [np.ascontiguousarray(scene.verts, np.float32),
                      np.ascontiguousarray(scene.tri_mat, np.uint32),
                      np.ascontiguousarray(scene.mat_type, np.int32),
                      np.ascontiguousarray(scene.mat_rho, np.float32),
                      np.ascontiguousarray(scene.mat_q, np.float32),
                      np.ascontiguousarray(scene.mat_Le, np.float32),
                      np.ascontiguousarray(scene.mat_ior, np.float32)]
        v, tm, mt, rho, q, Le, ior = self._keep
        d = SceneDesc()
        d.verts, d.tri_mat, d.n_tri = _p(v).value, _p(tm).value, v.shape[0]
        d.mat_type, d.mat_rho, d.mat_q = _p(mt).value, _p(rho).value, _p(q).value
        d.mat_Le, d.mat_ior, d.n_mat = _p(Le).value, _p(ior).value, len(mt)
        cam = scene.camera
        d.cam_pos[:] = cam.pos
        d.cam_look[:] = cam.look
        d.cam_up[:] = cam.up
        d.tan_half_fov = cam.tan_half_fov
        d.width, d.height = cam.width, cam.height
        self.desc = d
        if use_bvh is None:
            use_bvh = v.shape[0] > 256
        self.h = lib().orc_scene_create(C.byref(d), int(use_bvh))
        self.scene = scene
        self.P = cam.width * cam.height

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_scene_destroy(self.h)
            self.h = None

    @property
    def eps(self) -> float:
        return lib().orc_scene_eps(self.h)

    @property
    def power(self) -> float:
        return lib().orc_scene_power(self.h)

    def trace(self, rays: np.ndarray, brute_force: bool = False, nthreads: int | None = None):
        rays = np.ascontiguousarray(rays, np.float32)
        n = rays.shape[0]
        hit = np.empty(n, np.int32)
        t = np.empty(n, np.float32)
        lib().orc_trace(self.h, _p(rays), n, _p(hit), _p(t), int(brute_force), nthreads or default_threads())
        return hit, t

    def photon_flux(self, n_photons: int) -> float:
        return lib().orc_photon_flux(self.h, n_photons)


def trace_brute_force(verts: np.ndarray, rays: np.ndarray, nthreads: int | None = None):
    """Closest hit of every ray over every triangle (the plain definition)."""
    from types import SimpleNamespace
    from paper_1505_06022_amd.scenes import Camera
    sc = SimpleNamespace(verts=verts, tri_mat=np.zeros(len(verts), np.uint32),
                         mat_type=np.zeros(1, np.int32), mat_rho=np.zeros(1, np.float32),
                         mat_q=np.zeros(1, np.float32), mat_Le=np.zeros(1, np.float32),
                         mat_ior=np.ones(1, np.float32),
                         camera=Camera((0, 0, 0), (0, 0, 1), (0, 1, 0), 0.5, 1, 1))
    return OracleScene(sc, use_bvh=False).trace(rays, brute_force=True, nthreads=nthreads)


# --------------------------------------------------------------------------
# SPPM
# --------------------------------------------------------------------------
def run_opts(seed: int, nthreads: int | None = None, max_eye_depth=16, max_photon_bounces=32) -> RunOpts:
    o = RunOpts()
    o.seed, o.max_eye_depth, o.max_photon_bounces = seed, max_eye_depth, max_photon_bounces
    o.nthreads = nthreads or default_threads()
    return o


class HitPointBuf:
    def __init__(self, P: int):
        self.valid = np.zeros(P, np.uint8)
        self.x = np.zeros((P, 3), np.float32)
        self.n = np.zeros((P, 3), np.float32)
        self.wk = np.zeros(P, np.float32)
        self.W = np.zeros(P, np.float32)
        self.mat = np.full(P, -1, np.int32)
        self.tri = np.full(P, -1, np.int32)
        self.d_add = np.zeros(P, np.float64)
        self.c = HitPoints(*[_p(a).value for a in (self.valid, self.x, self.n, self.wk, self.W,
                                                     self.mat, self.tri, self.d_add)])


class PhotonBuf:
    def __init__(self, cap: int, with_mats: bool = False):
        self.x = np.zeros((cap, 3), np.float32)
        self.w = np.zeros((cap, 3), np.float32)
        self.phi = np.zeros(cap, np.float32)
        self.path = np.zeros(cap, np.uint32)
        self.bounce = np.zeros(cap, np.uint32)
        self.mats = np.full((cap, 32), -1, np.int32) if with_mats else None
        self.c = Photons(_p(self.x).value, _p(self.w).value, _p(self.phi).value, _p(self.path).value,
                         _p(self.bounce).value, _p(self.mats).value if with_mats else None, cap)
        self.n = 0

    def view(self):
        n = self.n
        return dict(x=self.x[:n], w=self.w[:n], phi=self.phi[:n], path=self.path[:n], bounce=self.bounce[:n])


def eye_pass(os_: OracleScene, seed: int, k: int, nthreads=None) -> HitPointBuf:
    hp = HitPointBuf(os_.P)
    lib().orc_eye_pass(os_.h, C.byref(run_opts(seed, nthreads)), k, C.byref(hp.c))
    return hp


def eye_pixels(os_: OracleScene, seed: int, k: int, pixels: np.ndarray) -> HitPointBuf:
    hp = HitPointBuf(os_.P)
    pix = np.ascontiguousarray(pixels, np.int64)
    lib().orc_eye_pixels(os_.h, C.byref(run_opts(seed, 1)), k, _p(pix), len(pix), C.byref(hp.c))
    return hp


def photon_pass(os_: OracleScene, seed: int, k: int, n_photons: int, paths: np.ndarray | None = None,
                cap: int | None = None, with_mats: bool = False, nthreads=None) -> PhotonBuf:
    n_paths = n_photons if paths is None else len(paths)
    cap = cap or max(64, n_paths * 8)
    pb = PhotonBuf(cap, with_mats)
    ids = None if paths is None else np.ascontiguousarray(paths, np.uint64)
    n = lib().orc_photon_pass(os_.h, C.byref(run_opts(seed, nthreads)), k, n_photons,
                              None if ids is None else _p(ids), n_paths, C.byref(pb.c))
    if n < 0:
        raise OverflowError("oracle photon store capacity exceeded")
    pb.n = int(n)
    return pb


def photon_emit(os_: OracleScene, seed: int, k: int, n: int):
    """Emission of photon paths [0, n) of iteration k: (origin, direction, emitting triangle)."""
    org = np.zeros((n, 3), np.float32)
    dirs = np.zeros((n, 3), np.float32)
    tri = np.zeros(n, np.int32)
    lib().orc_photon_emit(os_.h, seed, k, n, _p(org), _p(dirs), _p(tri))
    return org, dirs, tri


def gather(hp: HitPointBuf, ph: PhotonBuf, R2: np.ndarray, shift=40, method=1, nthreads=None, want_double=False):
    P = len(hp.valid)
    R2 = np.ascontiguousarray(R2, np.float64)
    M = np.zeros(P, np.uint32)
    Phi = np.zeros(P, np.uint64)
    phid = np.zeros(P, np.float64) if want_double else None
    lib().orc_gather(C.byref(hp.c), P, C.byref(ph.c), ph.n, _p(R2), shift, method,
                     nthreads or default_threads(), _p(M), _p(Phi), None if phid is None else _p(phid))
    return (M, Phi, phid) if want_double else (M, Phi)


def scene_lo(scene) -> np.ndarray:
    """Per-axis minimum over the scene's vertices (origin of the hashing grid)."""
    return np.ascontiguousarray(np.asarray(scene.verts, np.float32).reshape(-1, 3).min(0), np.float32)


def gather_stochastic(hp: HitPointBuf, ph: PhotonBuf, R2: np.ndarray, lo, n_photons: int, seed: int, k: int,
                      shift=40, want_counts=False):
    """Stochastic spatial hashing estimate of (M, Phi) for every hit point (Sec. 3.4)."""
    P = len(hp.valid)
    R2 = np.ascontiguousarray(R2, np.float64)
    lo = np.ascontiguousarray(lo, np.float32)
    M = np.zeros(P, np.uint32)
    Phi = np.zeros(P, np.uint64)
    bits = 12
    while bits < 24 and (1 << bits) < 4 * n_photons:
        bits += 1
    counts = np.zeros(1 << bits, np.uint32) if want_counts else None
    lib().orc_gather_stochastic(C.byref(hp.c), P, C.byref(ph.c), ph.n, _p(R2), shift, _p(lo), n_photons, seed, k,
                                _p(M), _p(Phi), None if counts is None else _p(counts))
    return (M, Phi, counts) if want_counts else (M, Phi)


def update(valid, M, Phi, alpha, N, R2, tau, shift=40):
    """In-place progressive update of (N, R2, tau) (float64 arrays)."""
    valid = np.ascontiguousarray(valid, np.uint8)
    M = np.ascontiguousarray(M, np.uint32)
    Phi = np.ascontiguousarray(Phi, np.uint64)
    for a in (N, R2, tau):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_update(len(valid), _p(valid), _p(M), _p(Phi), alpha, shift, _p(N), _p(R2), _p(tau))


def resolve(R2, tau, D, K) -> np.ndarray:
    n = len(R2)
    img = np.zeros(n, np.float32)
    R2, tau, D = (np.ascontiguousarray(a, np.float64) for a in (R2, tau, D))
    lib().orc_resolve(n, _p(R2), _p(tau), _p(D), K, _p(img))
    return img


class SppmResult:
    pass


def sppm_run(os_: OracleScene, seed: int, n_photons: int, K: int, alpha=0.7, r0=None, shift=40,
             gather_method=1, nthreads=None, history=False, k0=0, state=None, photon_cap=None):
    """K SPPM iterations from scratch (or from ``state``); returns state + image."""
    P = os_.P
    pp = SppmParams()
    pp.n_photons, pp.alpha, pp.shift, pp.gather_method = n_photons, alpha, shift, gather_method
    pp.r0 = float(r0)
    pp.photon_cap = photon_cap or n_photons * 8
    r = SppmResult()
    if state is None:
        r.N = np.zeros(P)
        r.R2 = np.full(P, float(r0) * float(r0))
        r.tau = np.zeros(P)
        r.D = np.zeros(P)
    else:
        r.N, r.R2, r.tau, r.D = (np.array(state[k], np.float64) for k in ("N", "R2", "tau", "D"))
    r.R2_hist = np.zeros((K, P)) if history else None
    r.M_hist = np.zeros((K, P), np.uint32) if history else None
    r.n_stored = np.zeros(K, np.int64)
    st = State(_p(r.N).value, _p(r.R2).value, _p(r.tau).value, _p(r.D).value,
               _p(r.R2_hist).value if history else None, _p(r.M_hist).value if history else None,
               _p(r.n_stored).value)
    rc = lib().orc_sppm_run(os_.h, C.byref(run_opts(seed, nthreads)), C.byref(pp), k0, K, C.byref(st))
    if rc != 0:
        raise OverflowError("oracle photon store capacity exceeded")
    r.K = k0 + K
    r.image = resolve(r.R2, r.tau, r.D, r.K)
    return r


def sppm_grad(os_: OracleScene, seed: int, n_photons: int, K: int, g: np.ndarray, param_mats,
              alpha=0.7, r0=None, shift=40, gather_method=1, nthreads=None, photon_cap=None):
    """Forward-mode gradient of sum_p g_p L_p w.r.t. the listed albedos and the emitter's Le.

    Returns (grad[n_par + 1], image)."""
    pp = SppmParams()
    pp.n_photons, pp.alpha, pp.shift, pp.gather_method = n_photons, alpha, shift, gather_method
    pp.r0 = float(r0)
    pp.photon_cap = photon_cap or n_photons * 8
    g = np.ascontiguousarray(g, np.float64)
    pm = np.ascontiguousarray(param_mats, np.int32)
    grad = np.zeros(len(pm) + 1, np.float64)
    img = np.zeros(os_.P, np.float32)
    rc = lib().orc_sppm_grad(os_.h, C.byref(run_opts(seed, nthreads)), C.byref(pp), K, _p(g), _p(pm), len(pm),
                             _p(grad), _p(img))
    if rc != 0:
        raise OverflowError("oracle photon store capacity exceeded")
    return grad, img


def fresnel(ci: float, eta: float) -> float:
    return lib().orc_fresnel(ci, eta)


def onb(n):
    n = np.ascontiguousarray(n, np.float32)
    b1 = np.zeros(3, np.float32)
    b2 = np.zeros(3, np.float32)
    lib().orc_onb(_p(n), _p(b1), _p(b2))
    return b1, b2


def cosine_dirs(n, seed: int, count: int) -> np.ndarray:
    n = np.ascontiguousarray(n, np.float32)
    out = np.zeros((count, 3), np.float32)
    lib().orc_cosine_dirs(_p(n), seed, count, _p(out))
    return out


def glass_dirs(d, n, ior: float, seed: int, count: int) -> np.ndarray:
    d = np.ascontiguousarray(d, np.float32)
    n = np.ascontiguousarray(n, np.float32)
    out = np.zeros((count, 3), np.float32)
    lib().orc_glass_dirs(_p(d), _p(n), ior, seed, count, _p(out))
    return out
