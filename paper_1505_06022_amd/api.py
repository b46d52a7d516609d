"""Python binding of libpm.so (ctypes).  Argument marshalling only.

Every function here forwards to the C ABI declared in include/pm.h under the
same name without the ``pm_`` prefix.  Device buffers are PyTorch tensors on
the current HIP device; the stream is PyTorch's current stream unless one is
given.  There is no CPU fallback: if the library is missing or fails to load,
the import error is raised.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpm.so")

PM_OK, PM_ERR_ARG, PM_ERR_HIP, PM_ERR_OVERFLOW, PM_ERR_STATE, PM_ERR_NOMEM = 0, -1, -2, -3, -4, -5

EXPORTS = ["pm_abi_version", "pm_last_error", "pm_build_bvh", "pm_build_bvh_host", "pm_bvh_destroy",
           "pm_bvh_get_info", "pm_bvh_download", "pm_trace_rays", "pm_trace_rays_ex", "pm_sppm_create", "pm_sppm_destroy",
           "pm_sppm_iterate", "pm_sppm_resolve", "pm_sppm_status", "pm_render", "pm_sppm_get_views",
           "pm_sppm_adjoint", "pm_sppm_save", "pm_sppm_load", "pm_batch_create", "pm_batch_destroy", "pm_batch_iterate", "pm_batch_resolve",
           "pm_batch_status", "pm_batch_get_info", "pm_batch_get_views", "pm_render_batch", "pm_probe_chase",
           "pm_trace_rays_multi", "pm_trace_rays_noalloc", "pm_probe_stream", "pm_sppm_get_stats"]


class PMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pm error {code}: {msg}")
        self.code = code


class BvhOpts(C.Structure):
    _fields_ = [("size", C.c_uint32), ("bins", C.c_int32), ("max_leaf", C.c_int32), ("n_threads", C.c_int32),
                ("trav_cost", C.c_float), ("builder", C.c_int32), ("split_alpha", C.c_float)]


BUILD_HOST_SAH, BUILD_GPU_LBVH = 0, 1


class BvhInfo(C.Structure):
    _fields_ = [("size", C.c_uint32), ("n_tri", C.c_int64), ("n_refs", C.c_int64), ("n_nodes", C.c_int64),
                ("n_leaves", C.c_int64),
                ("depth", C.c_int32), ("max_leaf", C.c_int32), ("sah_cost", C.c_double),
                ("device_bytes", C.c_int64), ("build_ms", C.c_double),
                ("grid_lo", C.c_float * 3), ("grid_step", C.c_float * 3)]


class TraceOpts(C.Structure):
    _fields_ = [("size", C.c_uint32), ("link_set", C.c_int32), ("counters", C.c_void_p), ("kernel", C.c_int32),
                ("refill", C.c_int32), ("reorder", C.c_int32), ("block", C.c_int32), ("tile_width", C.c_int32),
                ("slice", C.c_int32)]


(TRACE_AUTO, TRACE_PER_RAY, TRACE_PERSISTENT, TRACE_PAIRED, TRACE_POSTPONED, TRACE_TWO_RAYS, TRACE_PACKET,
 TRACE_SLICES) = range(8)
MAX_TRACE_BATCHES = 8


class TraceBatch(C.Structure):
    _fields_ = [("size", C.c_uint32), ("rays", C.c_void_p), ("n", C.c_int64), ("hit", C.c_void_p), ("t", C.c_void_p),
                ("opts", C.c_void_p)]


class SceneDesc(C.Structure):
    _fields_ = [("size", C.c_uint32), ("tri_verts", C.c_void_p), ("tri_mat", C.c_void_p), ("n_tri", C.c_int64),
                ("mat_type", C.c_void_p), ("mat_rho", C.c_void_p), ("mat_q", C.c_void_p),
                ("mat_Le", C.c_void_p), ("mat_ior", C.c_void_p), ("n_mat", C.c_int32),
                ("cam_pos", C.c_float * 3), ("cam_look", C.c_float * 3), ("cam_up", C.c_float * 3),
                ("tan_half_fov", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
                ("bvh", C.c_void_p)]


class SppmParams(C.Structure):
    _fields_ = [("size", C.c_uint32), ("n_photons", C.c_int64), ("alpha", C.c_double), ("r0", C.c_double),
                ("seed", C.c_uint64), ("max_eye_depth", C.c_int32), ("max_photon_bounces", C.c_int32),
                ("fixed_shift", C.c_int32), ("store_factor", C.c_int32), ("record_iterations", C.c_int32),
                ("photon_kernel", C.c_int32), ("refill", C.c_int32), ("single_link_set", C.c_int32),
                ("gather_mode", C.c_int32), ("pass_threads", C.c_int32), ("passes", C.c_int32),
                ("profile", C.c_int32)]


PROFILE_COUNT, PROFILE_TIME = 1, 2


class SppmStats(C.Structure):
    _fields_ = [("size", C.c_uint32), ("counted_iterations", C.c_int64)] + \
               [(n, C.c_uint64) for n in ("eye_paths", "eye_rays", "eye_box_tests", "eye_tri_tests", "photon_paths",
                                          "photon_rays", "photon_box_tests", "photon_tri_tests", "photons_stored", "gather_hit_points",
                                          "gather_buckets", "gather_examined", "gather_accepted")] + \
               [("timed_iterations", C.c_int64)] + \
               [(n, C.c_double) for n in ("ms_eye", "ms_photon", "ms_grid", "ms_gather", "ms_update", "ms_iteration")]


PHOTON_AUTO, PHOTON_PER_PATH, PHOTON_REGEN, PHOTON_PASSES, PHOTON_RAY_REGEN, PHOTON_POOL, PHOTON_TWO_PHASE = range(7)
GATHER_EXACT, GATHER_STOCHASTIC = 0, 1


class SppmViews(C.Structure):
    _fields_ = [("size", C.c_uint32), ("n_pixels", C.c_int64), ("iterations", C.c_int32),
                ("photon_capacity", C.c_int64), ("table_size", C.c_int64),
                ("N", C.c_void_p), ("R2", C.c_void_p), ("tau", C.c_void_p), ("D", C.c_void_p),
                ("hp_pos", C.c_void_p), ("hp_nrm", C.c_void_p), ("photons", C.c_void_p),
                ("photon_count", C.c_void_p), ("gather_M", C.c_void_p), ("gather_Phi", C.c_void_p)]


class BatchOpts(C.Structure):
    _fields_ = [("size", C.c_uint32), ("chunk", C.c_int32), ("block", C.c_int32), ("autotune", C.c_int32),
                ("use_graph", C.c_int32)]


class BatchInfo(C.Structure):
    _fields_ = [("size", C.c_uint32), ("n_scenes", C.c_int32), ("iterations", C.c_int32), ("chunk", C.c_int32),
                ("block", C.c_int32), ("uses_graph", C.c_int32), ("tuned_from_cache", C.c_int32),
                ("n_candidates", C.c_int32), ("cand_chunk", C.c_int32 * 8), ("cand_block", C.c_int32 * 8),
                ("cand_ms", C.c_double * 8)]


_lib = None


def lib() -> C.CDLL:
    """Load libpm.so (raises if it is absent: build it with paper_1505_06022_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_1505_06022_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, I64, I32 = C.c_void_p, C.c_int64, C.c_int32
        L.pm_abi_version.restype = C.c_int
        L.pm_last_error.restype = C.c_char_p
        L.pm_build_bvh.argtypes = [P, P, I64, P, P, P]
        L.pm_build_bvh_host.argtypes = [P, P, I64, P, P, P, P, P]
        L.pm_bvh_destroy.argtypes = [P]
        L.pm_bvh_get_info.argtypes = [P, P]
        L.pm_bvh_download.argtypes = [P, P, P, P]
        L.pm_trace_rays.argtypes = [P, P, I64, P, P, P]
        L.pm_trace_rays_ex.argtypes = [P, P, I64, P, P, P, P]
        L.pm_trace_rays_noalloc.argtypes = [P, P, I64, P, P, P, P]
        L.pm_sppm_create.argtypes = [P, P, P, P]
        L.pm_sppm_destroy.argtypes = [P]
        L.pm_sppm_iterate.argtypes = [P, I32, P]
        L.pm_sppm_resolve.argtypes = [P, P, P]
        L.pm_sppm_status.argtypes = [P, P]
        L.pm_render.argtypes = [P, P, I32, P, P]
        L.pm_sppm_get_views.argtypes = [P, P]
        L.pm_sppm_adjoint.argtypes = [P, P, P, I32, P, P]
        L.pm_sppm_save.argtypes = [P, P, P, P]
        L.pm_sppm_load.argtypes = [P, P, C.c_uint64, P]
        L.pm_batch_create.argtypes = [P, P, I32, P, P, P]
        L.pm_batch_destroy.argtypes = [P]
        L.pm_batch_iterate.argtypes = [P, I32, P]
        L.pm_batch_resolve.argtypes = [P, P, P]
        L.pm_batch_status.argtypes = [P, P]
        L.pm_batch_get_info.argtypes = [P, P]
        L.pm_batch_get_views.argtypes = [P, I32, P]
        L.pm_render_batch.argtypes = [P, P, I32, I32, P, P, P]
        L.pm_probe_chase.argtypes = [P, I32, I64, I32, P, P]
        L.pm_probe_stream.argtypes = [P, P, C.c_uint64, I32, P, P]
        L.pm_sppm_get_stats.argtypes = [P, P, I32, P]
        L.pm_trace_rays_multi.argtypes = [P, I32, P, P]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != PM_OK:
        raise PMError(rc, lib().pm_last_error().decode())


def _ptr(a) -> int:
    return a.ctypes.data if isinstance(a, np.ndarray) else a.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _opts(bins, max_leaf, n_threads, trav_cost=0.0, builder=0, split_alpha=0.0):
    o = BvhOpts()
    o.size, o.bins, o.max_leaf, o.n_threads = C.sizeof(BvhOpts), bins, max_leaf, n_threads
    o.trav_cost, o.builder, o.split_alpha = trav_cost, builder, split_alpha
    return o


def _info_dict(inf) -> dict:
    d = {}
    for k, _ in BvhInfo._fields_:
        if k == "size":
            continue
        v = getattr(inf, k)
        d[k] = list(v) if k.startswith("grid_") else v
    return d


def abi_version() -> int:
    return lib().pm_abi_version()


# ---------------------------------------------------------------------------
# BVH
# ---------------------------------------------------------------------------
class Bvh:
    """Device multiple-threaded BVH owned by the library."""

    def __init__(self, handle: int, n_tri: int):
        self.h = C.c_void_p(handle)
        self.n_tri = n_tri

    def info(self) -> dict:
        inf = BvhInfo()
        inf.size = C.sizeof(BvhInfo)
        _check(lib().pm_bvh_get_info(self.h, C.byref(inf)))
        return _info_dict(inf)

    def download(self, stream=None):
        """(nodes uint32 [6, n_nodes, 4], tris uint32 [n_refs, 12]) copied from the device."""
        inf = self.info()
        nodes = np.zeros((6, inf["n_nodes"], 4), np.uint32)
        tris = np.zeros((inf["n_refs"], 12), np.uint32)
        _check(lib().pm_bvh_download(self.h, _ptr(nodes), _ptr(tris), _stream(stream)))
        return nodes, tris

    def destroy(self):
        if self.h:
            _check(lib().pm_bvh_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def build_bvh(verts: np.ndarray, tri_mat: np.ndarray | None = None, bins=32, max_leaf=4, n_threads=0,
              trav_cost=0.0, builder=0, split_alpha=0.0, stream=None) -> Bvh:
    """Build a device BVH: builder 0 = SAH on the host (spatial splits with split_alpha > 0),
    1 = linear BVH on the GPU."""
    v = np.ascontiguousarray(verts, np.float32)
    m = None if tri_mat is None else np.ascontiguousarray(tri_mat, np.uint32)
    out = C.c_void_p()
    o = _opts(bins, max_leaf, n_threads, trav_cost, builder, split_alpha)
    _check(lib().pm_build_bvh(_ptr(v), None if m is None else _ptr(m), v.shape[0], C.byref(o), _stream(stream),
                              C.byref(out)))
    return Bvh(out.value, v.shape[0])


def build_bvh_host(verts: np.ndarray, tri_mat: np.ndarray | None = None, bins=32, max_leaf=4, n_threads=0,
                   trav_cost=0.0, split_alpha=0.0):
    """Host-only build: returns (nodes uint32 [6, n_nodes, 4], tris uint32 [n_refs, 12], info dict)."""
    v = np.ascontiguousarray(verts, np.float32)
    m = None if tri_mat is None else np.ascontiguousarray(tri_mat, np.uint32)
    o = _opts(bins, max_leaf, n_threads, trav_cost, 0, split_alpha)
    nn = C.c_int64()
    L = lib()
    inf = BvhInfo()
    inf.size = C.sizeof(BvhInfo)
    _check(L.pm_build_bvh_host(_ptr(v), None if m is None else _ptr(m), v.shape[0], C.byref(o), C.byref(nn),
                               None, None, C.byref(inf)))
    nodes = np.zeros((6, nn.value, 4), np.uint32)
    tris = np.zeros((inf.n_refs, 12), np.uint32)
    _check(L.pm_build_bvh_host(_ptr(v), None if m is None else _ptr(m), v.shape[0], C.byref(o), C.byref(nn),
                               _ptr(nodes), _ptr(tris), C.byref(inf)))
    return nodes, tris, _info_dict(inf)


def trace_rays(bvh: Bvh, rays, hit=None, t=None, link_set: int = -1, counters=None, kernel: int = 0, refill: int = 0,
               reorder: int = 0, block: int = 0, tile_width: int = 0, slice_rays: int = 0, stream=None):
    """Closest hit of each ray.  rays: float32 cuda tensor [n, 8]; returns (hit int32 [n], t float32 [n]).
    The options are pm_trace_opts' fields (slice_rays is its field slice)."""
    import torch
    assert rays.is_cuda and rays.dtype == torch.float32 and rays.is_contiguous() and rays.shape[-1] == 8
    n = rays.shape[0]
    if hit is None:
        hit = torch.empty(n, dtype=torch.int32, device=rays.device)
    if t is None:
        t = torch.empty(n, dtype=torch.float32, device=rays.device)
    if link_set == -1 and counters is None and kernel == 0 and refill == 0 and not reorder and not block \
            and not tile_width and not slice_rays:
        _check(lib().pm_trace_rays(bvh.h, _ptr(rays), n, _ptr(hit), _ptr(t), _stream(stream)))
    else:
        o = _trace_opts(link_set, counters, kernel, refill, reorder, block, tile_width, slice_rays)
        _check(lib().pm_trace_rays_ex(bvh.h, _ptr(rays), n, _ptr(hit), _ptr(t), C.byref(o), _stream(stream)))
    return hit, t


NOALLOC_MAX_RAYS = 1 << 22


def trace_rays_noalloc(bvh: Bvh, rays, hit, t, link_set: int = -1, counters=None, kernel: int = 0, refill: int = 0,
                       reorder: int = 1, block: int = 0, slice_rays: int = 0, stream=None):
    """The bucketed trace on the library's static scratch (pm_trace_rays_noalloc):
    the caller passes the outputs hit (int32 cuda [n]) and t (float32 cuda [n])."""
    import torch
    assert rays.is_cuda and rays.dtype == torch.float32 and rays.is_contiguous() and rays.shape[-1] == 8
    n = rays.shape[0]
    assert hit.dtype == torch.int32 and t.dtype == torch.float32 and hit.numel() >= n and t.numel() >= n
    o = _trace_opts(link_set, counters, kernel, refill, reorder, block, 0, slice_rays)
    _check(lib().pm_trace_rays_noalloc(bvh.h, _ptr(rays), n, _ptr(hit), _ptr(t), C.byref(o), _stream(stream)))
    return hit, t


def _trace_opts(link_set=-1, counters=None, kernel=0, refill=0, reorder=0, block=0, tile_width=0,
                slice_rays=0) -> TraceOpts:
    o = TraceOpts()
    o.size, o.link_set, o.kernel, o.refill = C.sizeof(TraceOpts), link_set, kernel, refill
    o.reorder, o.block, o.tile_width, o.slice = int(reorder), int(block), int(tile_width), int(slice_rays)
    o.counters = None if counters is None else counters.data_ptr()
    return o


def trace_rays_multi(bvh: Bvh, batches, stream=None):
    """Several ray batches traced concurrently (pm_trace_rays_multi).  batches:
    list of dicts with "rays" (float32 cuda [n, 8]), optional "hit" / "t"
    outputs, and any pm_trace_opts field as in trace_rays.  Returns [(hit, t)]."""
    import torch
    keep, out = [], []
    arr = (TraceBatch * len(batches))()
    for k, bt in enumerate(batches):
        bt = dict(bt)
        rays = bt.pop("rays")
        assert rays.is_cuda and rays.dtype == torch.float32 and rays.is_contiguous() and rays.shape[-1] == 8
        n = rays.shape[0]
        hit = bt.pop("hit", None)
        t = bt.pop("t", None)
        hit = torch.empty(n, dtype=torch.int32, device=rays.device) if hit is None else hit
        t = torch.empty(n, dtype=torch.float32, device=rays.device) if t is None else t
        o = _trace_opts(**bt)
        keep.append(o)
        arr[k].size, arr[k].rays, arr[k].n = C.sizeof(TraceBatch), _ptr(rays), n
        arr[k].hit, arr[k].t, arr[k].opts = _ptr(hit), _ptr(t), C.cast(C.pointer(o), C.c_void_p)
        out.append((hit, t))
    _check(lib().pm_trace_rays_multi(bvh.h, len(batches), arr, _stream(stream)))
    return out


def probe_stream(src, dst=None, out=None, stream=None):
    """Streaming copy of src into dst (dst given) or read of src with the XOR of
    its words into out (a cuda int32 tensor of one element), pm_probe_stream."""
    n = src.numel() * src.element_size()
    if dst is not None:
        assert dst.numel() * dst.element_size() >= n
        _check(lib().pm_probe_stream(_ptr(src), _ptr(dst), n, 0, None, _stream(stream)))
    else:
        _check(lib().pm_probe_stream(_ptr(src), None, n, 1, _ptr(out), _stream(stream)))


def probe_chase(rows, steps: int, n_lanes: int, out=None, stream=None):
    """Dependent random 16-byte reads (memory microbenchmark).  rows: int32 or
    uint32-valued cuda tensor of 2^k x 4 words; returns out (int32 [n_lanes]),
    each lane's XOR of the words it read."""
    import torch
    assert rows.is_cuda and rows.is_contiguous() and rows.dtype == torch.int32 and rows.dim() == 2 \
        and rows.shape[1] == 4
    nr = rows.shape[0]
    assert nr > 1 and nr & (nr - 1) == 0, "the row count must be a power of two"
    if out is None:
        out = torch.empty(n_lanes, dtype=torch.int32, device=rows.device)
    _check(lib().pm_probe_chase(_ptr(rows), nr.bit_length() - 1, n_lanes, steps, _ptr(out), _stream(stream)))
    return out


# ---------------------------------------------------------------------------
# SPPM
# ---------------------------------------------------------------------------
def sppm_params(n_photons: int, alpha=0.7, r0=0.05, seed=1, max_eye_depth=16, max_photon_bounces=32,
                fixed_shift=40, store_factor=8, record_iterations=0, photon_kernel=0, refill=0,
                single_link_set=0, gather_mode=0, pass_threads=0, passes=0, profile=0) -> SppmParams:
    p = SppmParams()
    p.size = C.sizeof(SppmParams)
    p.n_photons, p.alpha, p.r0, p.seed = n_photons, alpha, float(r0), seed
    p.max_eye_depth, p.max_photon_bounces = max_eye_depth, max_photon_bounces
    p.fixed_shift, p.store_factor = fixed_shift, store_factor
    p.record_iterations = record_iterations
    p.photon_kernel, p.refill = photon_kernel, refill
    p.single_link_set = single_link_set
    p.gather_mode = gather_mode
    p.pass_threads, p.passes = pass_threads, passes
    p.profile = profile
    return p


class _SceneArgs:
    """Scene description plus the host arrays it points into (kept alive)."""

    def __init__(self, scene, bvh: Bvh | None = None):
        self.keep = [np.ascontiguousarray(scene.verts, np.float32), np.ascontiguousarray(scene.tri_mat, np.uint32),
                     np.ascontiguousarray(scene.mat_type, np.int32), np.ascontiguousarray(scene.mat_rho, np.float32),
                     np.ascontiguousarray(scene.mat_q, np.float32), np.ascontiguousarray(scene.mat_Le, np.float32),
                     np.ascontiguousarray(scene.mat_ior, np.float32)]
        v, tm, mt, rho, q, Le, ior = self.keep
        d = SceneDesc()
        d.size = C.sizeof(SceneDesc)
        d.tri_verts, d.tri_mat, d.n_tri = _ptr(v), _ptr(tm), v.shape[0]
        d.mat_type, d.mat_rho, d.mat_q, d.mat_Le, d.mat_ior = _ptr(mt), _ptr(rho), _ptr(q), _ptr(Le), _ptr(ior)
        d.n_mat = len(mt)
        cam = scene.camera
        d.cam_pos[:] = cam.pos
        d.cam_look[:] = cam.look
        d.cam_up[:] = cam.up
        d.tan_half_fov = cam.tan_half_fov
        d.width, d.height = cam.width, cam.height
        d.bvh = bvh.h.value if bvh is not None else None
        self.desc = d
        self.bvh = bvh


def _device_view(ptr: int, shape, dtype):
    """Zero-copy tensor over a library-owned device buffer."""
    import torch
    typestr = {torch.float32: "<f4", torch.float64: "<f8", torch.int32: "<i4", torch.uint32: "<u4",
               torch.int64: "<i8", torch.uint64: "<u8"}[dtype]

    class _Iface:
        __cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (ptr, False), "version": 2,
                                    "strides": None}
    return torch.as_tensor(_Iface(), device="cuda")


def _views_dict(v) -> dict:
    import torch
    P, cap = v.n_pixels, v.photon_capacity
    return dict(
        iterations=v.iterations, table_size=v.table_size,
        N=_device_view(v.N, (P,), torch.float64), R2=_device_view(v.R2, (P,), torch.float64),
        tau=_device_view(v.tau, (P,), torch.float64), D=_device_view(v.D, (P,), torch.float64),
        hp_pos=_device_view(v.hp_pos, (P, 4), torch.float32),
        hp_nrm=_device_view(v.hp_nrm, (P, 4), torch.float32),
        photons=_device_view(v.photons, (cap, 8), torch.float32),
        photon_count=_device_view(v.photon_count, (4,), torch.int32),
        M=_device_view(v.gather_M, (P,), torch.int32),
        Phi=_device_view(v.gather_Phi, (P,), torch.int64),
    )


class Sppm:
    """One progressive photon mapping renderer (library-owned device state)."""

    def __init__(self, scene, params: SppmParams, bvh: Bvh | None = None, stream=None):
        self.args = _SceneArgs(scene, bvh)
        self.params = params
        self.width, self.height = scene.camera.width, scene.camera.height
        out = C.c_void_p()
        _check(lib().pm_sppm_create(C.byref(self.args.desc), C.byref(params), _stream(stream), C.byref(out)))
        self.h = out

    def iterate(self, n: int = 1, stream=None):
        _check(lib().pm_sppm_iterate(self.h, n, _stream(stream)))

    def resolve(self, image=None, stream=None):
        import torch
        if image is None:
            image = torch.empty((self.height, self.width), dtype=torch.float32, device="cuda")
        _check(lib().pm_sppm_resolve(self.h, _ptr(image), _stream(stream)))
        return image

    def status(self, stream=None):
        _check(lib().pm_sppm_status(self.h, _stream(stream)))

    def views(self) -> dict:
        """Tensors aliasing the handle's device buffers (valid until destroy)."""
        v = SppmViews()
        v.size = C.sizeof(SppmViews)
        _check(lib().pm_sppm_get_views(self.h, C.byref(v)))
        return _views_dict(v)

    def save(self, stream=None) -> bytes:
        """Checkpoint of the per-pixel state, iteration count and recorded radii."""
        n = C.c_uint64(0)
        _check(lib().pm_sppm_save(self.h, None, C.byref(n), _stream(stream)))
        buf = C.create_string_buffer(n.value)
        _check(lib().pm_sppm_save(self.h, buf, C.byref(n), _stream(stream)))
        return buf.raw[:n.value]

    def load(self, checkpoint: bytes, stream=None):
        """Continue from a checkpoint taken from a handle with the same scene and parameters."""
        buf = C.create_string_buffer(bytes(checkpoint), len(checkpoint))
        _check(lib().pm_sppm_load(self.h, buf, len(checkpoint), _stream(stream)))

    def stats(self, reset: bool = False, stream=None) -> dict:
        """Profiling counts and stage times (pm_sppm_get_stats)."""
        st = SppmStats()
        st.size = C.sizeof(SppmStats)
        _check(lib().pm_sppm_get_stats(self.h, C.byref(st), int(reset), _stream(stream)))
        return {n: getattr(st, n) for n, _ in SppmStats._fields_ if n != "size"}

    def adjoint(self, dloss_dimage, param_mats, grad=None, stream=None):
        """dLoss/drho for each material in param_mats, then dLoss/dLe (float64 cuda tensor)."""
        import torch
        g = dloss_dimage.to(torch.float32).contiguous()
        assert g.is_cuda and g.numel() == self.width * self.height
        pm = np.ascontiguousarray(param_mats, np.int32)
        if grad is None:
            grad = torch.empty(len(pm) + 1, dtype=torch.float64, device=g.device)
        _check(lib().pm_sppm_adjoint(self.h, _ptr(g), _ptr(pm) if len(pm) else None, len(pm), _ptr(grad),
                                     _stream(stream)))
        return grad

    def destroy(self):
        if self.h:
            _check(lib().pm_sppm_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def sppm_create(scene, params: SppmParams, bvh: Bvh | None = None, stream=None) -> Sppm:
    return Sppm(scene, params, bvh, stream)


def render(scene, params: SppmParams, K: int, image=None, bvh: Bvh | None = None, stream=None):
    """create -> K iterations -> resolve -> destroy, in one call."""
    import torch
    if image is None:
        image = torch.empty((scene.camera.height, scene.camera.width), dtype=torch.float32, device="cuda")
    args = _SceneArgs(scene, bvh)
    _check(lib().pm_render(C.byref(args.desc), C.byref(params), K, _ptr(image), _stream(stream)))
    return image


def _render_function():
    import torch

    class SPPMRender(torch.autograd.Function):
        """Differentiable SPPM render: image(albedos, Le).

        forward: K iterations with the given albedos of ``param_mats`` and the
        emitting material's Le (Russian roulette keeps the scene's nominal q);
        backward: pm_sppm_adjoint replays the K iterations.
        """

        @staticmethod
        def forward(ctx, albedos, Le, scene, param_mats, params, K, stream=None, bvh=None):
            sc = scene.with_rho(scene.mat_rho.copy())
            rho = sc.mat_rho
            rho[np.asarray(param_mats, np.int64)] = albedos.detach().cpu().numpy().astype(np.float32)
            em = np.nonzero(scene.mat_Le > 0)[0]
            if len(em) != 1:
                raise ValueError("Le is a parameter only for scenes with exactly one emitting material")
            sc.mat_Le = scene.mat_Le.copy()
            sc.mat_Le[em[0]] = np.float32(float(Le))
            p = SppmParams.from_buffer_copy(params)
            p.record_iterations = max(int(params.record_iterations), int(K))
            s = Sppm(sc, p, bvh=bvh, stream=stream)
            s.iterate(K, stream=stream)
            img = s.resolve(stream=stream)
            ctx.s, ctx.param_mats, ctx.stream = s, np.asarray(param_mats, np.int32), stream
            ctx.le_is_tensor = isinstance(Le, torch.Tensor)
            ctx.dtypes = (albedos.dtype, Le.dtype if ctx.le_is_tensor else torch.float32)
            ctx.devices = (albedos.device, Le.device if ctx.le_is_tensor else albedos.device)
            return img

        @staticmethod
        def backward(ctx, g):
            need_rho, need_le = ctx.needs_input_grad[0], ctx.needs_input_grad[1] and ctx.le_is_tensor
            if not (need_rho or need_le):
                return None, None, None, None, None, None, None, None
            grad = ctx.s.adjoint(g, ctx.param_mats, stream=ctx.stream)
            n = len(ctx.param_mats)
            g_rho = grad[:n].to(device=ctx.devices[0], dtype=ctx.dtypes[0]) if need_rho else None
            # a plain-number Le is a constant: its gradient position stays None
            g_le = grad[n].to(device=ctx.devices[1], dtype=ctx.dtypes[1]) if need_le else None
            return g_rho, g_le, None, None, None, None, None, None

    return SPPMRender


_SPPMRender = None


def sppm_render_diff(albedos, Le, scene, param_mats, params: SppmParams, K: int, stream=None, bvh: Bvh | None = None):
    """Differentiable render (torch.autograd): returns the [H, W] image.  bvh:
    optional BVH already built over the scene's triangles."""
    global _SPPMRender
    if _SPPMRender is None:
        _SPPMRender = _render_function()
    return _SPPMRender.apply(albedos, Le, scene, param_mats, params, K, stream, bvh)


# ---------------------------------------------------------------------------
# Batched rendering
# ---------------------------------------------------------------------------
def batch_opts(chunk=0, block=0, autotune=False, use_graph=True) -> BatchOpts:
    o = BatchOpts()
    o.size, o.chunk, o.block, o.autotune, o.use_graph = C.sizeof(BatchOpts), chunk, block, int(autotune), int(use_graph)
    return o


class Batch:
    """Many SPPM renderers advanced together, one persistent launch per stage."""

    def __init__(self, scenes, params, chunk=0, block=0, autotune=False, use_graph=True, stream=None):
        if isinstance(params, SppmParams):
            params = [params] * len(scenes)
        self.args = [_SceneArgs(sc) for sc in scenes]
        self.params = list(params)
        self.sizes = [(sc.camera.height, sc.camera.width) for sc in scenes]
        descs = (C.c_void_p * len(scenes))(*[C.addressof(a.desc) for a in self.args])
        prms = (C.c_void_p * len(scenes))(*[C.addressof(p) for p in self.params])
        self.opts = batch_opts(chunk, block, autotune, use_graph)
        out = C.c_void_p()
        _check(lib().pm_batch_create(descs, prms, len(scenes), C.byref(self.opts), _stream(stream), C.byref(out)))
        self.h = out

    def iterate(self, n: int = 1, stream=None):
        _check(lib().pm_batch_iterate(self.h, n, _stream(stream)))

    def resolve(self, images=None, stream=None):
        import torch
        if images is None:
            images = [torch.empty(hw, dtype=torch.float32, device="cuda") for hw in self.sizes]
        ptrs = (C.c_void_p * len(images))(*[im.data_ptr() for im in images])
        _check(lib().pm_batch_resolve(self.h, ptrs, _stream(stream)))
        return images

    def status(self, stream=None):
        _check(lib().pm_batch_status(self.h, _stream(stream)))

    def info(self) -> dict:
        inf = BatchInfo()
        inf.size = C.sizeof(BatchInfo)
        _check(lib().pm_batch_get_info(self.h, C.byref(inf)))
        n = inf.n_candidates
        return dict(n_scenes=inf.n_scenes, iterations=inf.iterations, chunk=inf.chunk, block=inf.block,
                    uses_graph=bool(inf.uses_graph), tuned_from_cache=bool(inf.tuned_from_cache),
                    candidates=[(inf.cand_chunk[i], inf.cand_block[i], inf.cand_ms[i]) for i in range(n)])

    def views(self, scene: int) -> dict:
        v = SppmViews()
        v.size = C.sizeof(SppmViews)
        _check(lib().pm_batch_get_views(self.h, scene, C.byref(v)))
        return _views_dict(v)

    def destroy(self):
        if self.h:
            _check(lib().pm_batch_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def render_batch(scenes, params, K: int, images=None, chunk=0, block=0, autotune=False, use_graph=True, stream=None):
    """create -> K iterations of every scene -> resolve -> destroy."""
    import torch
    if isinstance(params, SppmParams):
        params = [params] * len(scenes)
    args = [_SceneArgs(sc) for sc in scenes]
    params = list(params)
    if images is None:
        images = [torch.empty((sc.camera.height, sc.camera.width), dtype=torch.float32, device="cuda")
                  for sc in scenes]
    descs = (C.c_void_p * len(scenes))(*[C.addressof(a.desc) for a in args])
    prms = (C.c_void_p * len(scenes))(*[C.addressof(p) for p in params])
    ptrs = (C.c_void_p * len(images))(*[im.data_ptr() for im in images])
    o = batch_opts(chunk, block, autotune, use_graph)
    _check(lib().pm_render_batch(descs, prms, len(scenes), K, ptrs, C.byref(o), _stream(stream)))
    return images
