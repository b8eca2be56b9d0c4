"""ctypes binding of libpcgpu.so (the C ABI declared in include/pcgpu.h).

Argument marshalling only: every step runs in the library's HIP kernels.
Tensors are torch CUDA (ROCm) tensors; PyTorch supplies device memory and
the current stream.  If the library is not built this module raises at
import time -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcgpu.so")

PC_OK, PC_EINVAL, PC_EWORKSPACE, PC_EDEVICE = 0, 1, 2, 3
PC_ICP_CONVERGED, PC_ICP_MAXITER, PC_ICP_DEGENERATE, PC_ICP_NO_INLIERS = 0, 1, 2, 3
KMAX = 32
MAX_CLOUDS = 65536          # PCGPU_MAX_CLOUDS: clouds (pairs) per batched call

# every symbol the header declares
EXPORTS = (
    "pc_status_string",
    "knn_search_workspace_size", "knn_search",
    "estimate_normals_workspace_size", "estimate_normals", "estimate_normals_radius",
    "icp_point_to_plane_workspace_size", "icp_point_to_plane", "icp_point_to_plane_noalloc",
    "icp_point_to_point", "icp_combined",
    "icp_point_to_plane_with_normals_workspace_size", "icp_point_to_plane_with_normals",
    "icp_projective_workspace_size", "icp_projective",
    "estimate_normals_batched_workspace_size", "estimate_normals_batched",
    "icp_point_to_plane_batched_workspace_size", "icp_point_to_plane_batched",
    "icp_point_to_plane_with_normals_batched_workspace_size", "icp_point_to_plane_with_normals_batched",
    "pc_copy_probe", "icp_history", "pc_set_kernel_timer", "pc_kernel_timer_count",
    "pc_set_tuning", "pc_get_tuning",
    "pose_net_param_count", "pose_net_workspace_size", "pose_net_predict", "pose_net_train_step",
    "icp_learned_batched_workspace_size", "icp_learned_batched",
)
PC_INIT_LEARNED, PC_INIT_MULTI_START, PC_INIT_LEARNED_ONLY = 0, 1, 2


class Tuning(ctypes.Structure):
    """pc_tuning: accumulate block size, search leaf size, pyramid node
    budget, Morton-ordered ICP queries, and the reserved persistent-loop
    flag (must be 0)."""
    _fields_ = [("icp_block_threads", ctypes.c_int32), ("icp_leaf", ctypes.c_int32),
                ("node_budget", ctypes.c_float), ("sort_queries", ctypes.c_int32),
                ("icp_persistent", ctypes.c_int32)]


class PcgpuError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)}")


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1807_00399_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, f32, f64, sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_float,
                                  ctypes.c_double, ctypes.c_size_t)
    lib.pc_status_string.argtypes = [ctypes.c_int]
    lib.pc_status_string.restype = ctypes.c_char_p
    lib.knn_search_workspace_size.argtypes = [i64, i64, i32]
    lib.knn_search_workspace_size.restype = sz
    lib.knn_search.argtypes = [vp, i64, vp, i64, i32, vp, vp, vp, sz, vp]
    lib.knn_search.restype = ctypes.c_int
    lib.estimate_normals_workspace_size.argtypes = [i64, i32]
    lib.estimate_normals_workspace_size.restype = sz
    lib.estimate_normals.argtypes = [vp, i64, i32, ctypes.POINTER(ctypes.c_float), vp, vp, vp, sz, vp]
    lib.estimate_normals.restype = ctypes.c_int
    lib.estimate_normals_radius.argtypes = [vp, i64, f32, i32, ctypes.POINTER(ctypes.c_float), vp, vp, vp, sz, vp]
    lib.estimate_normals_radius.restype = ctypes.c_int
    lib.icp_point_to_plane_workspace_size.argtypes = [i64, i64, i32]
    lib.icp_point_to_plane_workspace_size.restype = sz
    lib.icp_point_to_plane.argtypes = [vp, i64, vp, vp, i64, vp, f32, i32, f64, vp, vp, vp, sz, vp]
    lib.icp_point_to_plane.restype = ctypes.c_int
    lib.icp_point_to_plane_noalloc.argtypes = [vp, i64, vp, vp, i64, vp, f32, i32, f64, vp, vp, vp]
    lib.icp_point_to_plane_noalloc.restype = ctypes.c_int
    lib.icp_point_to_plane_with_normals_workspace_size.argtypes = [i64, i64, i32]
    lib.icp_point_to_plane_with_normals_workspace_size.restype = sz
    lib.icp_point_to_plane_with_normals.argtypes = [vp, i64, vp, i64, i32, ctypes.POINTER(ctypes.c_float), vp, f32,
                                                    i32, f64, vp, vp, vp, vp, sz, vp]
    lib.icp_point_to_plane_with_normals.restype = ctypes.c_int
    lib.icp_point_to_point.argtypes = [vp, i64, vp, i64, vp, f32, i32, f64, vp, vp, vp, sz, vp]
    lib.icp_point_to_point.restype = ctypes.c_int
    lib.icp_combined.argtypes = [vp, i64, vp, vp, i64, vp, f32, f32, f32, i32, f64, vp, vp, vp, sz, vp]
    lib.icp_combined.restype = ctypes.c_int
    lib.icp_projective_workspace_size.argtypes = [i64, i32]
    lib.icp_projective_workspace_size.restype = sz
    lib.icp_projective.argtypes = [vp, i64, vp, vp, i32, i32, ctypes.POINTER(ctypes.c_float), vp, f32, i32, f64,
                                   vp, vp, vp, sz, vp]
    lib.icp_projective.restype = ctypes.c_int
    lib.estimate_normals_batched_workspace_size.argtypes = [i32, vp]
    lib.estimate_normals_batched_workspace_size.restype = sz
    lib.estimate_normals_batched.argtypes = [i32, vp, vp, vp, ctypes.POINTER(ctypes.c_float), vp, vp, vp, sz, vp]
    lib.estimate_normals_batched.restype = ctypes.c_int
    lib.icp_point_to_plane_batched_workspace_size.argtypes = [i32, vp, vp, i32]
    lib.icp_point_to_plane_batched_workspace_size.restype = sz
    lib.icp_point_to_plane_batched.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp, f64, vp, vp, vp, sz, vp]
    lib.icp_point_to_plane_batched.restype = ctypes.c_int
    lib.icp_point_to_plane_with_normals_batched_workspace_size.argtypes = [i32, vp, vp, i32]
    lib.icp_point_to_plane_with_normals_batched_workspace_size.restype = sz
    lib.icp_point_to_plane_with_normals_batched.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, f64, vp, vp, vp,
                                                            vp, sz, vp]
    lib.icp_point_to_plane_with_normals_batched.restype = ctypes.c_int
    lib.pc_copy_probe.argtypes = [vp, vp, sz, vp]
    lib.pc_copy_probe.restype = ctypes.c_int
    lib.icp_history.argtypes = [vp, sz, i64, i64, i32]
    lib.icp_history.restype = ctypes.c_void_p
    lib.pc_set_kernel_timer.argtypes = [vp, vp, i32]
    lib.pc_set_kernel_timer.restype = ctypes.c_int
    lib.pc_kernel_timer_count.argtypes = []
    lib.pc_kernel_timer_count.restype = ctypes.c_int
    lib.pc_set_tuning.argtypes = [ctypes.POINTER(Tuning)]
    lib.pc_set_tuning.restype = ctypes.c_int
    lib.pc_get_tuning.argtypes = [ctypes.POINTER(Tuning)]
    lib.pc_get_tuning.restype = None
    lib.pose_net_param_count.argtypes = []
    lib.pose_net_param_count.restype = ctypes.c_int
    lib.pose_net_workspace_size.argtypes = [i32, vp, vp]
    lib.pose_net_workspace_size.restype = sz
    lib.pose_net_predict.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.pose_net_predict.restype = ctypes.c_int
    lib.pose_net_train_step.argtypes = [vp, vp, vp, i32, f32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.pose_net_train_step.restype = ctypes.c_int
    lib.icp_learned_batched_workspace_size.argtypes = [i32, vp, vp, i32]
    lib.icp_learned_batched_workspace_size.restype = sz
    lib.icp_learned_batched.argtypes = [i32, vp, i32, vp, vp, vp, vp, vp, f32, i32, f64, f32, vp, vp, vp, vp, sz, vp]
    lib.icp_learned_batched.restype = ctypes.c_int
    return lib


lib = _load()


def status_string(s: int) -> str:
    return lib.pc_status_string(int(s)).decode()


def _check(st: int, what: str):
    if st != PC_OK:
        raise PcgpuError(st, what)


def _stream(stream=None, scope=None) -> int:
    """The HIP stream handle to launch on.  Inputs, outputs and workspaces
    are allocated (and the initial pose copied) on torch's current stream;
    when another stream is given, it first waits for the current one, and
    every device tensor in `scope` (the caller's locals) is recorded as in
    use on it, so the caching allocator does not hand that memory out
    while the library's kernels may still use it."""
    cur = torch.cuda.current_stream()
    s = stream if stream is not None else cur
    if s != cur:
        s.wait_stream(cur)
        for v in (scope or {}).values():
            if isinstance(v, torch.Tensor) and v.is_cuda:
                v.record_stream(s)
    return int(s.cuda_stream)


def _pts(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or t.dim() != 2 or t.shape[1] != 3:
        raise ValueError(f"{name} must be a float32 (n, 3) tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    return t.contiguous()


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


class Workspace:
    """Grow-only device scratch buffer (one per device)."""

    def __init__(self):
        self._buf: dict[int, torch.Tensor] = {}

    def get(self, nbytes: int, device: torch.device) -> torch.Tensor:
        idx = device.index if device.index is not None else torch.cuda.current_device()
        b = self._buf.get(idx)
        if b is None or b.numel() < nbytes:
            b = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
            self._buf[idx] = b
        return b


_ws = Workspace()


def knn_search(ref: torch.Tensor, qry: torch.Tensor, k: int, return_d2: bool = True, stream=None,
               workspace: torch.Tensor | None = None):
    """Exact k-NN: (idx int32 (nq,k), d2 float32 (nq,k) or None)."""
    ref = _pts(ref, "ref")
    qry = ref if qry is ref else _pts(qry, "qry")
    nq = qry.shape[0]
    idx = torch.empty((nq, k), dtype=torch.int32, device=ref.device)
    d2 = torch.empty((nq, k), dtype=torch.float32, device=ref.device) if return_d2 else None
    need = lib.knn_search_workspace_size(ref.shape[0], nq, k)
    ws = workspace if workspace is not None else _ws.get(need, ref.device)
    st = lib.knn_search(ref.data_ptr(), ref.shape[0], qry.data_ptr(), nq, int(k), idx.data_ptr(), _ptr(d2),
                        ws.data_ptr(), ws.numel(), _stream(stream, locals()))
    _check(st, "knn_search")
    return idx, d2


def estimate_normals(xyz: torch.Tensor, k: int, viewpoint=(0.0, 0.0, 0.0), curvature: bool = True,
                     stream=None, workspace: torch.Tensor | None = None):
    """PCA normals (n,3) float32 and curvature (n,) float32 or None."""
    xyz = _pts(xyz, "xyz")
    n = xyz.shape[0]
    nrm = torch.empty((n, 3), dtype=torch.float32, device=xyz.device)
    cur = torch.empty((n,), dtype=torch.float32, device=xyz.device) if curvature else None
    vp = (ctypes.c_float * 3)(*[float(v) for v in viewpoint])
    need = lib.estimate_normals_workspace_size(n, k)
    ws = workspace if workspace is not None else _ws.get(need, xyz.device)
    st = lib.estimate_normals(xyz.data_ptr(), n, int(k), vp, nrm.data_ptr(), _ptr(cur), ws.data_ptr(),
                              ws.numel(), _stream(stream, locals()))
    _check(st, "estimate_normals")
    return nrm, cur


def estimate_normals_radius(xyz: torch.Tensor, radius: float, k: int = 0, viewpoint=(0.0, 0.0, 0.0),
                            curvature: bool = True, stream=None, workspace: torch.Tensor | None = None):
    """Normals from radius (k = 0) or hybrid (k nearest within the radius)
    neighbourhoods: (n,3) float32 and curvature (n,) or None."""
    xyz = _pts(xyz, "xyz")
    n = xyz.shape[0]
    nrm = torch.empty((n, 3), dtype=torch.float32, device=xyz.device)
    cur = torch.empty((n,), dtype=torch.float32, device=xyz.device) if curvature else None
    vp = (ctypes.c_float * 3)(*[float(v) for v in viewpoint])
    need = lib.estimate_normals_workspace_size(n, max(int(k), 1))
    ws = workspace if workspace is not None else _ws.get(need, xyz.device)
    st = lib.estimate_normals_radius(xyz.data_ptr(), n, float(radius), int(k), vp, nrm.data_ptr(), _ptr(cur),
                                     ws.data_ptr(), ws.numel(), _stream(stream, locals()))
    _check(st, "estimate_normals_radius")
    return nrm, cur


STATS_DTYPE = [("status", "<i4"), ("iterations_run", "<i4"), ("inliers", "<i8"), ("rms", "<f8")]


def icp_point_to_plane(src: torch.Tensor, tgt: torch.Tensor, tgt_normals: torch.Tensor, init_T=None,
                       max_corr_dist: float = 0.05, max_iters: int = 30, conv_tol: float = 0.0,
                       stream=None, workspace: torch.Tensor | None = None, out_T: torch.Tensor | None = None,
                       out_stats: torch.Tensor | None = None, read_stats: bool = True):
    """Point-to-plane ICP.  Returns (T (4,4) float64 device tensor, stats).

    stats is a dict read back from the device when read_stats is True
    (this synchronises the stream), else the raw 24-byte device tensor."""
    src = _pts(src, "src")
    tgt = _pts(tgt, "tgt")
    tgt_normals = _pts(tgt_normals, "tgt_normals")
    if tgt_normals.shape[0] != tgt.shape[0]:
        raise ValueError("tgt_normals must match tgt")
    dev = src.device
    T0 = None
    if init_T is not None:
        T0 = torch.as_tensor(init_T, dtype=torch.float64).reshape(4, 4).to(dev).contiguous()
    T = out_T if out_T is not None else torch.empty((4, 4), dtype=torch.float64, device=dev)
    stats = out_stats if out_stats is not None else torch.zeros(24, dtype=torch.uint8, device=dev)
    need = lib.icp_point_to_plane_workspace_size(src.shape[0], tgt.shape[0], int(max_iters))
    ws = workspace if workspace is not None else _ws.get(need, dev)
    st = lib.icp_point_to_plane(src.data_ptr(), src.shape[0], tgt.data_ptr(), tgt_normals.data_ptr(),
                                tgt.shape[0], _ptr(T0), float(max_corr_dist), int(max_iters), float(conv_tol),
                                T.data_ptr(), stats.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream, locals()))
    _check(st, "icp_point_to_plane")
    if not read_stats:
        return T, stats
    return T, decode_stats(stats)


NOALLOC_SCRATCH_BYTES = 64 << 20


def icp_point_to_plane_noalloc(src: torch.Tensor, tgt: torch.Tensor, tgt_normals: torch.Tensor, out_T: torch.Tensor,
                               out_stats: torch.Tensor, init_T: torch.Tensor | None = None,
                               max_corr_dist: float = 0.05, max_iters: int = 30, conv_tol: float = 0.0,
                               stream=None):
    """icp_point_to_plane on the library's static device scratch (no
    workspace): the caller passes every buffer, outputs included
    (out_T (4,4) float64, out_stats 24 uint8, init_T (4,4) float64 or
    None, all on the device), and nothing is allocated here."""
    for t, name in ((src, "src"), (tgt, "tgt"), (tgt_normals, "tgt_normals")):
        if not (t.is_cuda and t.dtype == torch.float32 and t.dim() == 2 and t.shape[1] == 3 and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float32 (n, 3) device tensor")
    if tgt_normals.shape[0] != tgt.shape[0]:
        raise ValueError("tgt_normals must match tgt")
    if not (out_T.dtype == torch.float64 and out_T.numel() == 16 and out_T.is_cuda):
        raise ValueError("out_T must be a (4, 4) float64 device tensor")
    if not (out_stats.dtype == torch.uint8 and out_stats.numel() >= 24 and out_stats.is_cuda):
        raise ValueError("out_stats must be a 24-byte uint8 device tensor")
    if init_T is not None and not (init_T.dtype == torch.float64 and init_T.numel() == 16 and init_T.is_cuda):
        raise ValueError("init_T must be a (4, 4) float64 device tensor")
    st = lib.icp_point_to_plane_noalloc(src.data_ptr(), src.shape[0], tgt.data_ptr(), tgt_normals.data_ptr(),
                                        tgt.shape[0], _ptr(init_T), float(max_corr_dist), int(max_iters),
                                        float(conv_tol), out_T.data_ptr(), out_stats.data_ptr(),
                                        _stream(stream, locals()))
    _check(st, "icp_point_to_plane_noalloc")


def icp_point_to_plane_with_normals(src: torch.Tensor, tgt: torch.Tensor, k: int, viewpoint=(0.0, 0.0, 0.0),
                                    init_T=None, max_corr_dist: float = 0.05, max_iters: int = 30,
                                    conv_tol: float = 0.0, return_normals: bool = False, stream=None,
                                    workspace: torch.Tensor | None = None, out_T: torch.Tensor | None = None,
                                    out_stats: torch.Tensor | None = None, read_stats: bool = True,
                                    out_normals: torch.Tensor | None = None):
    """Target normals (k, viewpoint) and point-to-plane ICP in one call over
    one target pyramid.  Returns (T, stats) or (T, stats, normals).  With
    preallocated workspace and outputs the call launches kernels only, so it
    can be captured in a graph."""
    src = _pts(src, "src")
    tgt = _pts(tgt, "tgt")
    dev = src.device
    T0 = None
    if init_T is not None:
        T0 = torch.as_tensor(init_T, dtype=torch.float64).reshape(4, 4).to(dev).contiguous()
    T = out_T if out_T is not None else torch.empty((4, 4), dtype=torch.float64, device=dev)
    stats = out_stats if out_stats is not None else torch.zeros(24, dtype=torch.uint8, device=dev)
    nrm = out_normals
    if nrm is None and return_normals:
        nrm = torch.empty((tgt.shape[0], 3), dtype=torch.float32, device=dev)
    vp = (ctypes.c_float * 3)(*[float(v) for v in viewpoint])
    need = lib.icp_point_to_plane_with_normals_workspace_size(src.shape[0], tgt.shape[0], int(max_iters))
    ws = workspace if workspace is not None else _ws.get(need, dev)
    st = lib.icp_point_to_plane_with_normals(src.data_ptr(), src.shape[0], tgt.data_ptr(), tgt.shape[0], int(k), vp,
                                             _ptr(T0), float(max_corr_dist), int(max_iters), float(conv_tol),
                                             T.data_ptr(), stats.data_ptr(), _ptr(nrm), ws.data_ptr(), ws.numel(),
                                             _stream(stream, locals()))
    _check(st, "icp_point_to_plane_with_normals")
    out = (T, stats if not read_stats else decode_stats(stats))
    return out + (nrm,) if (return_normals or out_normals is not None) else out


def _icp_variant(fn, what, src, tgt, tgt_normals, init_T, max_corr_dist, max_iters, conv_tol, stream, workspace,
                 weights=None):
    src = _pts(src, "src")
    tgt = _pts(tgt, "tgt")
    if tgt_normals is not None:
        tgt_normals = _pts(tgt_normals, "tgt_normals")
        if tgt_normals.shape[0] != tgt.shape[0]:
            raise ValueError("tgt_normals must match tgt")
    dev = src.device
    T0 = None
    if init_T is not None:
        T0 = torch.as_tensor(init_T, dtype=torch.float64).reshape(4, 4).to(dev).contiguous()
    T = torch.empty((4, 4), dtype=torch.float64, device=dev)
    stats = torch.zeros(24, dtype=torch.uint8, device=dev)
    need = lib.icp_point_to_plane_workspace_size(src.shape[0], tgt.shape[0], int(max_iters))
    ws = workspace if workspace is not None else _ws.get(need, dev)
    if weights is None:
        st = fn(src.data_ptr(), src.shape[0], tgt.data_ptr(), tgt.shape[0], _ptr(T0), float(max_corr_dist),
                int(max_iters), float(conv_tol), T.data_ptr(), stats.data_ptr(), ws.data_ptr(), ws.numel(),
                _stream(stream, locals()))
    else:
        st = fn(src.data_ptr(), src.shape[0], tgt.data_ptr(), _ptr(tgt_normals), tgt.shape[0], _ptr(T0),
                float(weights[0]), float(weights[1]), float(max_corr_dist), int(max_iters), float(conv_tol),
                T.data_ptr(), stats.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream, locals()))
    _check(st, what)
    return T, decode_stats(stats)


def icp_point_to_point(src: torch.Tensor, tgt: torch.Tensor, init_T=None, max_corr_dist: float = 0.05,
                       max_iters: int = 30, conv_tol: float = 0.0, stream=None,
                       workspace: torch.Tensor | None = None):
    """Point-to-point ICP (closed-form fit per iteration).  Returns (T, stats dict)."""
    return _icp_variant(lib.icp_point_to_point, "icp_point_to_point", src, tgt, None, init_T, max_corr_dist,
                        max_iters, conv_tol, stream, workspace)


def icp_combined(src: torch.Tensor, tgt: torch.Tensor, tgt_normals, init_T=None, w_point: float = 0.5,
                 w_plane: float = 1.0, max_corr_dist: float = 0.05, max_iters: int = 30, conv_tol: float = 0.0,
                 stream=None, workspace: torch.Tensor | None = None):
    """ICP with the weighted point-to-point + point-to-plane metric.  Returns (T, stats dict)."""
    return _icp_variant(lib.icp_combined, "icp_combined", src, tgt, tgt_normals, init_T, max_corr_dist, max_iters,
                        conv_tol, stream, workspace, weights=(w_point, w_plane))


def icp_projective(src: torch.Tensor, tgt: torch.Tensor, tgt_normals: torch.Tensor, width: int, height: int,
                   intrinsics, init_T=None, max_corr_dist: float = 0.2, max_iters: int = 15, conv_tol: float = 0.0,
                   stream=None, workspace: torch.Tensor | None = None, out_T: torch.Tensor | None = None,
                   out_stats: torch.Tensor | None = None, read_stats: bool = True):
    """Point-to-plane ICP with projective association into the organized
    target (height*width, 3).  Returns (T, stats dict or raw device tensor)."""
    src = _pts(src, "src")
    tgt = _pts(tgt, "tgt")
    tgt_normals = _pts(tgt_normals, "tgt_normals")
    if tgt.shape[0] != width * height or tgt_normals.shape[0] != width * height:
        raise ValueError("organized target must have width*height points and normals")
    dev = src.device
    T0 = None
    if init_T is not None:
        T0 = torch.as_tensor(init_T, dtype=torch.float64).reshape(4, 4).to(dev).contiguous()
    T = out_T if out_T is not None else torch.empty((4, 4), dtype=torch.float64, device=dev)
    stats = out_stats if out_stats is not None else torch.zeros(24, dtype=torch.uint8, device=dev)
    K = (ctypes.c_float * 4)(*[float(v) for v in intrinsics])
    need = lib.icp_projective_workspace_size(src.shape[0], int(max_iters))
    ws = workspace if workspace is not None else _ws.get(need, dev)
    st = lib.icp_projective(src.data_ptr(), src.shape[0], tgt.data_ptr(), tgt_normals.data_ptr(), int(width),
                            int(height), K, _ptr(T0), float(max_corr_dist), int(max_iters), float(conv_tol),
                            T.data_ptr(), stats.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream, locals()))
    _check(st, "icp_projective")
    if not read_stats:
        return T, stats
    return T, decode_stats(stats)


def decode_stats(stats: torch.Tensor) -> dict:
    import numpy as np
    raw = stats.cpu().numpy().tobytes()
    rec = np.frombuffer(raw, dtype=np.dtype(STATS_DTYPE))[0]
    return {name: rec[name].item() for name, _ in STATS_DTYPE}


def icp_history(workspace: torch.Tensor, n_src: int, n_tgt: int, max_iters: int, iterations: int):
    """(iterations, 8) float64 host array: increment, inliers, sum r^2."""
    p = lib.icp_history(workspace.data_ptr(), workspace.numel(), n_src, n_tgt, max_iters)
    if not p or iterations <= 0:
        return None
    off = p - workspace.data_ptr()
    h = workspace[off: off + 8 * 8 * iterations].view(torch.float64).reshape(iterations, 8)
    return h.cpu().numpy()


def workspace_for_icp(n_src: int, n_tgt: int, max_iters: int, device) -> torch.Tensor:
    need = lib.icp_point_to_plane_workspace_size(n_src, n_tgt, max_iters)
    return torch.empty(need, dtype=torch.uint8, device=device)


def _offsets(sizes_or_offsets, what: str):
    """int64 host offsets (m + 1) from a list of sizes or of offsets."""
    import numpy as np
    a = np.ascontiguousarray(np.asarray(sizes_or_offsets, dtype=np.int64))
    if a.ndim != 1:
        raise ValueError(f"{what} must be 1-D")
    return a


def offsets_from_sizes(sizes):
    import numpy as np
    sizes = np.asarray(sizes, dtype=np.int64)
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def estimate_normals_batched(xyz: torch.Tensor, offsets, k, viewpoint=(0.0, 0.0, 0.0), curvature: bool = True,
                             stream=None, workspace: torch.Tensor | None = None):
    """PCA normals of packed clouds: offsets (m+1 int64), k per cloud (int or m ints)."""
    import numpy as np
    xyz = _pts(xyz, "xyz")
    off = _offsets(offsets, "offsets")
    m = off.shape[0] - 1
    if m < 1 or off[-1] != xyz.shape[0]:
        raise ValueError("offsets must have m + 1 entries ending at len(xyz)")
    kc = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.int32), (m,)))
    n = xyz.shape[0]
    nrm = torch.empty((n, 3), dtype=torch.float32, device=xyz.device)
    cur = torch.empty((n,), dtype=torch.float32, device=xyz.device) if curvature else None
    vp = (ctypes.c_float * 3)(*[float(v) for v in viewpoint])
    need = lib.estimate_normals_batched_workspace_size(m, off.ctypes.data)
    ws = workspace if workspace is not None else _ws.get(need, xyz.device)
    st = lib.estimate_normals_batched(m, xyz.data_ptr(), off.ctypes.data, kc.ctypes.data, vp, nrm.data_ptr(),
                                      _ptr(cur), ws.data_ptr(), ws.numel(), _stream(stream, locals()))
    _check(st, "estimate_normals_batched")
    return nrm, cur


def icp_point_to_plane_batched(src: torch.Tensor, src_off, tgt: torch.Tensor, tgt_normals: torch.Tensor, tgt_off,
                               init_T=None, max_corr_dist=0.05, max_iters=30, conv_tol: float = 0.0, stream=None,
                               workspace: torch.Tensor | None = None, out_T: torch.Tensor | None = None,
                               out_stats: torch.Tensor | None = None, read_stats: bool = True):
    """Batched point-to-plane ICP over packed pairs.  Returns (T (m,4,4)
    float64 device tensor, stats): a list of dicts when read_stats (this
    synchronises), else the raw (m * 24)-byte device tensor."""
    import numpy as np
    src = _pts(src, "src")
    tgt = _pts(tgt, "tgt")
    tgt_normals = _pts(tgt_normals, "tgt_normals")
    so, to = _offsets(src_off, "src_off"), _offsets(tgt_off, "tgt_off")
    m = so.shape[0] - 1
    if m < 1 or to.shape[0] != m + 1 or so[-1] != src.shape[0] or to[-1] != tgt.shape[0]:
        raise ValueError("offsets must have m + 1 entries ending at the array lengths")
    if tgt_normals.shape[0] != tgt.shape[0]:
        raise ValueError("tgt_normals must match tgt")
    dm = np.ascontiguousarray(np.broadcast_to(np.asarray(max_corr_dist, dtype=np.float32), (m,)))
    mi = np.ascontiguousarray(np.broadcast_to(np.asarray(max_iters, dtype=np.int32), (m,)))
    dev = src.device
    T0 = None
    if init_T is not None:
        T0 = torch.as_tensor(init_T, dtype=torch.float64).reshape(m, 4, 4).to(dev).contiguous()
    T = out_T if out_T is not None else torch.empty((m, 4, 4), dtype=torch.float64, device=dev)
    stats = out_stats if out_stats is not None else torch.zeros(24 * m, dtype=torch.uint8, device=dev)
    need = lib.icp_point_to_plane_batched_workspace_size(m, so.ctypes.data, to.ctypes.data, int(mi.max()))
    ws = workspace if workspace is not None else _ws.get(need, dev)
    st = lib.icp_point_to_plane_batched(m, src.data_ptr(), so.ctypes.data, tgt.data_ptr(), tgt_normals.data_ptr(),
                                        to.ctypes.data, _ptr(T0), dm.ctypes.data, mi.ctypes.data, float(conv_tol),
                                        T.data_ptr(), stats.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream, locals()))
    _check(st, "icp_point_to_plane_batched")
    if not read_stats:
        return T, stats
    return T, decode_stats_batched(stats)


def icp_point_to_plane_with_normals_batched(src: torch.Tensor, src_off, tgt: torch.Tensor, tgt_off, k,
                                            viewpoint=(0.0, 0.0, 0.0), init_T=None, max_corr_dist=0.05,
                                            max_iters=30, conv_tol: float = 0.0, stream=None,
                                            workspace: torch.Tensor | None = None, out_T: torch.Tensor | None = None,
                                            out_stats: torch.Tensor | None = None, read_stats: bool = True,
                                            out_normals: torch.Tensor | None = None):
    """Target normals (k per pair) and batched point-to-plane ICP over one
    pyramid of all targets.  Returns (T (m,4,4), stats) like
    icp_point_to_plane_batched; the normals go to out_normals when given."""
    import numpy as np
    src = _pts(src, "src")
    tgt = _pts(tgt, "tgt")
    so, to = _offsets(src_off, "src_off"), _offsets(tgt_off, "tgt_off")
    m = so.shape[0] - 1
    if m < 1 or to.shape[0] != m + 1 or so[-1] != src.shape[0] or to[-1] != tgt.shape[0]:
        raise ValueError("offsets must have m + 1 entries ending at the array lengths")
    if out_normals is not None and (out_normals.dtype != torch.float32 or not out_normals.is_contiguous()
                                    or tuple(out_normals.shape) != (tgt.shape[0], 3)):
        raise ValueError("out_normals must be a contiguous float32 (n_tgt, 3) tensor")
    kk = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.int32), (m,)))
    dm = np.ascontiguousarray(np.broadcast_to(np.asarray(max_corr_dist, dtype=np.float32), (m,)))
    mi = np.ascontiguousarray(np.broadcast_to(np.asarray(max_iters, dtype=np.int32), (m,)))
    dev = src.device
    T0 = None
    if init_T is not None:
        T0 = torch.as_tensor(init_T, dtype=torch.float64).reshape(m, 4, 4).to(dev).contiguous()
    T = out_T if out_T is not None else torch.empty((m, 4, 4), dtype=torch.float64, device=dev)
    stats = out_stats if out_stats is not None else torch.zeros(24 * m, dtype=torch.uint8, device=dev)
    vpt = (ctypes.c_float * 3)(*[float(v) for v in viewpoint])
    need = lib.icp_point_to_plane_with_normals_batched_workspace_size(m, so.ctypes.data, to.ctypes.data,
                                                                      int(mi.max()))
    ws = workspace if workspace is not None else _ws.get(need, dev)
    st = lib.icp_point_to_plane_with_normals_batched(m, src.data_ptr(), so.ctypes.data, tgt.data_ptr(),
                                                     to.ctypes.data, kk.ctypes.data, vpt, _ptr(T0), dm.ctypes.data,
                                                     mi.ctypes.data, float(conv_tol), T.data_ptr(), stats.data_ptr(),
                                                     _ptr(out_normals), ws.data_ptr(), ws.numel(), _stream(stream, locals()))
    _check(st, "icp_point_to_plane_with_normals_batched")
    if not read_stats:
        return T, stats
    return T, decode_stats_batched(stats)


def decode_stats_batched(stats: torch.Tensor) -> list:
    import numpy as np
    raw = stats.cpu().numpy().tobytes()
    recs = np.frombuffer(raw, dtype=np.dtype(STATS_DTYPE))
    return [{name: r[name].item() for name, _ in STATS_DTYPE} for r in recs]


def set_tuning(icp_block_threads: int = 128, icp_leaf: int = 16, node_budget: float = 1.0, sort_queries: int = 1,
               icp_persistent: int = 0):
    t = Tuning(int(icp_block_threads), int(icp_leaf), float(node_budget), int(sort_queries), int(icp_persistent))
    _check(lib.pc_set_tuning(ctypes.byref(t)), "pc_set_tuning")


def get_tuning() -> dict:
    t = Tuning()
    lib.pc_get_tuning(ctypes.byref(t))
    return {"icp_block_threads": t.icp_block_threads, "icp_leaf": t.icp_leaf, "node_budget": t.node_budget,
            "sort_queries": t.sort_queries, "icp_persistent": t.icp_persistent}


def copy_probe(dst: torch.Tensor, src: torch.Tensor, stream=None):
    _check(lib.pc_copy_probe(dst.data_ptr(), src.data_ptr(), src.numel() * src.element_size(),
                             _stream(stream, locals())), "pc_copy_probe")


# ---------------------------------------------------------------------------
# Learned pose initialiser and multi-start ICP
# ---------------------------------------------------------------------------
def _pair_offsets(src, src_off, tgt, tgt_off):
    so, to = _offsets(src_off, "src_off"), _offsets(tgt_off, "tgt_off")
    m = so.shape[0] - 1
    if m < 1 or to.shape[0] != m + 1 or so[-1] != src.shape[0] or to[-1] != tgt.shape[0]:
        raise ValueError("offsets must have m + 1 entries ending at the array lengths")
    return so, to, m


def _params(params: torch.Tensor, what: str) -> torch.Tensor:
    n = lib.pose_net_param_count()
    if params.dtype != torch.float32 or params.numel() != n or not params.is_contiguous() or not params.is_cuda:
        raise ValueError(f"{what} must be a contiguous float32 CUDA tensor of {n} values")
    return params


def pose_net_param_count() -> int:
    return lib.pose_net_param_count()


def pose_net_predict(params: torch.Tensor, src: torch.Tensor, src_off, tgt: torch.Tensor, tgt_off, stream=None,
                     workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Initial pose (m, 4, 4) float64 of every packed pair."""
    params = _params(params, "params")
    src, tgt = _pts(src, "src"), _pts(tgt, "tgt")
    so, to, m = _pair_offsets(src, src_off, tgt, tgt_off)
    T = torch.empty((m, 4, 4), dtype=torch.float64, device=src.device)
    need = lib.pose_net_workspace_size(m, so.ctypes.data, to.ctypes.data)
    ws = workspace if workspace is not None else _ws.get(need, src.device)
    _check(lib.pose_net_predict(params.data_ptr(), m, src.data_ptr(), so.ctypes.data, tgt.data_ptr(), to.ctypes.data,
                                T.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream, locals())), "pose_net_predict")
    return T


def pose_net_train_step(params: torch.Tensor, adam_m, adam_v, step: int, lr: float, src: torch.Tensor, src_off,
                        tgt: torch.Tensor, tgt_off, label_T: torch.Tensor, pair_weight=None, want_grad=False,
                        stream=None, workspace: torch.Tensor | None = None):
    """One training step (Adam when lr > 0).  Returns (per-pair loss tensor,
    summed gradient tensor or None)."""
    params = _params(params, "params")
    if lr > 0:
        adam_m, adam_v = _params(adam_m, "adam_m"), _params(adam_v, "adam_v")
    src, tgt = _pts(src, "src"), _pts(tgt, "tgt")
    so, to, m = _pair_offsets(src, src_off, tgt, tgt_off)
    dev = src.device
    lab = torch.as_tensor(label_T, dtype=torch.float64).reshape(m, 4, 4).to(dev).contiguous()
    w = None
    if pair_weight is not None:
        w = torch.as_tensor(pair_weight, dtype=torch.float32).reshape(m).to(dev).contiguous()
    loss = torch.empty(m, dtype=torch.float32, device=dev)
    grad = torch.empty(lib.pose_net_param_count(), dtype=torch.float32, device=dev) if want_grad else None
    need = lib.pose_net_workspace_size(m, so.ctypes.data, to.ctypes.data)
    ws = workspace if workspace is not None else _ws.get(need, dev)
    _check(lib.pose_net_train_step(params.data_ptr(), _ptr(adam_m) if lr > 0 else None,
                                   _ptr(adam_v) if lr > 0 else None, int(step), float(lr), m, src.data_ptr(),
                                   so.ctypes.data, tgt.data_ptr(), to.ctypes.data, lab.data_ptr(), _ptr(w),
                                   loss.data_ptr(), _ptr(grad), ws.data_ptr(), ws.numel(), _stream(stream, locals())),
           "pose_net_train_step")
    return loss, grad


def icp_learned_batched(mode: int, params, src: torch.Tensor, src_off, tgt: torch.Tensor, tgt_normals: torch.Tensor,
                        tgt_off, max_corr_dist: float, max_iters: int, conv_tol: float = 0.0,
                        accept_rms: float = 0.0, stream=None, workspace: torch.Tensor | None = None,
                        read_stats: bool = True):
    """Registration from the learned start with multi-start fallback
    (PC_INIT_LEARNED), multi-start only or learned only.  Returns (T (m,4,4),
    stats (list of dicts, or the raw device tensor), start index per pair
    (int32 device tensor; -1 = learned))."""
    if mode != PC_INIT_MULTI_START:
        params = _params(params, "params")
    src, tgt = _pts(src, "src"), _pts(tgt, "tgt")
    tgt_normals = _pts(tgt_normals, "tgt_normals")
    if tgt_normals.shape[0] != tgt.shape[0]:
        raise ValueError("tgt_normals must match tgt")
    so, to, m = _pair_offsets(src, src_off, tgt, tgt_off)
    dev = src.device
    T = torch.empty((m, 4, 4), dtype=torch.float64, device=dev)
    stats = torch.zeros(24 * m, dtype=torch.uint8, device=dev)
    start = torch.empty(m, dtype=torch.int32, device=dev)
    need = lib.icp_learned_batched_workspace_size(m, so.ctypes.data, to.ctypes.data, int(max_iters))
    if need == 0:
        raise ValueError("icp_learned_batched: sizes out of range")
    ws = workspace if workspace is not None else _ws.get(need, dev)
    _check(lib.icp_learned_batched(int(mode), _ptr(params) if mode != PC_INIT_MULTI_START else None, m,
                                   src.data_ptr(), so.ctypes.data, tgt.data_ptr(), tgt_normals.data_ptr(),
                                   to.ctypes.data, float(max_corr_dist), int(max_iters), float(conv_tol),
                                   float(accept_rms), T.data_ptr(), stats.data_ptr(), start.data_ptr(),
                                   ws.data_ptr(), ws.numel(), _stream(stream, locals())), "icp_learned_batched")
    if not read_stats:
        return T, stats, start
    return T, decode_stats_batched(stats), start
