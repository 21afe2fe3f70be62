"""ctypes binding of libclusco.so (include/clusco.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch supplies device memory (outputs and workspaces come from
its caching allocator) and the current stream.  If the library is not built
every call raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libclusco.so")

OK, ERR_INVALID_ARG, ERR_WORKSPACE, ERR_UNSUPPORTED, ERR_HIP = range(5)
PRECISION = {"fp32": 0, "bf16": 1, "split_bf16": 1, "fp16": 2, "split_fp16": 2, "fp64": 3,
             "bf16x4": 4, "split_bf16x4": 4}

SCHEDULES = {"staged": 0, "persistent": 1}


class Config(ctypes.Structure):
    """clusco_config"""
    _fields_ = [("products", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("band", ctypes.c_int32), ("frame", ctypes.c_int32), ("source", ctypes.c_int32),
                ("bucket", ctypes.c_int32)]

    def as_dict(self):
        return {"products": self.products,
                "schedule": {v: k for k, v in SCHEDULES.items()}.get(self.schedule, self.schedule),
                "band": self.band, "frame": self.frame,
                "source": ["default", "table", "forced"][self.source], "bucket": self.bucket}


_lib = None
_lock = threading.Lock()
_handles: dict[int, ctypes.c_void_p] = {}


class ClucsoError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str = ""):
        self.status = status
        names = {1: "INVALID_ARG", 2: "WORKSPACE", 3: "UNSUPPORTED", 4: "HIP"}
        super().__init__(f"{what}: CLUSCO_ERR_{names.get(status, status)}"
                         + (f" ({detail})" if detail else ""))


def lib():
    """Load libclusco.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; "
                               "g.build()'` first")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, i64, i32, d = (ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64, ctypes.c_int32,
                               ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        st = ctypes.c_int
        sig = {
            "clusco_create": (st, [ctypes.POINTER(vp), ctypes.c_int]),
            "clusco_destroy": (None, [vp]),
            "clusco_status_string": (ctypes.c_char_p, [st]),
            "clusco_last_error": (ctypes.c_char_p, [vp]),
            "clusco_set_tolerance": (st, [vp, st, d]),
            "clusco_flag_epsilon": (st, [vp, st, i64, ctypes.POINTER(d)]),
            "clusco_crmsd_workspace_size": (sz, [vp, i64, i64, st]),
            "clusco_crmsd_matrix": (st, [vp, vp, i64, i64, st, vp, vp, sz, vp]),
            "clusco_crmsd_matrix_noalloc": (st, [vp, vp, i64, i64, st, vp, vp]),
            "clusco_load_tuning": (st, [vp, ctypes.c_char_p]),
            "clusco_tuning_path": (ctypes.c_char_p, [vp]),
            "clusco_get_config": (st, [vp, i64, i64, st, ctypes.POINTER(Config)]),
            "clusco_get_config_batched": (st, [vp, i64, i64, st, ctypes.POINTER(Config)]),
            "clusco_force_config": (st, [vp, ctypes.POINTER(Config)]),
            "clusco_drmsd_workspace_size": (sz, [vp, i64, i64, st]),
            "clusco_cluster_workspace_size": (sz, [vp, i64, i32]),
            "clusco_cmo_workspace_size": (sz, [vp, i64, i64]),
            "clusco_cmo_matrix": (st, [vp, vp, i64, i64, ctypes.c_float, vp, vp, sz, vp]),
            "clusco_kmedoids": (st, [vp, vp, i64, i32, vp, i32, i32, vp, vp, vp, vp, vp, vp, sz,
                                     vp]),
            "clusco_drmsd_matrix": (st, [vp, vp, i64, i64, st, vp, vp, sz, vp]),
            "clusco_fixup_count": (st, [vp, vp, i64p, vp]),
            "clusco_stage_timing": (st, [vp, ctypes.c_int]),
            "clusco_stage_times": (st, [vp, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int)]),
            "clusco_crmsd_batched_workspace_size": (sz, [vp, i32, i64p, i64p, st]),
            "clusco_crmsd_batched": (st, [vp, i32, i64p, i64p, i64p, i64p, vp, st, vp, vp, sz, vp]),
            "clusco_crmsd_cross_workspace_size": (sz, [vp, i64, i64, i64, st]),
            "clusco_crmsd_cross": (st, [vp, vp, i64, vp, i64, i64, st, vp, vp, sz, vp]),
            "clusco_crmsd_backward_workspace_size": (sz, [vp, i64, i64, st]),
            "clusco_crmsd_backward": (st, [vp, vp, i64, i64, vp, vp, st, vp, vp, sz, vp]),
            "clusco_crmsd_cross_backward_workspace_size": (sz, [vp, i64, i64, i64, st]),
            "clusco_crmsd_cross_backward": (st, [vp, vp, i64, vp, i64, i64, vp, vp, st, vp, vp,
                                                 vp, sz, vp]),
            "clusco_crmsd_threshold_workspace_size": (sz, [vp, i64, i64, st]),
            "clusco_crmsd_threshold": (st, [vp, vp, i64, i64, st, ctypes.c_float, vp, vp, vp, i64,
                                            vp, vp, sz, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        return L


def handle(device: int) -> ctypes.c_void_p:
    h = _handles.get(device)
    if h is None:
        h = ctypes.c_void_p()
        rc = lib().clusco_create(ctypes.byref(h), device)
        if rc != OK:
            raise ClucsoError(rc, "clusco_create")
        _handles[device] = h
    return h


def _check(rc, h, what):
    if rc != OK:
        detail = lib().clusco_last_error(h)
        raise ClucsoError(rc, what, detail.decode() if detail else "")


def _prec(p) -> int:
    if isinstance(p, int):
        return p
    try:
        return PRECISION[p]
    except KeyError:
        raise ValueError(f"unknown precision {p!r}; use one of {sorted(PRECISION)}") from None


def _coords(x: torch.Tensor, name="coords") -> torch.Tensor:
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != torch.float32 or x.dim() != 3 or x.shape[2] != 3:
        raise TypeError(f"{name} must be float32 [N, L, 3], got {x.dtype} {tuple(x.shape)}")
    return x.contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else None


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _workspace(nbytes: int, device, ws: torch.Tensor | None):
    if ws is not None and ws.numel() >= nbytes and ws.device == device:
        return ws
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def set_tolerance(precision, tol: float, device: int = 0):
    """Fix-up tolerance (A) for a precision; tol <= 0 disables the FP64 fix-up."""
    h = handle(device)
    _check(lib().clusco_set_tolerance(h, _prec(precision), float(tol)), h, "clusco_set_tolerance")


def flag_epsilon(precision, L: int, device: int = 0) -> float:
    """Relative contraction error the fix-up flag assumes for this precision
    and model length (see clusco_flag_epsilon)."""
    h = handle(device)
    e = ctypes.c_double()
    _check(lib().clusco_flag_epsilon(h, _prec(precision), int(L), ctypes.byref(e)), h,
           "clusco_flag_epsilon")
    return float(e.value)


def load_tuning(path: str | None, device: int = 0):
    """Replace the handle's tuning table with the JSON file at `path`
    (None: drop it, back to the built-in default configuration)."""
    h = handle(device)
    _check(lib().clusco_load_tuning(h, path.encode() if path is not None else None), h,
           "clusco_load_tuning")


def tuning_path(device: int = 0) -> str:
    return lib().clusco_tuning_path(handle(device)).decode()


def get_config(N: int, L: int, precision="bf16", device: int = 0, batched: bool = False) -> dict:
    """The kernel configuration calls with these sizes will use (batched: the
    one an ensemble of these sizes takes inside a batched call)."""
    h = handle(device)
    c = Config()
    name = "clusco_get_config_batched" if batched else "clusco_get_config"
    _check(getattr(lib(), name)(h, int(N), int(L), _prec(precision), ctypes.byref(c)), h, name)
    return c.as_dict()


def force_config(products: int | None = None, schedule: str = "staged", band: int = 16,
                 frame: int = 1, device: int = 0):
    """Force one configuration for every later call (products None: back to
    the tuning table)."""
    h = handle(device)
    if products is None:
        _check(lib().clusco_force_config(h, None), h, "clusco_force_config")
        return
    c = Config(int(products), SCHEDULES[schedule], int(band), int(frame), 0, -1)
    _check(lib().clusco_force_config(h, ctypes.byref(c)), h, "clusco_force_config")


def workspace_size(N: int, L: int, precision="fp32", device: int = 0) -> int:
    return int(lib().clusco_crmsd_workspace_size(handle(device), N, L, _prec(precision)))


def crmsd_matrix(x: torch.Tensor, precision="fp32", out: torch.Tensor | None = None,
                 ws: torch.Tensor | None = None) -> torch.Tensor:
    """Packed all-vs-all cRMSD [N(N-1)/2] of x [N, L, 3] (float32, on the GPU)."""
    x = _coords(x)
    N, L = x.shape[0], x.shape[1]
    dev = x.device
    h = handle(dev.index)
    p = _prec(precision)
    need = int(lib().clusco_crmsd_workspace_size(h, N, L, p))
    if need == 0:
        raise ClucsoError(ERR_INVALID_ARG, "clusco_crmsd_workspace_size", f"N={N} L={L}")
    ws = _workspace(need, dev, ws)
    P = N * (N - 1) // 2
    if out is None:
        out = torch.empty(P, dtype=torch.float32, device=dev)
    elif out.numel() != P or out.dtype != torch.float32 or not out.is_contiguous():
        raise TypeError("out must be a contiguous float32 tensor of N(N-1)/2 elements")
    rc = lib().clusco_crmsd_matrix(h, _ptr(x), N, L, p, _ptr(out), _ptr(ws), ws.numel(),
                                   _stream(dev))
    _check(rc, h, "clusco_crmsd_matrix")
    return out


SCRATCH_BYTES = 64 << 20   # CLUSCO_SCRATCH_BYTES


def crmsd_matrix_noalloc(x: torch.Tensor, out: torch.Tensor, precision="fp32") -> torch.Tensor:
    """clusco_crmsd_matrix_noalloc: the packed all-vs-all cRMSD of x into the
    caller's `out`, using the library's built-in device scratch (allocates
    nothing; calls on one device must not overlap)."""
    x = _coords(x)
    N, L = x.shape[0], x.shape[1]
    dev = x.device
    h = handle(dev.index)
    P = N * (N - 1) // 2
    if out.numel() != P or out.dtype != torch.float32 or not out.is_contiguous() or \
            out.device != dev:
        raise TypeError("out must be a contiguous float32 tensor of N(N-1)/2 elements on "
                        "the device of x")
    rc = lib().clusco_crmsd_matrix_noalloc(h, _ptr(x), N, L, _prec(precision), _ptr(out),
                                           _stream(dev))
    _check(rc, h, "clusco_crmsd_matrix_noalloc")
    return out


def drmsd_workspace_size(N: int, L: int, precision="bf16", device: int = 0) -> int:
    return int(lib().clusco_drmsd_workspace_size(handle(device), N, L, _prec(precision)))


def drmsd_matrix(x: torch.Tensor, precision="bf16", out: torch.Tensor | None = None,
                 ws: torch.Tensor | None = None) -> torch.Tensor:
    """Packed all-vs-all dRMSD [N(N-1)/2] of x [N, L, 3] (float32, on the GPU)."""
    x = _coords(x)
    N, L = x.shape[0], x.shape[1]
    dev = x.device
    h = handle(dev.index)
    p = _prec(precision)
    need = int(lib().clusco_drmsd_workspace_size(h, N, L, p))
    if need == 0:
        raise ClucsoError(ERR_INVALID_ARG, "clusco_drmsd_workspace_size", f"N={N} L={L}")
    ws = _workspace(need, dev, ws)
    P = N * (N - 1) // 2
    if out is None:
        out = torch.empty(P, dtype=torch.float32, device=dev)
    elif out.numel() != P or out.dtype != torch.float32 or not out.is_contiguous():
        raise TypeError("out must be a contiguous float32 tensor of N(N-1)/2 elements")
    rc = lib().clusco_drmsd_matrix(h, _ptr(x), N, L, p, _ptr(out), _ptr(ws), ws.numel(),
                                   _stream(dev))
    _check(rc, h, "clusco_drmsd_matrix")
    return out


def cmo_workspace_size(N: int, L: int, device: int = 0) -> int:
    return int(lib().clusco_cmo_workspace_size(handle(device), N, L))


def cmo_matrix(x: torch.Tensor, cutoff: float = 8.0, out: torch.Tensor | None = None,
               ws: torch.Tensor | None = None) -> torch.Tensor:
    """Packed all-vs-all contact map overlap [N(N-1)/2] (Sorensen index, 0..100)
    of x [N, L, 3] (float32, on the GPU), contacts below `cutoff` Angstrom."""
    x = _coords(x)
    N, L = x.shape[0], x.shape[1]
    dev = x.device
    h = handle(dev.index)
    need = int(lib().clusco_cmo_workspace_size(h, N, L))
    if need == 0:
        raise ClucsoError(ERR_INVALID_ARG, "clusco_cmo_workspace_size", f"N={N} L={L}")
    ws = _workspace(need, dev, ws)
    P = N * (N - 1) // 2
    if out is None:
        out = torch.empty(P, dtype=torch.float32, device=dev)
    elif out.numel() != P or out.dtype != torch.float32 or not out.is_contiguous():
        raise TypeError("out must be a contiguous float32 tensor of N(N-1)/2 elements")
    rc = lib().clusco_cmo_matrix(h, _ptr(x), N, L, float(cutoff), _ptr(out), _ptr(ws),
                                 ws.numel(), _stream(dev))
    _check(rc, h, "clusco_cmo_matrix")
    return out


def kmedoids(D: torch.Tensor, N: int, k: int, init=None, max_iter: int = 100,
             ws: torch.Tensor | None = None, check_every: int = 4) -> dict:
    """K-means with member centres over a packed score matrix D [N(N-1)/2]
    (float32, on the GPU).  init: k distinct model indices (host sequence;
    default: evenly spaced models).  check_every > 0 polls convergence every
    that many steps (synchronising); 0 enqueues all max_iter steps
    asynchronously.  Returns device tensors labels [N],
    medoids [k], sizes [k], mean_r [k] and info [3] (representative cluster,
    updates run, converged)."""
    if D.dtype != torch.float32 or not D.is_cuda or not D.is_contiguous():
        raise TypeError("D must be a contiguous float32 CUDA tensor")
    if D.numel() != N * (N - 1) // 2:
        raise ValueError("D must hold N(N-1)/2 scores")
    if init is None:
        init = [(c * N) // k for c in range(k)]
    h_init = (ctypes.c_int32 * k)(*[int(v) for v in init])
    dev = D.device
    h = handle(dev.index)
    need = int(lib().clusco_cluster_workspace_size(h, N, k))
    if need == 0:
        raise ClucsoError(ERR_INVALID_ARG, "clusco_cluster_workspace_size", f"N={N} k={k}")
    ws = _workspace(need, dev, ws)
    out = {"labels": torch.empty(N, dtype=torch.int32, device=dev),
           "medoids": torch.empty(k, dtype=torch.int32, device=dev),
           "sizes": torch.empty(k, dtype=torch.int64, device=dev),
           "mean_r": torch.empty(k, dtype=torch.float64, device=dev),
           "info": torch.empty(3, dtype=torch.int64, device=dev)}
    rc = lib().clusco_kmedoids(h, _ptr(D), N, k, h_init, max_iter, check_every,
                               _ptr(out["labels"]), _ptr(out["medoids"]), _ptr(out["sizes"]), _ptr(out["mean_r"]),
                               _ptr(out["info"]), _ptr(ws), ws.numel(), _stream(dev))
    _check(rc, h, "clusco_kmedoids")
    return out


def fixup_count(ws: torch.Tensor) -> int:
    """32x32 pair blocks the last forward on this workspace sent to the FP64 fix-up."""
    h = handle(ws.device.index)
    n = ctypes.c_int64()
    _check(lib().clusco_fixup_count(h, _ptr(ws), ctypes.byref(n), _stream(ws.device)), h,
           "clusco_fixup_count")
    return int(n.value)


def stage_timing(device: int, max_calls: int):
    """Record HIP events around the stages of the next max_calls forward calls."""
    h = handle(device)
    _check(lib().clusco_stage_timing(h, int(max_calls)), h, "clusco_stage_timing")


def stage_times(device: int):
    """([prep, contraction+epilogue, fix-up] summed ms, calls) since the last read."""
    h = handle(device)
    ms = (ctypes.c_double * 3)()
    n = ctypes.c_int()
    _check(lib().clusco_stage_times(h, ms, ctypes.byref(n)), h, "clusco_stage_times")
    return [ms[k] for k in range(3)], n.value


def crmsd_cross(a: torch.Tensor, b: torch.Tensor, precision="fp32",
                out: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """Dense cRMSD [Na, Nb] between a [Na, L, 3] and b [Nb, L, 3] (Nb = 1: every
    model against one reference)."""
    a = _coords(a, "a")
    b = _coords(b, "b")
    if a.shape[1] != b.shape[1] or a.device != b.device:
        raise TypeError("a and b need the same L and device")
    Na, Nb, L = a.shape[0], b.shape[0], a.shape[1]
    dev = a.device
    h = handle(dev.index)
    p = _prec(precision)
    need = int(lib().clusco_crmsd_cross_workspace_size(h, Na, Nb, L, p))
    if need == 0:
        raise ClucsoError(ERR_INVALID_ARG, "clusco_crmsd_cross_workspace_size")
    ws = _workspace(need, dev, ws)
    if out is None:
        out = torch.empty(Na, Nb, dtype=torch.float32, device=dev)
    elif out.numel() != Na * Nb or out.dtype != torch.float32 or not out.is_contiguous():
        raise TypeError("out must be a contiguous float32 tensor of Na*Nb elements")
    rc = lib().clusco_crmsd_cross(h, _ptr(a), Na, _ptr(b), Nb, L, p, _ptr(out), _ptr(ws),
                                  ws.numel(), _stream(dev))
    _check(rc, h, "clusco_crmsd_cross")
    return out


def _i64(arr):
    import numpy as np
    a = np.ascontiguousarray(arr, dtype=np.int64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


class Batch:
    """Shapes and offsets of E ensembles stored back to back in one float32
    buffer; packed outputs back to back in another."""

    def __init__(self, shapes):
        import numpy as np
        self.shapes = [(int(n), int(l)) for n, l in shapes]
        self.N = np.array([n for n, _ in self.shapes], dtype=np.int64)
        self.L = np.array([l for _, l in self.shapes], dtype=np.int64)
        sizes = self.N * self.L * 3
        self.coord_off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
        pairs = self.N * (self.N - 1) // 2
        self.out_off = np.concatenate([[0], np.cumsum(pairs)[:-1]]).astype(np.int64)
        self.n_coords = int(sizes.sum())
        self.n_out = int(pairs.sum())

    def pack(self, ensembles, device):
        flat = torch.cat([e.reshape(-1) for e in ensembles]) if ensembles else \
            torch.empty(0, dtype=torch.float32)
        return flat.to(device=device, dtype=torch.float32).contiguous()

    def split(self, out):
        return [out[o:o + n * (n - 1) // 2] for o, (n, _) in zip(self.out_off, self.shapes)]


def batched_workspace_size(batch: Batch, precision="fp32", device: int = 0) -> int:
    _, pN = _i64(batch.N)
    _, pL = _i64(batch.L)
    return int(lib().clusco_crmsd_batched_workspace_size(handle(device), len(batch.shapes), pN,
                                                         pL, _prec(precision)))


def crmsd_batched(batch: Batch, coords: torch.Tensor, precision="fp32",
                  out: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """All-vs-all cRMSD of every ensemble of `batch`; coords is the flat float32
    buffer of all models (Batch.pack).  Returns the flat packed output
    (Batch.split gives the per-ensemble views)."""
    if not isinstance(coords, torch.Tensor) or not coords.is_cuda or coords.dtype != torch.float32:
        raise TypeError("coords must be a float32 CUDA tensor")
    coords = coords.contiguous()
    if coords.numel() < batch.n_coords:
        raise TypeError("coords holds fewer values than the batch needs")
    dev = coords.device
    h = handle(dev.index)
    p = _prec(precision)
    E = len(batch.shapes)
    aN, pN = _i64(batch.N)
    aL, pL = _i64(batch.L)
    aC, pC = _i64(batch.coord_off)
    aO, pO = _i64(batch.out_off)
    need = int(lib().clusco_crmsd_batched_workspace_size(h, E, pN, pL, p))
    if need == 0 and E > 0:
        raise ClucsoError(ERR_INVALID_ARG, "clusco_crmsd_batched_workspace_size")
    ws = _workspace(need, dev, ws)
    if out is None:
        out = torch.empty(batch.n_out, dtype=torch.float32, device=dev)
    elif out.numel() < batch.n_out or out.dtype != torch.float32 or not out.is_contiguous():
        raise TypeError("out too small")
    rc = lib().clusco_crmsd_batched(h, E, pN, pL, pC, pO, _ptr(coords), p, _ptr(out), _ptr(ws),
                                    ws.numel(), _stream(dev))
    _check(rc, h, "clusco_crmsd_batched")
    return out


def crmsd_backward(x: torch.Tensor, rmsd: torch.Tensor, grad_out: torch.Tensor,
                   precision="fp32", grad: torch.Tensor | None = None,
                   ws: torch.Tensor | None = None) -> torch.Tensor:
    """d/dx of sum_k grad_out[k] * rmsd_k for the packed all-vs-all scores."""
    x = _coords(x)
    N, L = x.shape[0], x.shape[1]
    P = N * (N - 1) // 2
    if rmsd.numel() != P or grad_out.numel() != P:
        raise TypeError("rmsd and grad_out must hold N(N-1)/2 values")
    rmsd = rmsd.to(torch.float32).contiguous()
    grad_out = grad_out.to(torch.float32).contiguous()
    dev = x.device
    h = handle(dev.index)
    p = _prec(precision)
    need = int(lib().clusco_crmsd_backward_workspace_size(h, N, L, p))
    ws = _workspace(need, dev, ws)
    if grad is None:
        grad = torch.empty_like(x)
    rc = lib().clusco_crmsd_backward(h, _ptr(x), N, L, _ptr(rmsd), _ptr(grad_out), p, _ptr(grad),
                                     _ptr(ws), ws.numel(), _stream(dev))
    _check(rc, h, "clusco_crmsd_backward")
    return grad


def crmsd_cross_backward(a: torch.Tensor, b: torch.Tensor, rmsd: torch.Tensor,
                         grad_out: torch.Tensor, precision="fp32", need_b: bool = True,
                         ws: torch.Tensor | None = None):
    """(d/da, d/db) of sum grad_out[ia, ib] * rmsd[ia, ib] for the dense cross scores."""
    a = _coords(a, "a")
    b = _coords(b, "b")
    Na, Nb, L = a.shape[0], b.shape[0], a.shape[1]
    if rmsd.numel() != Na * Nb or grad_out.numel() != Na * Nb:
        raise TypeError("rmsd and grad_out must hold Na*Nb values")
    rmsd = rmsd.to(torch.float32).contiguous()
    grad_out = grad_out.to(torch.float32).contiguous()
    dev = a.device
    h = handle(dev.index)
    p = _prec(precision)
    need = int(lib().clusco_crmsd_cross_backward_workspace_size(h, Na, Nb, L, p))
    ws = _workspace(need, dev, ws)
    ga = torch.empty_like(a)
    gb = torch.empty_like(b) if need_b else None
    rc = lib().clusco_crmsd_cross_backward(h, _ptr(a), Na, _ptr(b), Nb, L, _ptr(rmsd),
                                           _ptr(grad_out), p, _ptr(ga), _ptr(gb), _ptr(ws),
                                           ws.numel(), _stream(dev))
    _check(rc, h, "clusco_crmsd_cross_backward")
    return ga, gb


def crmsd_threshold(x: torch.Tensor, cutoff: float, precision="fp32",
                    capacity: int | None = None, ws: torch.Tensor | None = None,
                    sync: bool = True):
    """Pairs (i, j), i < j, with cRMSD below `cutoff` (A), in no particular order.

    Returns (i, j, score, count): int32, int32 and float32 device tensors of
    min(count, capacity) entries and the number of such pairs.  With
    capacity=None every pair is kept (a second call with exact arrays is made
    when the first guess is too small).  With sync=False the arrays are
    returned at full capacity with count as a device uint64 tensor.
    """
    x = _coords(x)
    N, L = x.shape[0], x.shape[1]
    dev = x.device
    h = handle(dev.index)
    p = _prec(precision)
    P = N * (N - 1) // 2
    need = int(lib().clusco_crmsd_threshold_workspace_size(h, N, L, p))
    ws = _workspace(need, dev, ws)
    auto = capacity is None
    cap = min(P, 1 << 22) if auto else int(capacity)
    for attempt in range(2):
        oi = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        oj = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        os_ = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)   # holds the uint64 count
        rc = lib().clusco_crmsd_threshold(h, _ptr(x), N, L, p, ctypes.c_float(cutoff), _ptr(oi),
                                          _ptr(oj), _ptr(os_), cap, _ptr(cnt), _ptr(ws),
                                          ws.numel(), _stream(dev))
        _check(rc, h, "clusco_crmsd_threshold")
        if not sync:
            return oi, oj, os_, cnt
        n = int(cnt.item())
        if n <= cap or not auto:
            k = min(n, cap)
            return oi[:k], oj[:k], os_[:k], n
        cap = n
    raise RuntimeError("pair count changed between identical calls")
