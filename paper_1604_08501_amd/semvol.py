"""Python binding of libsem.so: the strong-form spectral-element volume term
(Sec. 2, Eq. (volterm)) on an MI355X.

Argument marshalling only.  Every function hands device pointers of torch
tensors and torch's current HIP stream to the C-ABI declared in
``include/sem.h``; all arithmetic runs in the library's HIP kernels.  There
is no CPU fallback: without a built ``libsem.so`` every call raises.

Layouts (see ``include/sem.h``): ``q``/``rhs`` ``[Ne, 5, Nq^3]``, ``geo``
``[Ne, 10, Nq^3]``, ``D`` ``[Nq, Nq]``, ``rho_ref`` ``[Ne, Nq^3]`` (dtype of
``q``), ``theta_ref`` ``[Ne, Nq^3]`` float64.
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import Optional, Sequence

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsem.so")

SEM_OK, SEM_ERR_INVALID_ARG, SEM_ERR_UNSUPPORTED, SEM_ERR_HIP, SEM_ERR_NO_MEMORY = 0, -1, -2, -3, -4
SEM_F64, SEM_F32 = 0, 1
SEM_PLAN_AUTOTUNE, SEM_PLAN_USE_CACHE, SEM_RK3_SEPARATE_STAGES = 1, 2, 4
SEM_LAYOUT_DEFAULT, SEM_LAYOUT_FULL, SEM_LAYOUT_ALIAS = 0, 1, 2
SEM_DIR_R, SEM_DIR_S, SEM_DIR_T = 1, 2, 4
LAYOUTS = {"default": SEM_LAYOUT_DEFAULT, "full": SEM_LAYOUT_FULL, "alias": SEM_LAYOUT_ALIAS}

# every symbol include/sem.h declares
EXPORTS = (
    "sem_last_error", "sem_version", "sem_tile_options", "sem_volume_rhs", "sem_volume_rhs_tiled",
    "sem_volume_rhs_ext", "sem_volume_rhs_ladder", "sem_volume_rhs_affine", "sem_volume_rhs_adjoint",
    "sem_axpby", "sem_batch_plan", "sem_batch_execute",
    "sem_plan_describe", "sem_plan_destroy", "sem_rk3_graph_create", "sem_rk3_graph_launch",
    "sem_rk3_graph_describe", "sem_rk3_graph_destroy", "sem_set_max_workgroups",
    "sem_surface_rhs", "sem_batch_rhs_static", "sem_rhs",
)


class SemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[semvol status {status}] {msg}")
        self.status = status


class sem_phys(ctypes.Structure):
    _fields_ = [("p0", ctypes.c_double), ("gamma", ctypes.c_double),
                ("R", ctypes.c_double), ("grav", ctypes.c_double)]


class sem_tile(ctypes.Structure):
    _fields_ = [("elems_per_block", ctypes.c_int32), ("layout", ctypes.c_int32)]


class sem_block(ctypes.Structure):
    _fields_ = [("Nq", ctypes.c_int32), ("Ne", ctypes.c_int32), ("D", ctypes.c_void_p),
                ("geo", ctypes.c_void_p), ("q", ctypes.c_void_p), ("rho_ref", ctypes.c_void_p),
                ("theta_ref", ctypes.c_void_p), ("rhs", ctypes.c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libsem.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1604_08501_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, d, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32
    P = ctypes.POINTER
    sig = {
        "sem_last_error": ([], ctypes.c_char_p),
        "sem_version": ([], ctypes.c_char_p),
        "sem_tile_options": ([i32, i32, P(sem_tile), i32], i32),
        "sem_volume_rhs": ([i32, i32, i32, vp, vp, vp, vp, vp, P(sem_phys), vp, i32, vp], i32),
        "sem_volume_rhs_tiled": ([i32, i32, i32, vp, vp, vp, vp, vp, P(sem_phys), vp, i32,
                                  P(sem_tile), vp], i32),
        "sem_volume_rhs_ext": ([i32, i32, i32, i32, u32, vp, vp, vp, vp, vp, P(sem_phys), vp, i32,
                                vp], i32),
        "sem_volume_rhs_ladder": ([i32, i32, i32, vp, vp, vp, P(sem_phys), vp, vp], i32),
        "sem_volume_rhs_affine": ([i32, i32, i32, vp, vp, vp, vp, vp, P(sem_phys), vp, i32, vp],
                                  i32),
        "sem_volume_rhs_adjoint": ([i32, i32, i32, vp, vp, vp, P(sem_phys), vp, vp, i32, vp], i32),
        "sem_axpby": ([i64, i32, d, vp, d, vp, d, vp, vp, vp], i32),
        "sem_batch_plan": ([P(sem_block), i32, i32, P(sem_phys), u32, vp, P(vp)], i32),
        "sem_batch_execute": ([vp, vp], i32),
        "sem_plan_describe": ([vp, ctypes.c_char_p, i32], i32),
        "sem_plan_destroy": ([vp], i32),
        "sem_rk3_graph_create": ([P(sem_block), i32, i32, P(sem_phys), u32, vp, vp, vp, vp, i64, d,
                                  vp, P(vp)], i32),
        "sem_rk3_graph_launch": ([vp, vp], i32),
        "sem_rk3_graph_describe": ([vp, ctypes.c_char_p, i32], i32),
        "sem_rk3_graph_destroy": ([vp], i32),
        "sem_set_max_workgroups": ([i64], i32),
        "sem_surface_rhs": ([i32, i32, i32, vp, vp, vp, vp, P(sem_phys), vp, i32, vp], i32),
        "sem_batch_rhs_static": ([P(sem_block), i32, i32, P(sem_phys), vp], i32),
        "sem_rhs": ([i32, i32, i32, vp, vp, vp, vp, vp, vp, P(sem_phys), vp, i32, vp], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(status: int) -> None:
    if status != SEM_OK:
        raise SemError(status, lib().sem_last_error().decode(errors="replace"))


def version() -> str:
    return lib().sem_version().decode()


def set_max_workgroups(cap: int) -> None:
    """Process-wide cap on the workgroups of the strided (k-slice and
    t-column) launches; 0 restores one workgroup per tile."""
    _check(lib().sem_set_max_workgroups(int(cap)))


def tile_options(dtype: torch.dtype, Nq: int):
    """Compiled single-order tile shapes for (dtype, Nq) as
    ``[(elems_per_block, "full" | "alias"), ...]``."""
    buf = (sem_tile * 64)()
    n = lib().sem_tile_options(_code(dtype), Nq, buf, 64)
    names = {SEM_LAYOUT_FULL: "full", SEM_LAYOUT_ALIAS: "alias"}
    return [(buf[i].elems_per_block, names[buf[i].layout]) for i in range(min(n, 64))]


def _code(dtype: torch.dtype) -> int:
    if dtype == torch.float64:
        return SEM_F64
    if dtype == torch.float32:
        return SEM_F32
    raise TypeError(f"unsupported dtype {dtype} (float64 or float32)")


def _phys(phys) -> sem_phys:
    if phys is None:
        phys = (1.0e5, 1.4, 287.0, 9.81)
    if isinstance(phys, sem_phys):
        return phys
    if hasattr(phys, "as_tuple"):
        phys = phys.as_tuple()
    return sem_phys(*[float(x) for x in phys])


def _dev(t: Optional[torch.Tensor], name: str, dtype=None, shape=None) -> Optional[int]:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _shape(q: torch.Tensor, D: torch.Tensor):
    if q.dim() != 3 or q.shape[1] != 5:
        raise ValueError(f"q must be [Ne, 5, Nq^3], got {tuple(q.shape)}")
    Nq = D.shape[0]
    if D.dim() != 2 or D.shape[1] != Nq or q.shape[2] != Nq ** 3:
        raise ValueError(f"D [{tuple(D.shape)}] does not match q [{tuple(q.shape)}]")
    return q.shape[0], Nq


def volume_rhs(q, geo, D, rho_ref=None, theta_ref=None, phys=None, out=None, accumulate=False,
               elems_per_block: int = 0, layout: str = "default", stream=None) -> torch.Tensor:
    """Volume term of Eq. (volterm) plus the gravity source (``rhs = v(q)``,
    or ``out += v(q)`` with ``accumulate``).  ``elems_per_block``/``layout``
    pick a compiled tile shape (see :func:`tile_options`); every shape
    computes the same values."""
    Ne, Nq = _shape(q, D)
    M = Nq ** 3
    dt = q.dtype
    if out is None:
        out = torch.empty_like(q)
    args = (_dev(D, "D", dt), _dev(geo, "geo", dt, (Ne, 10, M)), _dev(q, "q", dt),
            _dev(rho_ref, "rho_ref", dt, (Ne, M)),
            _dev(theta_ref, "theta_ref", torch.float64, (Ne, M)))
    o = _dev(out, "out", dt, q.shape)
    ph = _phys(phys)
    if layout not in LAYOUTS:
        raise ValueError(f"layout must be one of {sorted(LAYOUTS)}")
    tile = sem_tile(int(elems_per_block), LAYOUTS[layout])
    _check(lib().sem_volume_rhs_tiled(Ne, Nq, _code(dt), *args, ctypes.byref(ph), o,
                                      int(bool(accumulate)), ctypes.byref(tile), _stream(stream)))
    return out


def volume_rhs_ext(q, geo, D, rho_ref=None, theta_ref=None, phys=None, dirs=7, out=None,
                   accumulate=False, stream=None) -> torch.Tensor:
    """Volume term with 5 or 8 fields (``q`` ``[Ne, nf, Nq^3]``, fields 5-7 the
    passive tracers) over the reference directions ``dirs`` (3 = r+s, the
    paper's benchmark kernel; 7 = r+s+t); Nq up to 16."""
    if q.dim() != 3 or q.shape[1] not in (5, 8):
        raise ValueError(f"q must be [Ne, 5 or 8, Nq^3], got {tuple(q.shape)}")
    Ne, nf = q.shape[0], q.shape[1]
    Nq = D.shape[0]
    M = Nq ** 3
    if D.dim() != 2 or D.shape[1] != Nq or q.shape[2] != M:
        raise ValueError(f"D [{tuple(D.shape)}] does not match q [{tuple(q.shape)}]")
    dt = q.dtype
    if out is None:
        out = torch.empty_like(q)
    ph = _phys(phys)
    _check(lib().sem_volume_rhs_ext(
        Ne, Nq, _code(dt), nf, int(dirs), _dev(D, "D", dt), _dev(geo, "geo", dt, (Ne, 10, M)),
        _dev(q, "q", dt), _dev(rho_ref, "rho_ref", dt, (Ne, M)),
        _dev(theta_ref, "theta_ref", torch.float64, (Ne, M)), ctypes.byref(ph),
        _dev(out, "out", dt, q.shape), int(bool(accumulate)), _stream(stream)))
    return out


LADDER_LEVELS = 6


def volume_rhs_ladder(level, q, geo, D, phys=None, out=None, stream=None) -> torch.Tensor:
    """The paper's benchmark kernel (FP32, 8 fields, r and s, no reference
    state, no source; ``out += v``) at optimisation level ``level`` (1 naive ..
    5, 6 = production kernel).  ``out`` is accumulated into (zeros if None)."""
    if q.dim() != 3 or q.shape[1] != 8:
        raise ValueError(f"q must be [Ne, 8, Nq^3], got {tuple(q.shape)}")
    Ne = q.shape[0]
    Nq = D.shape[0]
    M = Nq ** 3
    if D.dim() != 2 or D.shape[1] != Nq or q.shape[2] != M:
        raise ValueError(f"D [{tuple(D.shape)}] does not match q [{tuple(q.shape)}]")
    dt = torch.float32
    if out is None:
        out = torch.zeros_like(q)
    ph = _phys(phys)
    _check(lib().sem_volume_rhs_ladder(
        int(level), Ne, Nq, _dev(D, "D", dt), _dev(geo, "geo", dt, (Ne, 10, M)), _dev(q, "q", dt),
        ctypes.byref(ph), _dev(out, "out", dt, q.shape), _stream(stream)))
    return out


def volume_rhs_affine(q, geo_elem, D, rho_ref=None, theta_ref=None, phys=None, out=None,
                      accumulate=False, stream=None) -> torch.Tensor:
    """Volume term for affine elements: ``geo_elem`` ``[Ne, 10]`` holds the
    metric terms and 1/J once per element."""
    Ne, Nq = _shape(q, D)
    M = Nq ** 3
    dt = q.dtype
    if out is None:
        out = torch.empty_like(q)
    ph = _phys(phys)
    _check(lib().sem_volume_rhs_affine(
        Ne, Nq, _code(dt), _dev(D, "D", dt), _dev(geo_elem, "geo_elem", dt, (Ne, 10)),
        _dev(q, "q", dt), _dev(rho_ref, "rho_ref", dt, (Ne, M)),
        _dev(theta_ref, "theta_ref", torch.float64, (Ne, M)), ctypes.byref(ph),
        _dev(out, "out", dt, q.shape), int(bool(accumulate)), _stream(stream)))
    return out


def volume_rhs_adjoint(q, geo, D, lam, phys=None, out=None, accumulate=False,
                       stream=None) -> torch.Tensor:
    """Vector-Jacobian product ``(dv/dq)^T lam`` (the reference state drops out)."""
    Ne, Nq = _shape(q, D)
    M = Nq ** 3
    dt = q.dtype
    if out is None:
        out = torch.empty_like(q)
    ph = _phys(phys)
    _check(lib().sem_volume_rhs_adjoint(
        Ne, Nq, _code(dt), _dev(D, "D", dt), _dev(geo, "geo", dt, (Ne, 10, M)), _dev(q, "q", dt),
        ctypes.byref(ph), _dev(lam, "lam", dt, q.shape), _dev(out, "out", dt, q.shape),
        int(bool(accumulate)), _stream(stream)))
    return out


def surface_rhs(q, geo, nbr, theta_ref=None, phys=None, out=None, accumulate=False,
                stream=None) -> torch.Tensor:
    """Surface term s of ``dq/dt = v + s`` (``out = s``, or ``out += s`` with
    ``accumulate``): ``nbr`` is an int32 ``[Ne, 6]`` tensor of the elements
    across the faces r-, r+, s-, s+, t-, t+ (an index outside ``[0, Ne)`` is a
    boundary face that adds nothing)."""
    if q.dim() != 3 or q.shape[1] != 5:
        raise ValueError(f"q must be [Ne, 5, Nq^3], got {tuple(q.shape)}")
    Ne, M = q.shape[0], q.shape[2]
    Nq = round(M ** (1.0 / 3.0))
    if Nq ** 3 != M:
        raise ValueError(f"q's node count {M} is not a cube")
    dt = q.dtype
    if out is None:
        out = torch.empty_like(q)
    ph = _phys(phys)
    _check(lib().sem_surface_rhs(
        Ne, Nq, _code(dt), _dev(nbr, "nbr", torch.int32, (Ne, 6)),
        _dev(geo, "geo", dt, (Ne, 10, M)), _dev(q, "q", dt),
        _dev(theta_ref, "theta_ref", torch.float64, (Ne, M)), ctypes.byref(ph),
        _dev(out, "out", dt, q.shape), int(bool(accumulate)), _stream(stream)))
    return out


def rhs(q, geo, D, nbr, rho_ref=None, theta_ref=None, phys=None, out=None, accumulate=False,
        stream=None) -> torch.Tensor:
    """The whole rate ``v(q) + s(q)`` (volume and surface term, Sec. 2) in one
    launch: ``out = v + s`` or ``out += v + s``; ``nbr`` ``[Ne, 6]`` int32 as
    for :func:`surface_rhs`."""
    Ne, Nq = _shape(q, D)
    M = Nq ** 3
    dt = q.dtype
    if out is None:
        out = torch.empty_like(q)
    ph = _phys(phys)
    _check(lib().sem_rhs(Ne, Nq, _code(dt), _dev(D, "D", dt), _dev(geo, "geo", dt, (Ne, 10, M)),
                         _dev(q, "q", dt), _dev(rho_ref, "rho_ref", dt, (Ne, M)),
                         _dev(theta_ref, "theta_ref", torch.float64, (Ne, M)),
                         _dev(nbr, "nbr", torch.int32, (Ne, 6)), ctypes.byref(ph),
                         _dev(out, "out", dt, q.shape), int(bool(accumulate)), _stream(stream)))
    return out


def axpby(a: float, x, b: float, y, c: float, z, out=None, stream=None) -> torch.Tensor:
    """``out = a*x + b*(y + c*z)`` elementwise (x may be None when a == 0)."""
    if out is None:
        out = torch.empty_like(y)
    n = y.numel()
    dt = y.dtype
    for t, nm in ((z, "z"), (out, "out")) + (((x, "x"),) if x is not None else ()):
        if t.numel() != n:
            raise ValueError(f"{nm} has {t.numel()} values, expected {n}")
    _check(lib().sem_axpby(n, _code(dt), float(a), _dev(x, "x", dt), float(b), _dev(y, "y", dt),
                           float(c), _dev(z, "z", dt), _dev(out, "out", dt), _stream(stream)))
    return out


class VolumeRHS(torch.autograd.Function):
    """``v(q)`` with a hand-written backward: ``grad_q = (dv/dq)^T grad_v``.

    ``VolumeRHS.apply(q, geo, D, rho_ref, theta_ref, phys_tuple)``; only q is
    differentiated (geo, D and the reference state are data)."""

    @staticmethod
    def forward(ctx, q, geo, D, rho_ref=None, theta_ref=None, phys=None):
        ctx.save_for_backward(q, geo, D)
        ctx.phys = phys
        return volume_rhs(q, geo, D, rho_ref, theta_ref, phys)

    @staticmethod
    def backward(ctx, grad):
        q, geo, D = ctx.saved_tensors
        g = volume_rhs_adjoint(q, geo, D, grad.contiguous(), ctx.phys)
        return g, None, None, None, None, None


def _block_dtype(blocks: Sequence[dict]) -> torch.dtype:
    if not blocks:
        raise ValueError("at least one block is required")
    return blocks[0]["q"].dtype


def _blocks(blocks: Sequence[dict], dtype: torch.dtype):
    arr = (sem_block * len(blocks))()
    keep = []
    for i, b in enumerate(blocks):
        q, D = b["q"], b["D"]
        Ne, Nq = _shape(q, D)
        M = Nq ** 3
        arr[i] = sem_block(Nq, Ne, _dev(D, "D", dtype), _dev(b["geo"], "geo", dtype, (Ne, 10, M)),
                           _dev(q, "q", dtype), _dev(b.get("rho_ref"), "rho_ref", dtype, (Ne, M)),
                           _dev(b.get("theta_ref"), "theta_ref", torch.float64, (Ne, M)),
                           _dev(b["rhs"], "rhs", dtype, q.shape))
        keep.append(b)
    return arr, keep


class BatchPlan:
    """Mixed-order batch: ``blocks`` is a list of dicts with tensors ``q``,
    ``geo``, ``D``, ``rhs`` and optional ``rho_ref``/``theta_ref``; every
    block may have its own order.  ``execute()`` is one kernel launch."""

    def __init__(self, blocks: Sequence[dict], phys=None, autotune: bool = False,
                 use_cache: bool = False, stream=None):
        self.dtype = _block_dtype(blocks)
        arr, self._keep = _blocks(blocks, self.dtype)
        self._phys = _phys(phys)
        flags = (SEM_PLAN_AUTOTUNE if autotune else 0) | (SEM_PLAN_USE_CACHE if use_cache else 0)
        h = ctypes.c_void_p()
        _check(lib().sem_batch_plan(arr, len(blocks), _code(self.dtype), ctypes.byref(self._phys),
                                    flags, _stream(stream), ctypes.byref(h)))
        self._h = h

    def execute(self, stream=None) -> None:
        _check(lib().sem_batch_execute(self._h, _stream(stream)))

    def describe(self) -> dict:
        buf = ctypes.create_string_buffer(8192)
        _check(lib().sem_plan_describe(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            _check(lib().sem_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_rhs_static(blocks: Sequence[dict], phys=None, stream=None) -> None:
    """The mixed-order batch of ``BatchPlan(blocks).execute()`` (built-in
    tile shapes) in one call that allocates no device memory; ``blocks`` as
    for ``BatchPlan``, every block's ``rhs`` overwritten."""
    dtype = _block_dtype(blocks)
    arr, _ = _blocks(blocks, dtype)
    ph = _phys(phys)
    _check(lib().sem_batch_rhs_static(arr, len(blocks), _code(dtype), ctypes.byref(ph),
                                      _stream(stream)))


class RK3Graph:
    """One SSP-RK3 step of ``dq/dt = v(q)`` captured in a HIP graph.

    ``q_n``, ``q_1``, ``q_2``, ``L`` are flat buffers of equal length; every
    block's ``q`` is a view into ``q_n`` and its ``rhs`` the view at the same
    offset in ``L``.  ``step()`` advances ``q_n`` in place by ``dt``.  By
    default each stage is one launch whose epilogue writes the stage update;
    ``separate_stages=True`` writes the rate into ``L`` and applies an axpby."""

    def __init__(self, blocks: Sequence[dict], q_n, q_1, q_2, L, dt: float, phys=None,
                 autotune: bool = False, use_cache: bool = False, separate_stages: bool = False,
                 stream=None):
        self.dtype = q_n.dtype
        arr, self._keep = _blocks(blocks, self.dtype)
        self._bufs = (q_n, q_1, q_2, L)
        n = q_n.numel()
        for t, nm in zip(self._bufs, ("q_n", "q_1", "q_2", "L")):
            _dev(t, nm, self.dtype)
            if t.numel() != n:
                raise ValueError(f"{nm} has {t.numel()} values, expected {n}")
        self._phys = _phys(phys)
        flags = ((SEM_PLAN_AUTOTUNE if autotune else 0) | (SEM_PLAN_USE_CACHE if use_cache else 0)
                 | (SEM_RK3_SEPARATE_STAGES if separate_stages else 0))
        h = ctypes.c_void_p()
        _check(lib().sem_rk3_graph_create(arr, len(blocks), _code(self.dtype),
                                          ctypes.byref(self._phys), flags, q_n.data_ptr(),
                                          q_1.data_ptr(), q_2.data_ptr(), L.data_ptr(), n, float(dt),
                                          _stream(stream), ctypes.byref(h)))
        self._h = h

    def step(self, stream=None) -> None:
        _check(lib().sem_rk3_graph_launch(self._h, _stream(stream)))

    def describe(self) -> dict:
        buf = ctypes.create_string_buffer(8192)
        _check(lib().sem_rk3_graph_describe(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            _check(lib().sem_rk3_graph_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
