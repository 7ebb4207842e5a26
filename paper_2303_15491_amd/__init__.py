"""MI355X (gfx950) piecewise-linear Morse-Smale segmentation.

Python binding of ``libplmss.so`` (C ABI in ``include/plmss.h``).  This module
only marshals arguments: torch provides device memory and the current HIP
stream, every step of the segmentation runs in the library's HIP kernels.
There is no CPU fallback; without the built library every call raises.

Method: Maack et al., "Parallel Computation of Piecewise Linear Morse-Smale
Segmentations", arXiv 2303.15491, Sec. "Method".
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["PlmssError", "library", "segment", "segment_static", "STATIC_MAX_VERTICES", "order_field", "steepest", "compress", "ms_ids",
           "segment_batch", "workspace_bytes", "batch_workspace_bytes", "batch_needs", "Plan",
           "tune_get", "tune_set", "KNOBS", "marching_rows", "marching_index", "marching_geometry", "marching_geometry_union", "MARCH_SEPARATORS",
           "MARCH_BOUNDARIES"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libplmss.so")

OK, E_ARG, E_DIMS, E_TOO_LARGE, E_NAN, E_WORKSPACE, E_HIP, E_NOCONV, E_INTERNAL = 0, -1, -2, -3, -4, -5, -6, -7, -8
F32, F64 = 0, 1
MARCH_SEPARATORS, MARCH_BOUNDARIES = 0, 1
STATIC_MAX_VERTICES = 1 << 21  # PLMSS_STATIC_MAX_VERTICES


class PlmssError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        msg = _lib_status(code)
        super().__init__(f"{what}: {msg} (status {code})" if what else f"{msg} (status {code})")
        self.code = code


class Dims(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64)]


class Job(ctypes.Structure):
    _fields_ = [("field", ctypes.c_void_p), ("dims", Dims), ("dtype", ctypes.c_int32),
                ("asc", ctypes.c_void_p), ("desc", ctypes.c_void_p), ("ms", ctypes.c_void_p),
                ("order", ctypes.c_void_p), ("info", ctypes.c_void_p)]


_lib = None

_SIGNATURES = {
    "plmss_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "plmss_build_info": ([], ctypes.c_char_p),
    "plmss_workspace_bytes": ([Dims, ctypes.c_int32, ctypes.c_int32], ctypes.c_size_t),
    "plmss_segment": ([ctypes.POINTER(Job), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "plmss_static_scratch_bytes": ([], ctypes.c_size_t),
    "plmss_segment_static": ([ctypes.POINTER(Job), ctypes.c_void_p], ctypes.c_int),
    "plmss_order_workspace_bytes": ([Dims, ctypes.c_int32], ctypes.c_size_t),
    "plmss_order_field": ([ctypes.c_void_p, Dims, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                           ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "plmss_steepest": ([ctypes.c_void_p, ctypes.c_void_p, Dims, ctypes.c_int32, ctypes.c_void_p,
                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "plmss_compress": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p], ctypes.c_int),
    "plmss_ms_workspace_bytes": ([ctypes.c_int64], ctypes.c_size_t),
    "plmss_ms_ids": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "plmss_marching_rows": ([Dims], ctypes.c_int64),
    "plmss_marching_workspace_bytes": ([Dims], ctypes.c_size_t),
    "plmss_marching_index": ([ctypes.c_void_p, Dims, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                              ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "plmss_marching_geometry": ([ctypes.c_void_p, Dims, ctypes.c_int32, ctypes.c_void_p, ctypes.c_uint64,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "plmss_batch_workspace_bytes": ([ctypes.c_int32, ctypes.POINTER(Job)], ctypes.c_size_t),
    "plmss_segment_batch": ([ctypes.c_int32, ctypes.POINTER(Job), ctypes.c_void_p, ctypes.c_size_t,
                             ctypes.c_void_p], ctypes.c_int),
    "plmss_batch_needs": ([ctypes.c_int32, ctypes.POINTER(Job), ctypes.POINTER(ctypes.c_int64)], ctypes.c_int32),
    "plmss_plan_create": ([ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                           ctypes.c_int32], ctypes.c_void_p),
    "plmss_plan_destroy": ([ctypes.c_void_p], None),
    "plmss_plan_workspace_bytes": ([ctypes.c_void_p], ctypes.c_size_t),
    "plmss_plan_set": ([ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Job), ctypes.c_void_p, ctypes.c_size_t,
                        ctypes.c_void_p], ctypes.c_int),
    "plmss_plan_launch": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "plmss_plan_launch_graph": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "plmss_trace_create": ([ctypes.c_int32], ctypes.c_void_p),
    "plmss_trace_destroy": ([ctypes.c_void_p], None),
    "plmss_trace_begin": ([ctypes.c_void_p], ctypes.c_int),
    "plmss_trace_end": ([ctypes.c_void_p], ctypes.c_int),
    "plmss_trace_read": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float),
                          ctypes.c_int32], ctypes.c_int32),
    "plmss_kernel_name": ([ctypes.c_int32], ctypes.c_char_p),
    "plmss_tune_set": ([ctypes.c_int32, ctypes.c_int64], ctypes.c_int32),
    "plmss_tune_get": ([ctypes.c_int32], ctypes.c_int64),
}

# Launch-shape knobs (plmss_tune_*): name -> id.
KNOBS = {"order_workers": 0, "order_invert": 1, "sort_workers": 2, "persist_blocks": 3, "scan_depth": 4,
         "order_packed": 5, "scan_rounds": 6, "order_concurrent": 7,
         "packed_codes": 8, "pair_stream": 9}


def library():
    """The loaded ``libplmss.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PlmssError(E_HIP, f"{LIB_PATH} is missing; build it with "
                                    "`python -m paper_2303_15491_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _lib_status(code: int) -> str:
    try:
        return library().plmss_status_string(code).decode()
    except Exception:  # the library itself may be what is missing
        return "status"


def _check(rc: int, what: str):
    if rc != OK:
        raise PlmssError(rc, what)


def tune_set(**values):
    """Sets launch-shape knobs by name (see ``KNOBS``); results never change."""
    lib = library()
    for name, v in values.items():
        if name not in KNOBS:
            raise KeyError(name)
        _check(lib.plmss_tune_set(KNOBS[name], int(v)), f"plmss_tune_set({name}={v})")


def tune_get() -> dict:
    """Current value of every launch-shape knob."""
    lib = library()
    return {name: int(lib.plmss_tune_get(k)) for name, k in KNOBS.items()}


def _torch():
    import torch

    return torch


def dims_of(shape) -> Dims:
    """Grid dims of an (nz, ny, nx), (ny, nx) or (nx,) shaped field."""
    shape = tuple(int(s) for s in shape)
    if len(shape) == 1:
        return Dims(shape[0], 1, 1)
    if len(shape) == 2:
        return Dims(shape[1], shape[0], 1)
    if len(shape) == 3:
        return Dims(shape[2], shape[1], shape[0])
    raise ValueError("a field must be 1-, 2- or 3-dimensional")


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError("field must be float32 or float64")


def _field_check(field):
    if not field.is_cuda:
        raise ValueError("field must be a device tensor")
    if not field.is_contiguous():
        raise ValueError("field must be C-contiguous")
    return _dtype_code(field)


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _workspace(nbytes: int, device, workspace=None):
    torch = _torch()
    if workspace is not None:
        if workspace.numel() * workspace.element_size() < nbytes:
            raise PlmssError(E_WORKSPACE, "workspace")
        return workspace
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def workspace_bytes(shape, dtype=None, with_order: bool = False) -> int:
    torch = _torch()
    code = F64 if dtype == torch.float64 else F32
    return int(library().plmss_workspace_bytes(dims_of(shape), code, int(with_order)))


def segment(field, with_order: bool = False, workspace=None, stream=None, out=None):
    """Morse-Smale segmentation of one device field.

    Returns a dict of int32 device tensors of the field's shape: ``asc``,
    ``desc``, ``ms`` (and ``order`` when ``with_order``), plus ``info``, an
    int32 device tensor {status, #minima, #maxima, K}.  Asynchronous on the
    current stream; read ``info`` to learn K or a NaN error.
    """
    torch = _torch()
    code = _field_check(field)
    dims = dims_of(field.shape)
    dev = field.device
    if out is None:
        out = {k: torch.empty(field.shape, dtype=torch.int32, device=dev) for k in ("asc", "desc", "ms")}
        if with_order:
            out["order"] = torch.empty(field.shape, dtype=torch.int32, device=dev)
        out["info"] = torch.empty(4, dtype=torch.int32, device=dev)
    _check_outs(field, out, with_order)
    lib = library()
    ws = _workspace(lib.plmss_workspace_bytes(dims, code, int(with_order)), dev, workspace)
    job = Job(field.data_ptr(), dims, code, out["asc"].data_ptr(), out["desc"].data_ptr(),
              out["ms"].data_ptr(), out["order"].data_ptr() if with_order else None,
              out["info"].data_ptr())
    _check(lib.plmss_segment(ctypes.byref(job), _ptr(ws), ws.numel(), _stream(stream)), "plmss_segment")
    return out


def _check_outs(field, out, with_order, what="output"):
    """Outputs a kernel writes must hold exactly the field's vertices as
    contiguous int32 device tensors (info: 4 entries); anything else would be
    written past its end."""
    torch = _torch()
    for k in ("asc", "desc", "ms") + (("order",) if with_order else ()):
        t = out.get(k)
        if t is None and k == "order":
            raise ValueError("with_order needs an order tensor in out")
        if (t is None or not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous()
                or t.numel() != field.numel()):
            raise ValueError(f"{what} {k} must be a contiguous int32 device tensor of the field's size")
    info = out.get("info")
    if info is None or not info.is_cuda or info.dtype != torch.int32 or not info.is_contiguous() \
            or info.numel() < 4:
        raise ValueError(f"{what} info must be a contiguous int32 device tensor of 4 entries")


def _segment_outs(field, with_order):
    torch = _torch()
    out = {k: torch.empty(field.shape, dtype=torch.int32, device=field.device) for k in ("asc", "desc", "ms")}
    if with_order:
        out["order"] = torch.empty(field.shape, dtype=torch.int32, device=field.device)
    out["info"] = torch.empty(4, dtype=torch.int32, device=field.device)
    return out


def segment_static(field, with_order: bool = False, stream=None, out=None):
    """:func:`segment` without a workspace: the library's own per-GPU scratch
    array is used (``plmss_segment_static``), so nothing is allocated but the
    outputs (none at all when ``out`` is given).  Fields of at most
    ``STATIC_MAX_VERTICES`` vertices; calls that overlap on one GPU race."""
    code = _field_check(field)
    if out is None:
        out = _segment_outs(field, with_order)
    _check_outs(field, out, with_order)
    job = Job(field.data_ptr(), dims_of(field.shape), code, out["asc"].data_ptr(), out["desc"].data_ptr(),
              out["ms"].data_ptr(), out["order"].data_ptr() if with_order else None,
              out["info"].data_ptr())
    _check(library().plmss_segment_static(ctypes.byref(job), _stream(stream)), "plmss_segment_static")
    return out


def order_field(field, workspace=None, stream=None):
    """Simulation-of-Simplicity order field (int32 device tensor) and info."""
    torch = _torch()
    code = _field_check(field)
    dims = dims_of(field.shape)
    lib = library()
    order = torch.empty(field.shape, dtype=torch.int32, device=field.device)
    info = torch.empty(4, dtype=torch.int32, device=field.device)
    ws = _workspace(lib.plmss_order_workspace_bytes(dims, code), field.device, workspace)
    _check(lib.plmss_order_field(_ptr(field), dims, code, _ptr(order), _ptr(info), _ptr(ws), ws.numel(),
                                 _stream(stream)), "plmss_order_field")
    return order, info


def steepest(field=None, order=None, stream=None):
    """Steepest ascending/descending neighbours (up, dn, info) from a float
    field or from a materialised order field."""
    torch = _torch()
    src = order if order is not None else field
    if src is None:
        raise ValueError("need a field or an order field")
    if not src.is_cuda or not src.is_contiguous():
        raise ValueError("input must be a contiguous device tensor")
    code = F32
    if order is None:
        code = _field_check(field)
    elif order.dtype != torch.int32:
        raise TypeError("order must be int32")
    up = torch.empty(src.shape, dtype=torch.int32, device=src.device)
    dn = torch.empty(src.shape, dtype=torch.int32, device=src.device)
    info = torch.empty(4, dtype=torch.int32, device=src.device)
    _check(library().plmss_steepest(_ptr(field) if order is None else None, _ptr(order), dims_of(src.shape), code,
                                    _ptr(up), _ptr(dn), _ptr(info), _stream(stream)), "plmss_steepest")
    return up, dn, info


def compress(desc, asc, stream=None):
    """Path compression in place: on entry up/dn pointers, on return labels."""
    torch = _torch()
    for t in (desc, asc):
        if not t.is_cuda or not t.is_contiguous() or t.dtype != torch.int32:
            raise ValueError("pointer arrays must be contiguous int32 device tensors")
    if desc.numel() != asc.numel():
        raise ValueError("size mismatch")
    _check(library().plmss_compress(_ptr(desc), _ptr(asc), desc.numel(), _stream(stream)), "plmss_compress")
    return desc, asc


def ms_ids(asc, desc, workspace=None, stream=None):
    """MS region ids (int32 device tensor) and info from asc/desc labels."""
    torch = _torch()
    for t in (desc, asc):
        if not t.is_cuda or not t.is_contiguous() or t.dtype != torch.int32:
            raise ValueError("label arrays must be contiguous int32 device tensors")
    n = asc.numel()
    lib = library()
    ms = torch.empty(asc.shape, dtype=torch.int32, device=asc.device)
    info = torch.empty(4, dtype=torch.int32, device=asc.device)
    ws = _workspace(lib.plmss_ms_workspace_bytes(n), asc.device, workspace)
    _check(lib.plmss_ms_ids(_ptr(asc), _ptr(desc), n, _ptr(ms), _ptr(info), _ptr(ws), ws.numel(),
                            _stream(stream)), "plmss_ms_ids")
    return ms, info


def marching_rows(shape) -> int:
    """Rows of cells of a grid: (ny-1)(nz-1) rows of cubes, ny-1 rows of
    squares for nz == 1, 0 for grids without cells."""
    return int(library().plmss_marching_rows(dims_of(shape)))


def marching_index(labels, mode: int = MARCH_SEPARATORS, with_codes: bool = False, workspace=None,
                   stream=None, out=None):
    """Multi-label marching index of an int32 device label field.

    Returns ``(codes, row_offsets)``: ``codes`` a uint8 device tensor of
    rows * (nx-1) * C cell codes (C = 6 tetrahedra per cube, 2 triangles per
    square), or None without ``with_codes``; ``row_offsets`` an int64 device
    tensor of rows + 1 exclusive primitive offsets, the last being the total.
    ``mode`` is MARCH_SEPARATORS or MARCH_BOUNDARIES.  ``out`` may pass
    ``(codes, row_offsets)`` tensors to fill.
    """
    torch = _torch()
    if not labels.is_cuda or not labels.is_contiguous() or labels.dtype != torch.int32:
        raise ValueError("labels must be a contiguous int32 device tensor")
    dims = dims_of(labels.shape)
    lib = library()
    rows = int(lib.plmss_marching_rows(dims))
    if rows < 0:
        raise PlmssError(E_DIMS, "plmss_marching_rows")
    cells = rows * max(int(dims.nx) - 1, 0) * (6 if dims.nz > 1 else 2)
    if out is not None:
        codes, offs = out
        if offs.dtype != torch.int64 or offs.numel() < rows + 1 or not offs.is_contiguous():
            raise ValueError("row_offsets must be a contiguous int64 tensor of rows + 1 entries")
        if codes is not None and (codes.dtype != torch.uint8 or codes.numel() < cells
                                  or not codes.is_contiguous()):
            raise ValueError("codes must be a contiguous uint8 tensor of one byte per cell")
    else:
        offs = torch.empty(rows + 1, dtype=torch.int64, device=labels.device)
        codes = torch.empty(max(cells, 1), dtype=torch.uint8, device=labels.device) if with_codes else None
    ws = _workspace(lib.plmss_marching_workspace_bytes(dims), labels.device, workspace)
    _check(lib.plmss_marching_index(_ptr(labels), dims, int(mode), _ptr(codes), _ptr(offs), _ptr(ws), ws.numel(),
                                    _stream(stream)), "plmss_marching_index")
    return (codes[:cells] if codes is not None else None), offs


def marching_geometry(labels, mode: int = MARCH_SEPARATORS, with_xyz: bool = True, with_sides: bool = True,
                      row_offsets=None, stream=None, out=None):
    """Multi-label marching geometry of an int32 device label field.

    Returns ``(xyz, sides, count)``: ``xyz`` a float32 device tensor of shape
    (count, 3, 3) triangles in 3-D or (count, 2, 2) segments in 2-D (grid
    units), ``sides`` an int32 (count, 2) tensor of the labels each primitive
    separates (either None when not asked for).  ``row_offsets`` is
    :func:`marching_index`'s output for the same labels and mode; without it
    the index runs first.  Reading the total synchronises with the device
    unless ``out=(xyz, sides, count)`` supplies the outputs and their
    capacity.
    """
    torch = _torch()
    if not labels.is_cuda or not labels.is_contiguous() or labels.dtype != torch.int32:
        raise ValueError("labels must be a contiguous int32 device tensor")
    dims = dims_of(labels.shape)
    three = dims.nz > 1
    pts = (3, 3) if three else (2, 2)
    rows = int(library().plmss_marching_rows(dims))
    if rows < 0:
        raise PlmssError(E_DIMS, "plmss_marching_rows")
    if row_offsets is None:
        _, row_offsets = marching_index(labels, mode, with_codes=False, stream=stream)
    elif (not row_offsets.is_cuda or row_offsets.dtype != torch.int64 or not row_offsets.is_contiguous()
          or row_offsets.numel() < rows + 1):
        raise ValueError("row_offsets must be a contiguous int64 device tensor of rows + 1 entries")
    if out is not None:
        xyz, sides, count = out
        count = int(count)
        if count < 0:
            raise ValueError("count (the output capacity) must be >= 0")
        per_xyz = pts[0] * pts[1]
        for name, t, dt, per in (("xyz", xyz, torch.float32, per_xyz), ("sides", sides, torch.int32, 2)):
            if t is None:
                continue
            if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {dt} device tensor")
            if t.numel() < count * per:
                raise ValueError(f"{name} holds {t.numel()} elements, fewer than {count} primitives need "
                                 f"({count * per})")
    else:
        count = int(row_offsets[-1].item())
        xyz = torch.empty((max(count, 1),) + pts, dtype=torch.float32, device=labels.device) if with_xyz else None
        sides = torch.empty((max(count, 1), 2), dtype=torch.int32, device=labels.device) if with_sides else None
    _check(library().plmss_marching_geometry(_ptr(labels), dims, int(mode), _ptr(row_offsets), count, _ptr(xyz),
                                             _ptr(sides), _stream(stream)), "plmss_marching_geometry")
    return (xyz[:count] if xyz is not None else None), (sides[:count] if sides is not None else None), count


def marching_geometry_union(asc, desc, mode: int = MARCH_SEPARATORS, stream=None):
    """Geometry of the union of the ascending and descending segmentations
    (Sec. "Triangulation Options"): the primitives of ``asc`` followed by
    those of ``desc``, where the two surfaces meet they intersect.  Returns
    ``(xyz, sides, count_asc, count_desc)``; each half is one
    :func:`marching_geometry` call written into its part of one output."""
    torch = _torch()
    offs = [marching_index(t, mode, stream=stream)[1] for t in (asc, desc)]
    counts = [int(o[-1].item()) for o in offs]
    dims = dims_of(asc.shape)
    pts = (3, 3) if dims.nz > 1 else (2, 2)
    total = counts[0] + counts[1]
    xyz = torch.empty((max(total, 1),) + pts, dtype=torch.float32, device=asc.device)
    sides = torch.empty((max(total, 1), 2), dtype=torch.int32, device=asc.device)
    start = 0
    for t, o, c in zip((asc, desc), offs, counts):
        if c:
            marching_geometry(t, mode, row_offsets=o, stream=stream, out=(xyz[start:start + c], sides[start:start + c], c))
        start += c
    return xyz[:total], sides[:total], counts[0], counts[1]


def _jobs(fields, outs):
    torch = _torch()
    arr = (Job * len(fields))()
    for i, (f, o) in enumerate(zip(fields, outs)):
        for k in ("asc", "desc", "ms", "order"):
            t = o.get(k)
            if t is None and k == "order":
                continue
            if (t is None or not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous()
                    or t.numel() != f.numel()):
                raise ValueError(f"output {k} of field {i} must be a contiguous int32 device tensor of its size")
        info = o.get("info")
        if info is not None and (not info.is_cuda or info.dtype != torch.int32 or not info.is_contiguous()
                                 or info.numel() < 4):
            raise ValueError(f"info of field {i} must be a contiguous int32 device tensor of 4 entries")
        order = o.get("order")
        arr[i] = Job(f.data_ptr(), dims_of(f.shape), _dtype_code(f), o["asc"].data_ptr(), o["desc"].data_ptr(),
                     o["ms"].data_ptr(), order.data_ptr() if order is not None else None,
                     info.data_ptr() if info is not None else None)
    return arr


def _outs_for(fields, with_order=False):
    torch = _torch()
    outs = []
    for f in fields:
        o = {k: torch.empty(f.shape, dtype=torch.int32, device=f.device) for k in ("asc", "desc", "ms")}
        if with_order:
            o["order"] = torch.empty(f.shape, dtype=torch.int32, device=f.device)
        o["info"] = torch.empty(4, dtype=torch.int32, device=f.device)
        outs.append(o)
    return outs


def batch_needs(fields):
    """(vertices, fields, scan tiles, chase tiles) a batch needs from a Plan."""
    arr = (Job * len(fields))()
    for i, f in enumerate(fields):
        arr[i] = Job(1, dims_of(f.shape), _dtype_code(f), 1, 1, 1, None, None)
    needs = (ctypes.c_int64 * 4)()
    _check(library().plmss_batch_needs(len(fields), arr, needs), "plmss_batch_needs")
    return tuple(int(v) for v in needs)


def batch_workspace_bytes(fields) -> int:
    arr = (Job * len(fields))()
    for i, f in enumerate(fields):
        arr[i] = Job(1, dims_of(f.shape), _dtype_code(f), 1, 1, 1, None, None)
    return int(library().plmss_batch_workspace_bytes(len(fields), arr))


def segment_batch(fields, with_order: bool = False, workspace=None, stream=None, outs=None):
    """Segment many device fields of any sizes in one pass; returns one dict
    per field as :func:`segment` does (with ``order`` when ``with_order``;
    given ``outs``, the fields whose dict holds an ``order`` tensor get it)."""
    for f in fields:
        _field_check(f)
    if outs is None:
        outs = _outs_for(fields, with_order)
    arr = _jobs(fields, outs)
    lib = library()
    nbytes = lib.plmss_batch_workspace_bytes(len(fields), arr)
    if nbytes == 0:
        raise PlmssError(E_ARG, "plmss_batch_workspace_bytes")
    ws = _workspace(nbytes, fields[0].device, workspace)
    _check(lib.plmss_segment_batch(len(fields), arr, _ptr(ws), ws.numel(), _stream(stream)), "plmss_segment_batch")
    return outs


class Plan:
    """A capacity plan: batches of up to the given totals, launched through one
    replayable hipGraph (see ``plmss_plan_*`` in plmss.h)."""

    def __init__(self, max_vertices: int, max_fields: int, max_scan_tiles: int, max_chase_tiles: int,
                 dtype=None, device="cuda", with_order: bool = False):
        torch = _torch()
        code = F64 if dtype == torch.float64 else F32
        self._lib = library()
        self.with_order = bool(with_order)
        self._h = self._lib.plmss_plan_create(int(max_vertices), int(max_fields), int(max_scan_tiles),
                                              int(max_chase_tiles), code, int(self.with_order))
        if not self._h:
            raise PlmssError(E_ARG, "plmss_plan_create")
        nbytes = self._lib.plmss_plan_workspace_bytes(self._h)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self._jobs = None

    def set(self, fields, outs=None, stream=None):
        """Points the plan at a batch; returns the output dicts (with an
        ``order`` tensor each when the plan builds order fields)."""
        for f in fields:
            _field_check(f)
        if outs is None:
            outs = _outs_for(fields, self.with_order)
        self._jobs = _jobs(fields, outs)  # kept alive with the tables
        self._fields, self._outs = fields, outs
        _check(self._lib.plmss_plan_set(self._h, len(fields), self._jobs, _ptr(self.workspace),
                                        self.workspace.numel(), _stream(stream)), "plmss_plan_set")
        return outs

    def launch(self, graph: bool = True, stream=None):
        fn = self._lib.plmss_plan_launch_graph if graph else self._lib.plmss_plan_launch
        _check(fn(self._h, _ptr(self.workspace), self.workspace.numel(), _stream(stream)), "plmss_plan_launch")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.plmss_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
