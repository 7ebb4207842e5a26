"""Serial CPU oracle for the piecewise-linear Morse-Smale segmentation.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It is the plain
definition of what the GPU library computes (Maack et al., arXiv 2303.15491,
Sec. "Method"), written in serial C (``plmss_oracle.c``) and shares no code
with the GPU library.

Every function takes and returns numpy arrays; fields are C-contiguous with
shape ``(nz, ny, nx)`` (or ``(ny, nx)``, ``(nx,)``), so that vertex id
``v = x + nx*(y + ny*z)`` is the flat index.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "plmss_oracle.c")
_LIB = os.path.join(_HERE, "libplmss_oracle.so")

OK, E_ARG, E_DIMS, E_TOO_LARGE, E_NAN, E_NOMEM = 0, -1, -2, -3, -4, -7


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/libplmss_oracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        i64, i32p, i64p, vp = ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p
        lib.plmss_oracle_order.argtypes = [vp, ctypes.c_int, i64, i64, i64, vp, vp]
        lib.plmss_oracle_steepest.argtypes = [vp, i64, i64, i64, vp, vp]
        lib.plmss_oracle_labels.argtypes = [vp, vp, vp, i64, vp, vp]
        lib.plmss_oracle_ms.argtypes = [vp, vp, i64, vp, vp]
        lib.plmss_oracle_segment.argtypes = [vp, ctypes.c_int, i64, i64, i64, vp, vp, vp, vp, vp, vp, vp]
        lib.plmss_oracle_trace.argtypes = [vp, ctypes.c_int, i64, i64, i64, i64, vp, vp, vp, vp]
        lib.plmss_oracle_compress.argtypes = [vp, i64, ctypes.c_int, vp, i64]
        lib.plmss_oracle_compress.restype = ctypes.c_int64
        lib.plmss_oracle_degree_sum.argtypes = [i64, i64, i64]
        lib.plmss_oracle_degree_sum.restype = ctypes.c_int64
        lib.plmss_oracle_neighbours.argtypes = [i64, i64, i64, i64, vp]
        lib.plmss_oracle_marching_rows.argtypes = [i64, i64, i64]
        lib.plmss_oracle_marching_rows.restype = ctypes.c_int64
        lib.plmss_oracle_marching.argtypes = [vp, i64, i64, i64, ctypes.c_int, vp, vp]
        lib.plmss_oracle_marching_geometry.argtypes = [vp, i64, i64, i64, ctypes.c_int, vp, vp, i64]
        lib.plmss_oracle_marching_geometry.restype = ctypes.c_int64
        for name in ("plmss_oracle_order", "plmss_oracle_steepest", "plmss_oracle_labels",
                     "plmss_oracle_ms", "plmss_oracle_segment", "plmss_oracle_trace",
                     "plmss_oracle_neighbours", "plmss_oracle_marching"):
            getattr(lib, name).restype = ctypes.c_int
        del i32p, i64p
        _lib = lib
    return _lib


def _dims(field: np.ndarray):
    if field.ndim == 1:
        return field.shape[0], 1, 1
    if field.ndim == 2:
        return field.shape[1], field.shape[0], 1
    if field.ndim == 3:
        return field.shape[2], field.shape[1], field.shape[0]
    raise ValueError("field must be 1-, 2- or 3-dimensional")


def _prep(field: np.ndarray):
    field = np.asarray(field)
    if field.dtype == np.float32:
        dt = 0
    elif field.dtype == np.float64:
        dt = 1
    else:
        raise TypeError("field must be float32 or float64")
    return np.ascontiguousarray(field), dt


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def segment(field: np.ndarray) -> dict:
    """Full segmentation of one field: order, up, dn, asc, desc, ms (int32,
    same shape as the field) and n_min, n_max, K."""
    f, dt = _prep(field)
    nx, ny, nz = _dims(f)
    out = {k: np.empty(f.shape, np.int32) for k in ("order", "up", "dn", "asc", "desc", "ms")}
    info = np.zeros(3, np.int64)
    rc = _load().plmss_oracle_segment(_p(f), dt, nx, ny, nz, _p(out["order"]), _p(out["up"]),
                                      _p(out["dn"]), _p(out["asc"]), _p(out["desc"]),
                                      _p(out["ms"]), _p(info))
    if rc:
        raise OracleError(rc, "segment")
    out.update(n_min=int(info[0]), n_max=int(info[1]), K=int(info[2]))
    return out


def order_field(field: np.ndarray):
    """Order field and the sorted vertex array (Sec. "Preprocessing")."""
    f, dt = _prep(field)
    nx, ny, nz = _dims(f)
    order = np.empty(f.shape, np.int32)
    perm = np.empty(f.size, np.int32)
    rc = _load().plmss_oracle_order(_p(f), dt, nx, ny, nz, _p(order), _p(perm))
    if rc:
        raise OracleError(rc, "order")
    return order, perm


def steepest(order: np.ndarray):
    """Steepest ascending (up) and descending (dn) neighbour of every vertex."""
    order = np.ascontiguousarray(order, dtype=np.int32)
    nx, ny, nz = _dims(order)
    up = np.empty(order.shape, np.int32)
    dn = np.empty(order.shape, np.int32)
    rc = _load().plmss_oracle_steepest(_p(order), nx, ny, nz, _p(up), _p(dn))
    if rc:
        raise OracleError(rc, "steepest")
    return up, dn


def labels(perm: np.ndarray, up: np.ndarray, dn: np.ndarray):
    """Extremum labels (asc, desc) from the sorted vertex array and pointers."""
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    up = np.ascontiguousarray(up, dtype=np.int32)
    dn = np.ascontiguousarray(dn, dtype=np.int32)
    asc = np.empty(up.shape, np.int32)
    desc = np.empty(up.shape, np.int32)
    rc = _load().plmss_oracle_labels(_p(perm), _p(up), _p(dn), up.size, _p(asc), _p(desc))
    if rc:
        raise OracleError(rc, "labels")
    return asc, desc


def ms_ids(asc: np.ndarray, desc: np.ndarray):
    """MS region ids (lexicographic rank of the (asc, desc) pair) and K."""
    asc = np.ascontiguousarray(asc, dtype=np.int32)
    desc = np.ascontiguousarray(desc, dtype=np.int32)
    ms = np.empty(asc.shape, np.int32)
    k = np.zeros(1, np.int64)
    rc = _load().plmss_oracle_ms(_p(asc), _p(desc), asc.size, _p(ms), _p(k))
    if rc:
        raise OracleError(rc, "ms")
    return ms, int(k[0])


def trace(field: np.ndarray, v: int):
    """(maximum, minimum, up_steps, dn_steps) reached from vertex v by walking
    the integral lines with Simulation-of-Simplicity comparisons."""
    f, dt = _prep(field)
    nx, ny, nz = _dims(f)
    res = np.zeros(4, np.int64)
    rc = _load().plmss_oracle_trace(_p(f), dt, nx, ny, nz, int(v), _p(res[0:]), _p(res[1:]),
                                    _p(res[2:]), _p(res[3:]))
    if rc:
        raise OracleError(rc, "trace")
    return int(res[0]), int(res[1]), int(res[2]), int(res[3])


def compress(dsc: np.ndarray, descending: bool = False, max_hist: int = 0):
    """The paper's list-based path compression, in place on a copy.  Returns
    (final pointers, number of iterations, history[iterations][n])."""
    d = np.ascontiguousarray(dsc, dtype=np.int32).ravel().copy()
    hist = np.zeros((max(max_hist, 0), d.size), np.int32)
    it = _load().plmss_oracle_compress(_p(d), d.size, int(bool(descending)),
                                       _p(hist) if max_hist > 0 else None, max_hist)
    if it < 0:
        raise OracleError(int(it), "compress")
    return d, int(it), hist[: min(int(it), max_hist)]


def degree_sum(nx: int, ny: int, nz: int) -> int:
    """Sum of vertex degrees (twice the edge count) of the triangulated grid."""
    return int(_load().plmss_oracle_degree_sum(nx, ny, nz))


def neighbours(nx: int, ny: int, nz: int, v: int):
    """Sorted neighbour ids of vertex v."""
    nb = np.zeros(14, np.int64)
    k = _load().plmss_oracle_neighbours(nx, ny, nz, int(v), _p(nb))
    if k < 0:
        raise OracleError(k, "neighbours")
    return sorted(int(a) for a in nb[:k])


def marching(labels: np.ndarray, mode: int = 0, with_codes: bool = True) -> dict:
    """Multi-label marching index (Sec. "Multi-Label Marching
    Triangles/Tetrahedra") of an int32 label field: per-cell codes (uint8,
    cell ((row * (nx-1)) + x) * cells_per_cube + t), row_offsets (int64,
    rows + 1 entries, exclusive prefix of the output primitives per row, the
    last entry the total) and total.  mode 0: region separators, 1: region
    boundaries."""
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    nx, ny, nz = _dims(labels)
    lib = _load()
    rows = int(lib.plmss_oracle_marching_rows(nx, ny, nz))
    per = 6 if nz > 1 else 2
    codes = np.zeros(rows * (nx - 1) * per if rows else 0, np.uint8)
    offsets = np.zeros(rows + 1, np.int64)
    rc = lib.plmss_oracle_marching(_p(labels), nx, ny, nz, int(mode), _p(codes) if with_codes and rows else None,
                                   _p(offsets))
    if rc:
        raise OracleError(rc, "marching")
    return {"codes": codes if with_codes else None, "row_offsets": offsets, "total": int(offsets[-1]),
            "rows": rows, "cells_per_cube": per}


def marching_geometry(labels: np.ndarray, mode: int = 0, capacity=None) -> dict:
    """Multi-label marching geometry (Sec. "Multi-Label Marching
    Triangles/Tetrahedra", case figures; "Triangulation Options") of an int32
    label field: the primitives the index counts, in cell order.  Returns
    ``xyz`` (float32, (T, 3, 3) triangles in 3-D, (T, 2, 2) segments in
    2-D; grid units), ``sides`` (int32, (T, 2)) and ``count``."""
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    nx, ny, nz = _dims(labels)
    lib = _load()
    if capacity is None:
        capacity = marching(labels, mode, with_codes=False)["total"]
    pts, dim = (3, 3) if nz > 1 else (2, 2)
    xyz = np.zeros((max(capacity, 1), pts, dim), np.float32)
    sides = np.zeros((max(capacity, 1), 2), np.int32)
    n = int(lib.plmss_oracle_marching_geometry(_p(labels), nx, ny, nz, int(mode), _p(xyz), _p(sides), int(capacity)))
    if n < 0:
        raise OracleError(n, "marching_geometry")
    return {"xyz": xyz[:n], "sides": sides[:n], "count": n}
