"""The C-ABI library loads, exports every declared entry point and rejects bad
arguments synchronously (no GPU needed: the checks run before any HIP call)."""
import ctypes
import os
import re

import pytest

import paper_2303_15491_amd as plmss

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "plmss.h")) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"\b(plmss_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("plmss_segment", "plmss_workspace_bytes", "plmss_order_field", "plmss_steepest",
              "plmss_compress", "plmss_ms_ids", "plmss_segment_batch", "plmss_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = plmss.library()
    for name in _declared():
        assert hasattr(lib, name), name
    assert b"gfx950" in lib.plmss_build_info()


def test_status_strings():
    lib = plmss.library()
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        s = lib.plmss_status_string(code).decode()
        assert s and s != "unknown status"
    assert lib.plmss_status_string(42).decode() == "unknown status"


FAKE = 0x1000  # never dereferenced: every case below fails its checks first


def _job(nx, ny, nz, dtype=plmss.F32, field=FAKE, asc=FAKE):
    return plmss.Job(field, plmss.Dims(nx, ny, nz), dtype, asc, FAKE, FAKE, None, None)


def test_segment_argument_errors():
    lib = plmss.library()
    seg = lib.plmss_segment
    assert seg(None, None, 0, None) == plmss.E_ARG
    assert seg(ctypes.byref(_job(4, 4, 1, field=None)), None, 0, None) == plmss.E_ARG
    assert seg(ctypes.byref(_job(4, 4, 1, asc=None)), None, 0, None) == plmss.E_ARG
    assert seg(ctypes.byref(_job(4, 4, 1, dtype=7)), None, 0, None) == plmss.E_ARG
    assert seg(ctypes.byref(_job(0, 4, 1)), None, 0, None) == plmss.E_DIMS
    assert seg(ctypes.byref(_job(4, -1, 1)), None, 0, None) == plmss.E_DIMS
    assert seg(ctypes.byref(_job(2048, 2048, 512)), None, 0, None) == plmss.E_TOO_LARGE
    assert seg(ctypes.byref(_job(2**31, 1, 1)), None, 0, None) == plmss.E_TOO_LARGE
    need = lib.plmss_workspace_bytes(plmss.Dims(4, 4, 1), plmss.F32, 0)
    assert seg(ctypes.byref(_job(4, 4, 1)), None, need, None) == plmss.E_WORKSPACE
    assert seg(ctypes.byref(_job(4, 4, 1)), ctypes.c_void_p(FAKE), need - 1, None) == plmss.E_WORKSPACE
    assert seg(ctypes.byref(_job(4, 4, 1)), ctypes.c_void_p(FAKE + 4), need, None) == plmss.E_WORKSPACE


def test_static_entry_point_argument_errors():
    """plmss_segment_static checks its arguments and its size limit before it
    touches the GPU (its scratch array is looked up only after them)."""
    lib = plmss.library()
    seg = lib.plmss_segment_static
    assert seg(None, None) == plmss.E_ARG
    assert seg(ctypes.byref(_job(4, 4, 1, field=None)), None) == plmss.E_ARG
    assert seg(ctypes.byref(_job(4, 4, 1, dtype=3)), None) == plmss.E_ARG
    assert seg(ctypes.byref(_job(0, 4, 1)), None) == plmss.E_DIMS
    assert seg(ctypes.byref(_job(plmss.STATIC_MAX_VERTICES + 1, 1, 1)), None) == plmss.E_TOO_LARGE
    assert seg(ctypes.byref(_job(256, 256, 33)), None) == plmss.E_TOO_LARGE
    # the array holds the workspace of the largest accepted field
    assert lib.plmss_static_scratch_bytes() >= lib.plmss_workspace_bytes(
        plmss.Dims(plmss.STATIC_MAX_VERTICES, 1, 1), plmss.F64, 0)


def test_step_entry_point_argument_errors():
    lib = plmss.library()
    d = plmss.Dims(8, 8, 8)
    assert lib.plmss_order_field(None, d, 0, FAKE, None, FAKE, 1 << 30, None) == plmss.E_ARG
    assert lib.plmss_order_field(FAKE, plmss.Dims(0, 1, 1), 0, FAKE, None, FAKE, 1 << 30, None) == plmss.E_DIMS
    assert lib.plmss_order_field(FAKE, d, 0, FAKE, None, FAKE, 16, None) == plmss.E_WORKSPACE
    assert lib.plmss_steepest(None, None, d, 0, FAKE, FAKE, None, None) == plmss.E_ARG
    assert lib.plmss_steepest(FAKE, None, d, 3, FAKE, FAKE, None, None) == plmss.E_ARG
    assert lib.plmss_steepest(FAKE, None, plmss.Dims(1, 0, 1), 0, FAKE, FAKE, None, None) == plmss.E_DIMS
    assert lib.plmss_compress(None, FAKE, 10, None) == plmss.E_ARG
    assert lib.plmss_compress(FAKE, FAKE, 0, None) == plmss.E_DIMS
    assert lib.plmss_compress(FAKE, FAKE, 2**31, None) == plmss.E_TOO_LARGE
    assert lib.plmss_ms_ids(FAKE, FAKE, 0, FAKE, None, FAKE, 1 << 30, None) == plmss.E_DIMS
    assert lib.plmss_ms_ids(FAKE, FAKE, 100, FAKE, None, FAKE, 8, None) == plmss.E_WORKSPACE


def test_workspace_sizes():
    lib = plmss.library()
    small = lib.plmss_workspace_bytes(plmss.Dims(64, 64, 1), plmss.F32, 0)
    big = lib.plmss_workspace_bytes(plmss.Dims(512, 512, 512), plmss.F32, 1)
    assert 0 < small < big
    assert big < 64 * 512**3  # about 28 bytes per vertex, twice with an order field, plus tables
    labels_only = lib.plmss_workspace_bytes(plmss.Dims(512, 512, 512), plmss.F32, 0)
    assert labels_only < 32 * 512**3 and big == 2 * labels_only
    assert lib.plmss_workspace_bytes(plmss.Dims(0, 1, 1), plmss.F32, 0) == 0
    assert lib.plmss_ms_workspace_bytes(0) == 0


def test_python_binding_refuses_host_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError):
        plmss.segment(torch.zeros(4, 4))
    with pytest.raises(ValueError):
        plmss.marching_index(torch.zeros(4, 4, dtype=torch.int32))
    with pytest.raises(ValueError):
        plmss.marching_geometry(torch.zeros(4, 4, dtype=torch.int32))


def test_tuning_knobs_validate_ranges():
    saved = plmss.tune_get()
    lib = plmss.library()
    try:
        assert set(saved) == set(plmss.KNOBS)
        assert lib.plmss_tune_get(99) == -1
        assert lib.plmss_tune_set(99, 1) == plmss.E_ARG
        assert lib.plmss_tune_set(plmss.KNOBS["sort_workers"], 0) == plmss.E_ARG
        assert lib.plmss_tune_set(plmss.KNOBS["sort_workers"], 5000) == plmss.E_ARG
        assert lib.plmss_tune_get(plmss.KNOBS["sort_workers"]) == saved["sort_workers"]
        assert lib.plmss_tune_set(plmss.KNOBS["scan_depth"], 24) == plmss.E_ARG
        assert lib.plmss_tune_set(plmss.KNOBS["scan_depth"], 64) == plmss.E_ARG
        assert lib.plmss_tune_set(plmss.KNOBS["order_packed"], 2) == plmss.E_ARG
        assert lib.plmss_tune_set(plmss.KNOBS["order_invert"], 65) == plmss.E_ARG
        assert lib.plmss_tune_set(plmss.KNOBS["scan_rounds"], 0) == plmss.E_ARG
        assert lib.plmss_tune_set(plmss.KNOBS["packed_codes"], 2) == plmss.E_ARG
        assert lib.plmss_tune_set(plmss.KNOBS["pair_stream"], 3) == plmss.E_ARG
        assert lib.plmss_tune_set(plmss.KNOBS["pair_stream"], -1) == plmss.E_ARG
        assert saved["pair_stream"] == 2
        plmss.tune_set(order_workers=0, order_invert=0, sort_workers=512, persist_blocks=4096, scan_depth=8,
                       order_packed=1, scan_rounds=1, order_concurrent=0, packed_codes=1, pair_stream=0)
        assert plmss.tune_get() == {"order_workers": 0, "order_invert": 0, "sort_workers": 512,
                                    "persist_blocks": 4096, "scan_depth": 8, "order_packed": 1, "scan_rounds": 1,
                                    "order_concurrent": 0, "packed_codes": 1, "pair_stream": 0}
        with pytest.raises(plmss.PlmssError):
            plmss.tune_set(order_workers=10)
        with pytest.raises(KeyError):
            plmss.tune_set(nothing=1)
    finally:
        plmss.tune_set(**saved)


def test_marching_argument_errors_and_rows():
    import oracle

    orc_rows = oracle._load().plmss_oracle_marching_rows
    lib = plmss.library()
    d = plmss.Dims(8, 8, 8)
    ws = lib.plmss_marching_workspace_bytes(d)
    assert ws >= 8 and ws % 256 == 0
    mi = lib.plmss_marching_index
    assert mi(None, d, 0, None, FAKE, FAKE, ws, None) == plmss.E_ARG
    assert mi(FAKE, d, 0, None, None, FAKE, ws, None) == plmss.E_ARG
    assert mi(FAKE, d, 2, None, FAKE, FAKE, ws, None) == plmss.E_ARG
    assert mi(FAKE, d, -1, None, FAKE, FAKE, ws, None) == plmss.E_ARG
    assert mi(FAKE, d, 0, FAKE + 1, FAKE, FAKE, ws, None) == plmss.E_ARG  # odd codes address
    assert mi(FAKE, plmss.Dims(0, 8, 8), 0, None, FAKE, FAKE, ws, None) == plmss.E_DIMS
    assert mi(FAKE, plmss.Dims(2048, 2048, 512), 0, None, FAKE, FAKE, ws, None) == plmss.E_TOO_LARGE
    assert mi(FAKE, d, 0, None, FAKE, None, ws, None) == plmss.E_WORKSPACE
    assert mi(FAKE, d, 0, None, FAKE, FAKE, ws - 1, None) == plmss.E_WORKSPACE
    assert mi(FAKE, d, 1, None, FAKE, FAKE + 8, ws, None) == plmss.E_WORKSPACE
    for dims in ((8, 8, 8), (2, 2, 2), (5, 7, 3), (9, 4, 1), (1, 4, 4), (4, 1, 4), (4, 4, 1), (7, 1, 1),
                 (1, 1, 1), (512, 512, 512), (3, 1, 5)):
        rows = lib.plmss_marching_rows(plmss.Dims(*dims))
        assert rows == orc_rows(*dims), dims
        assert rows == plmss.marching_rows(dims[::-1])
        assert lib.plmss_marching_workspace_bytes(plmss.Dims(*dims)) >= 8 * ((rows + 255) // 256)
    assert lib.plmss_marching_rows(plmss.Dims(0, 1, 1)) == -1
    assert lib.plmss_marching_workspace_bytes(plmss.Dims(0, 1, 1)) == 0


def test_marching_geometry_argument_errors():
    lib = plmss.library()
    d = plmss.Dims(8, 8, 8)
    g = lib.plmss_marching_geometry
    assert g(None, d, 0, FAKE, 10, FAKE, FAKE, None) == plmss.E_ARG
    assert g(FAKE, d, 0, None, 10, FAKE, FAKE, None) == plmss.E_ARG
    assert g(FAKE, d, 3, FAKE, 10, FAKE, FAKE, None) == plmss.E_ARG
    assert g(FAKE, d, 0, FAKE, 10, FAKE + 2, FAKE, None) == plmss.E_ARG  # xyz not 4-byte aligned
    assert g(FAKE, d, 0, FAKE, 10, FAKE, FAKE + 4, None) == plmss.E_ARG  # sides not 8-byte aligned
    assert g(FAKE, plmss.Dims(0, 8, 8), 0, FAKE, 10, FAKE, FAKE, None) == plmss.E_DIMS
    assert g(FAKE, plmss.Dims(2048, 2048, 512), 0, FAKE, 10, FAKE, FAKE, None) == plmss.E_TOO_LARGE
    # grids without cells and calls without outputs launch nothing
    assert g(FAKE, plmss.Dims(8, 1, 1), 0, FAKE, 10, FAKE, FAKE, None) == plmss.OK
    assert g(FAKE, d, 1, FAKE, 10, None, None, None) == plmss.OK
