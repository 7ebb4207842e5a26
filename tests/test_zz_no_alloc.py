"""The segmentation entry point that allocates nothing (plmss_segment_static,
called through the C ABI) against the workspace entry point (plmss_segment)
and the oracle: bit-exact labels, order field and info, on two calls in a row
whose second field is smaller than the first, so that stale contents of the
shared scratch array cannot pass for results."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import paper_2303_15491_amd as plmss
from paper_2303_15491_amd import fields

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t

    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def _static(torch, f, with_order):
    """plmss_segment_static through ctypes; returns host arrays."""
    lib = plmss.library()
    dev = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    out = {k: torch.full(f.shape, -1, dtype=torch.int32, device="cuda") for k in ("asc", "desc", "ms", "order")}
    out["info"] = torch.full((4,), -1, dtype=torch.int32, device="cuda")
    code = plmss.F64 if f.dtype == np.float64 else plmss.F32
    job = plmss.Job(dev.data_ptr(), plmss.dims_of(f.shape), code, out["asc"].data_ptr(), out["desc"].data_ptr(),
                    out["ms"].data_ptr(), out["order"].data_ptr() if with_order else None, out["info"].data_ptr())
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.plmss_segment_static(ctypes.byref(job), stream)
    assert rc == plmss.OK, rc
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _check(torch, f, with_order, label):
    _say(f"static {label} shape={f.shape} dtype={f.dtype} order={with_order}")
    got = _static(torch, f, with_order)
    plain = plmss.segment(torch.from_numpy(np.ascontiguousarray(f)).cuda(), with_order=with_order)
    torch.cuda.synchronize()
    ref = oracle.segment(f)
    keys = ("asc", "desc", "ms", "order") if with_order else ("asc", "desc", "ms")
    for k in keys:
        np.testing.assert_array_equal(got[k], plain[k].cpu().numpy(), err_msg=f"{label} {k} vs plmss_segment")
        np.testing.assert_array_equal(got[k], ref[k], err_msg=f"{label} {k} vs oracle")
    np.testing.assert_array_equal(got["info"], plain["info"].cpu().numpy())
    assert got["info"].tolist() == [0, ref["n_min"], ref["n_max"], ref["K"]], label


def test_static_scratch_two_calls_second_smaller(torch):
    big = fields.smoothed_noise((128, 128, 128), 1.5, seed=41)  # the largest field the array holds
    assert big.size == plmss.STATIC_MAX_VERTICES
    small = fields.smoothed_noise((23, 41, 77), 2.0, seed=42)
    _check(torch, big, True, "first (max size)")
    _check(torch, small, True, "second (smaller)")
    _check(torch, small.astype(np.float64), False, "third (float64, labels only)")
    _check(torch, fields.workload_c1(), True, "fourth (2-D)")


def test_static_scratch_rejects_oversize(torch):
    lib = plmss.library()
    job = plmss.Job(1, plmss.Dims(plmss.STATIC_MAX_VERTICES + 1, 1, 1), plmss.F32, 1, 1, 1, None, None)
    assert lib.plmss_segment_static(ctypes.byref(job), None) == plmss.E_TOO_LARGE
    job = plmss.Job(1, plmss.Dims(0, 1, 1), plmss.F32, 1, 1, 1, None, None)
    assert lib.plmss_segment_static(ctypes.byref(job), None) == plmss.E_DIMS
    assert lib.plmss_segment_static(None, None) == plmss.E_ARG
    assert lib.plmss_static_scratch_bytes() >= plmss.workspace_bytes((128, 128, 128), with_order=False)
