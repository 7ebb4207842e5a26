"""GPU parity: the HIP library, called through its C ABI, against the CPU
oracle on the same seeded inputs.  Labels are integers, so the bar is
bit-exact equality of every output (asc, desc, ms, order, #minima, #maxima, K).
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2303_15491_amd as plmss
from paper_2303_15491_amd import fields

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t

    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    return t.cpu().numpy()


def _compare_full(torch, f, with_order=False, label=""):
    _say(f"segment {label} shape={f.shape} dtype={f.dtype} order={with_order}")
    ref = oracle.segment(f)
    out = plmss.segment(_dev(torch, f), with_order=with_order)
    torch.cuda.synchronize()
    info = _host(out["info"])
    assert info[0] == 0
    for k in ("asc", "desc", "ms"):
        np.testing.assert_array_equal(_host(out[k]), ref[k], err_msg=f"{label} {k}")
    if with_order:
        np.testing.assert_array_equal(_host(out["order"]), ref["order"], err_msg=f"{label} order")
    assert (info[1], info[2], info[3]) == (ref["n_min"], ref["n_max"], ref["K"]), label
    return ref, out


def test_fig1_worked_example(torch):
    with open(os.path.join(GOLDEN, "fig1_wallmodes.json")) as fh:
        g = json.load(fh)
    f = np.array(g["field"], np.float32).reshape(4, 4)
    _say("fig1")
    out = plmss.segment(_dev(torch, f), with_order=True)
    torch.cuda.synchronize()
    assert _host(out["asc"]).ravel().tolist() == g["asc"]
    assert _host(out["desc"]).ravel().tolist() == g["desc"]
    assert _host(out["ms"]).ravel().tolist() == g["ms"]
    assert _host(out["order"]).ravel().tolist() == g["field"]
    assert _host(out["info"]).tolist() == [0, 2, 2, g["K"]]


@pytest.mark.parametrize("with_order", [False, True])
def test_config_2d_gaussian_mix(torch, with_order):
    _compare_full(torch, fields.workload_c1(), with_order, "c1")


@pytest.mark.parametrize("shape", [(37, 70, 130), (16, 8, 64), (17, 9, 65), (3, 200, 7), (40, 1, 33), (5, 77, 1),
                                   (1, 300, 257)])
def test_ragged_tiles_both_paths(torch, shape):
    f = fields.smoothed_noise(shape, 1.5, seed=sum(shape))
    _, a = _compare_full(torch, f, False, f"ragged{shape}")
    _, b = _compare_full(torch, f, True, f"ragged{shape}+order")
    for k in ("asc", "desc", "ms"):
        assert torch.equal(a[k], b[k])


@pytest.mark.parametrize("knobs", [
    {"scan_depth": 8}, {"scan_depth": 32}, {"order_invert": 0}, {"order_invert": 5},
    {"order_invert": 1, "order_workers": 0}, {"order_invert": 1, "order_workers": 64},
    {"order_packed": 0, "order_invert": 1}, {"order_packed": 0, "order_invert": 0},
    {"order_packed": 0, "order_invert": 3, "order_workers": 64},
    {"order_packed": 0, "order_invert": 64, "order_workers": 0},
    {"sort_workers": 64}, {"sort_workers": 4096},
    {"scan_rounds": 1}, {"scan_rounds": 8, "scan_depth": 32}, {"scan_rounds": 2, "scan_depth": 8},
    {"order_concurrent": 1}, {"order_concurrent": 1, "order_packed": 0},
    {"packed_codes": 0}, {"packed_codes": 0, "scan_depth": 8},
    {"pair_stream": 1}, {"pair_stream": 0, "sort_workers": 64},
])
def test_launch_shapes_keep_results(torch, knobs):
    """Every launch-shape knob setting gives the oracle's labels (tile depths
    that split a field unevenly, ragged last windows, one-tile workers)."""
    saved = plmss.tune_get()
    try:
        plmss.tune_set(**knobs)
        f = fields.smoothed_noise((45, 70, 130), 1.5, seed=5)
        _compare_full(torch, f, True, f"knobs {knobs}")
        _compare_full(torch, fields.smoothed_noise((40, 1, 33), 2.0, seed=6), True, f"knobs {knobs} thin")
    finally:
        plmss.tune_set(**saved)


@pytest.mark.parametrize("shape,offset", [((40, 24, 96), 0), ((40, 24, 97), 0), ((40, 24, 96), 1)])
def test_whole_line_rows_and_the_rest(torch, shape, offset):
    """A field whose label rows are whole 128-byte lines (x a multiple of 32,
    arrays on line boundaries) takes the streaming chase and MS write-back;
    one with a ragged x, or with label arrays one element off a line, takes
    the plain ones.  Both give the oracle's labels."""
    f = fields.smoothed_noise(shape, 1.5, seed=11)
    ref = oracle.segment(f)
    n = f.size
    buf = {k: torch.empty(n + 64, dtype=torch.int32, device="cuda") for k in ("asc", "desc", "ms")}
    out = {k: buf[k][offset:offset + n].view(shape) for k in buf}
    out["info"] = torch.empty(4, dtype=torch.int32, device="cuda")
    _say(f"whole lines shape={shape} offset={offset}")
    plmss.segment(_dev(torch, f), out=out)
    torch.cuda.synchronize()
    for k in ("asc", "desc", "ms"):
        np.testing.assert_array_equal(_host(out[k]), ref[k], err_msg=f"{shape} {offset} {k}")
    assert _host(out["info"]).tolist()[:4] == [0, ref["n_min"], ref["n_max"], ref["K"]]


def test_segment_rejects_outputs_of_the_wrong_form(torch):
    """Output tensors are checked before any launch: a short, mistyped,
    strided or host tensor would otherwise be written past its end."""
    f = _dev(torch, fields.smoothed_noise((16, 20, 24), 1.5, seed=12))
    good = {k: torch.empty(f.shape, dtype=torch.int32, device="cuda") for k in ("asc", "desc", "ms")}
    good["info"] = torch.empty(4, dtype=torch.int32, device="cuda")
    bad_outs = [
        dict(good, asc=torch.empty(f.numel() - 1, dtype=torch.int32, device="cuda")),
        dict(good, desc=torch.empty(f.shape, dtype=torch.int64, device="cuda")),
        dict(good, ms=torch.empty(f.numel() * 2, dtype=torch.int32, device="cuda")[::2]),
        dict(good, ms=torch.empty(f.shape, dtype=torch.int32)),
        dict(good, info=torch.empty(3, dtype=torch.int32, device="cuda")),
        {k: v for k, v in good.items() if k != "info"},
    ]
    for fn in (plmss.segment, plmss.segment_static):
        for o in bad_outs:
            with pytest.raises(ValueError):
                fn(f, out=o)
        with pytest.raises(ValueError):
            fn(f, with_order=True, out=good)  # no order tensor
        fn(f, out=good)
    torch.cuda.synchronize()
    assert _host(good["info"])[0] == 0


def test_degenerate_dims(torch):
    _compare_full(torch, np.arange(1000, dtype=np.float32), True, "line")
    _compare_full(torch, np.array([1.5], np.float32), True, "single")
    _compare_full(torch, np.array([2.0, 1.0], np.float32), True, "pair")
    _compare_full(torch, fields.smoothed_noise((50, 60), 2.0, 7).reshape(1, 50, 60), False, "nz1")
    _compare_full(torch, np.full((7, 9, 11), 3.0, np.float32), True, "constant")


def test_ties_signed_zero_subnormal_infinity(torch):
    rng = np.random.default_rng(12)
    tiny = np.float32(1.4e-45)
    vals = np.array([0.0, -0.0, tiny, -tiny, 2 * tiny, np.inf, -np.inf, 1.0, -1.0, 0.5], np.float32)
    _compare_full(torch, rng.choice(vals, size=(19, 23, 70)), True, "specials")
    _compare_full(torch, rng.integers(0, 4, size=(33, 66, 67)).astype(np.float32), True, "ties")
    _compare_full(torch, rng.choice(vals, size=(19, 23, 70)).astype(np.float64), True, "specials-f64")


def test_float64_widened_is_identical(torch):
    f = fields.smoothed_noise((24, 40, 70), 1.5, 9)
    _, a = _compare_full(torch, f, True, "f32")
    _, b = _compare_full(torch, f.astype(np.float64), True, "f64")
    for k in ("asc", "desc", "ms", "order"):
        assert torch.equal(a[k], b[k])


@pytest.mark.parametrize("knobs", [
    {"order_packed": 1, "order_invert": 1}, {"order_packed": 1, "order_invert": 0},
    {"order_packed": 1, "order_invert": 3, "order_workers": 64}, {"order_packed": 0, "order_invert": 1},
])
def test_float64_order_field_knobs(torch, knobs):
    """Float64 values that are not widened float32 (all 64 key bits carry
    information, with ties and both signs) through every order-field layout."""
    saved = plmss.tune_get()
    try:
        plmss.tune_set(**knobs)
        rng = np.random.default_rng(17)
        f = fields.smoothed_noise((30, 41, 67), 1.5, 11).astype(np.float64)
        f += rng.standard_normal(f.shape) * 1e-12
        f[rng.random(f.shape) < 0.01] = 0.25  # ties
        _compare_full(torch, f, True, f"f64 knobs {knobs}")
    finally:
        plmss.tune_set(**saved)


def _one_minimum_many_maxima(nx):
    """Two rows: the lower rises to the right (its left end is the only
    minimum), the upper alternates high and low (every high vertex is a
    maximum), so one minimum pairs with nx / 2 maxima."""
    x = np.arange(nx, dtype=np.float64)
    return np.stack([1e-3 * x, 10.0 + (x % 2 == 0)]).astype(np.float32)


@pytest.mark.parametrize("nx", [1500, 4096])
def test_ms_ids_one_minimum_many_maxima(torch, nx):
    """MS ids when one minimum pairs with thousands of maxima (one long run
    of equal asc in the sorted pairs, spread over many chase tiles): the
    same ids as the oracle, alone and inside a batch with ordinary fields."""
    f = _one_minimum_many_maxima(nx)
    ref, _ = _compare_full(torch, f, True, f"one minimum, {nx // 2} maxima")
    assert ref["n_min"] == 1 and ref["n_max"] >= nx // 2
    others = [fields.smoothed_noise((20, 30, 40), 1.5, seed=31), fields.smoothed_noise((64, 64), 2.0, seed=32)]
    batch = [others[0], f, others[1]]
    _say("batch with a large group")
    outs = plmss.segment_batch([_dev(torch, a) for a in batch], with_order=True)
    torch.cuda.synchronize()
    for a, o in zip(batch, outs):
        r = oracle.segment(a)
        for k in ("asc", "desc", "ms", "order"):
            np.testing.assert_array_equal(_host(o[k]), r[k], err_msg=f"large-group batch {a.shape} {k}")
        assert int(o["info"][3]) == r["K"]


# Lengths at the edges of the order field's inversion: one id chunk (2^15),
# id ranges of 2^15 .. 2^23 ids (their size follows the length), tiles of
# the regrouping that straddle two ranges, and a last range shorter than a tile.
@pytest.mark.parametrize("n", [4095, 4096, 32767, 32768, 32769, 65537, 2 ** 21 + 4097, 2 ** 22 - 1, 2 ** 22,
                               2 ** 22 + 1, 2 ** 23 + 3000])
def test_order_field_at_range_and_chunk_edges(torch, n):
    """The order field of a line of n random values (every order equally
    likely, ties included): equal to the oracle's, and no lost pair reported."""
    rng = np.random.default_rng(n)
    f = rng.standard_normal(n).astype(np.float32)
    f[rng.random(n) < 0.001] = 0.5  # a few ties
    _say(f"order field n={n}")
    order, info = plmss.order_field(_dev(torch, f))
    torch.cuda.synchronize()
    assert int(info[0]) == 0
    ref, _ = oracle.order_field(f)
    np.testing.assert_array_equal(_host(order), ref)


def test_nan_reported_on_device(torch):
    f = fields.smoothed_noise((8, 9, 10), 1.5, 3)
    f[3, 4, 5] = np.nan
    _say("nan")
    for with_order in (False, True):
        out = plmss.segment(_dev(torch, f), with_order=with_order)
        torch.cuda.synchronize()
        assert int(out["info"][0]) == plmss.E_NAN


def test_step_entry_points_match_oracle(torch):
    f = fields.smoothed_noise((21, 35, 90), 1.5, 13)
    ref = oracle.segment(f)
    _say("order_field")
    order, info = plmss.order_field(_dev(torch, f))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_host(order), ref["order"])
    assert int(info[0]) == 0
    _say("steepest from field")
    up, dn, info = plmss.steepest(field=_dev(torch, f))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_host(up), ref["up"])
    np.testing.assert_array_equal(_host(dn), ref["dn"])
    assert (int(info[1]), int(info[2])) == (ref["n_min"], ref["n_max"])
    _say("steepest from order")
    up2, dn2, _ = plmss.steepest(order=_dev(torch, ref["order"]))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_host(up2), ref["up"])
    np.testing.assert_array_equal(_host(dn2), ref["dn"])
    _say("compress")
    d, a = plmss.compress(_dev(torch, ref["up"]), _dev(torch, ref["dn"]))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_host(d), ref["desc"])
    np.testing.assert_array_equal(_host(a), ref["asc"])
    _say("ms_ids")
    ms, info = plmss.ms_ids(_dev(torch, ref["asc"]), _dev(torch, ref["desc"]))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_host(ms), ref["ms"])
    assert int(info[3]) == ref["K"]


def test_compress_long_chain(torch):
    n = 1 << 20
    up = np.minimum(np.arange(n, dtype=np.int32) + 1, n - 1)
    _say("compress chain")
    d, a = plmss.compress(_dev(torch, up), _dev(torch, np.arange(n, dtype=np.int32)))
    torch.cuda.synchronize()
    assert (_host(d) == n - 1).all() and (_host(a) == np.arange(n)).all()


@pytest.mark.parametrize("with_order", [False, True])
def test_config_3d_256_full_oracle(torch, with_order):
    """256^3 against the oracle element by element; with the order field this
    also covers the digit scans split over several blocks per digit (4096
    radix workers)."""
    f = fields.workload_c2(256)
    _compare_full(torch, f, with_order, f"c2-256 order={with_order}")


@pytest.fixture(scope="module")
def c3_oracle():
    """The 512^3 float32 field and its oracle segmentation, computed once
    (about a minute and 4 GB of host memory)."""
    _say("c3-512 generate")
    f = fields.workload_c3(512)
    _say("c3-512 oracle")
    return f, oracle.segment(f)


def _compare_to_ref(torch, field_dev, ref, label):
    out = plmss.segment(field_dev, with_order=True)
    torch.cuda.synchronize()
    info = _host(out["info"])
    assert info[0] == 0, label
    assert (info[1], info[2], info[3]) == (ref["n_min"], ref["n_max"], ref["K"]), label
    for k in ("order", "asc", "desc", "ms"):
        got = _host(out[k])
        bad = np.flatnonzero(got.ravel() != ref[k].ravel())
        assert bad.size == 0, f"{label} {k}: {bad.size} vertices differ, first at {bad[:5].tolist()}"
    del out
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_config_3d_512_full_oracle(torch, c3_oracle):
    """The headline 512^3 float32 field against the oracle, every vertex of
    every output (order field, asc, desc, ms) and every count."""
    f, ref = c3_oracle
    _say("c3-512 f32 segment")
    _compare_to_ref(torch, _dev(torch, f), ref, "c3-512 f32")


@pytest.mark.timeout(900)
def test_config_3d_512_float64_copy_full_oracle(torch, c3_oracle):
    """The float64 copy of the same field (every value widened exactly)
    against the same oracle result: widening preserves the vertex order, so
    every output is the float32 field's."""
    f, ref = c3_oracle
    _say("c3-512 f64 segment")
    _compare_to_ref(torch, _dev(torch, f.astype(np.float64)), ref, "c3-512 f64")
