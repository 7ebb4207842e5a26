"""GPU parity of the multi-label marching index (Sec. "Multi-Label Marching
Triangles/Tetrahedra"): the HIP pass, called through the C ABI, against the
CPU oracle on the same seeded label fields.  Codes and offsets are integers:
every byte and every offset must be equal."""
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


def _compare(torch, labels, mode, label=""):
    _say(f"marching {label} shape={labels.shape} mode={mode}")
    ref = oracle.marching(labels, mode)
    codes, offs = plmss.marching_index(_dev(torch, labels), mode, with_codes=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(offs.cpu().numpy(), ref["row_offsets"], err_msg=f"{label} offsets")
    np.testing.assert_array_equal(codes.cpu().numpy(), ref["codes"], err_msg=f"{label} codes")
    # without codes the offsets are the same
    none, offs2 = plmss.marching_index(_dev(torch, labels), mode, with_codes=False)
    torch.cuda.synchronize()
    assert none is None
    np.testing.assert_array_equal(offs2.cpu().numpy(), ref["row_offsets"], err_msg=f"{label} offsets, no codes")
    return ref


# shapes (nz, ny, nx): ragged against the 64-cube lane chunks and the rows
# per wave / per block split, ones with more than 1024 count blocks (several
# rounds of the block-sum scan: 6000 rows at one row per wave), planar ones,
# and grids without cells
SHAPES_3D = [(2, 2, 2), (3, 5, 130), (4, 3, 65), (9, 17, 64), (5, 9, 66), (12, 9, 70), (3, 300, 300),
             (2, 2, 4097), (2, 6001, 5)]
SHAPES_2D = [(2, 2), (5, 130), (300, 257), (5000, 5), (1025, 65)]


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6])
@pytest.mark.parametrize("mode", [0, 1])
def test_random_labels_3d(torch, k, mode):
    for i, shape in enumerate(SHAPES_3D[:6]):
        _compare(torch, fields.random_labels(shape, k, seed=100 * k + i), mode, f"k={k}")


@pytest.mark.parametrize("k", [1, 2, 3, 5])
@pytest.mark.parametrize("mode", [0, 1])
def test_random_labels_2d(torch, k, mode):
    for i, shape in enumerate(SHAPES_2D):
        _compare(torch, fields.random_labels(shape, k, seed=200 * k + i), mode, f"2d k={k}")


@pytest.mark.parametrize("mode", [0, 1])
def test_many_blocks(torch, mode):
    _compare(torch, fields.random_labels(SHAPES_3D[6], 3, seed=7), mode, "3x300x300")
    _compare(torch, fields.region_labels(SHAPES_3D[7], seed=8), mode, "2x2x4097")
    _compare(torch, fields.random_labels(SHAPES_3D[8], 3, seed=9), mode, "2x6001x5")
    _compare(torch, fields.random_labels((70001, 3), 3, seed=10), mode, "70001x3")  # 16 rows per wave


@pytest.mark.parametrize("shape", [(1, 1, 1), (7,), (3, 4, 1), (4, 1, 4), (4, 4, 1), (1, 1, 9), (2, 1, 1), (1, 6),
                                   (6, 1), (1,)])
def test_grids_without_cells(torch, shape):
    labels = fields.random_labels(shape, 3, seed=1)
    ref = _compare(torch, labels, 0, f"degenerate {shape}")
    assert ref["rows"] == 0 and ref["total"] == 0


def test_one_plane_is_planar(torch):
    """A 3-D shape one plane thick is the 2-D grid of that plane."""
    labels = fields.random_labels((6, 70), 3, seed=4)
    r2 = _compare(torch, labels, 0, "plane")
    r3 = _compare(torch, labels.reshape(1, 6, 70), 0, "plane as 3-D")
    np.testing.assert_array_equal(r2["codes"], r3["codes"])
    assert r3["cells_per_cube"] == 2


def test_region_labels(torch):
    for i, shape in enumerate([(40, 40, 40), (33, 65, 129), (1, 257, 255), (700, 700)]):
        labels = fields.region_labels(shape, seed=30 + i)
        for mode in (0, 1):
            _compare(torch, labels, mode, f"regions {shape}")


def test_every_tetrahedron_code_appears(torch):
    """The random-label cases above reach all fifteen codes of the table."""
    with open(os.path.join(GOLDEN, "tet_binary_codes.json")) as fh:
        table = json.load(fh)
    want = sorted(int(r["code"]) for r in table["rows"])
    labels = fields.random_labels((6, 7, 70), 4, seed=3)
    codes, _ = plmss.marching_index(_dev(torch, labels), 0, with_codes=True)
    torch.cuda.synchronize()
    assert sorted(set(codes.cpu().numpy().tolist())) == want


def test_ms_labels_of_a_segmentation(torch):
    """The index over the MS, ascending and descending labels of a real
    segmentation, each side computing its own labels."""
    f = fields.smoothed_noise((24, 40, 70), 1.5, seed=11)
    ref = oracle.segment(f)
    out = plmss.segment(_dev(torch, f))
    torch.cuda.synchronize()
    for key in ("ms", "asc", "desc"):
        for mode in (0, 1):
            r = oracle.marching(ref[key], mode)
            codes, offs = plmss.marching_index(out[key], mode, with_codes=True)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(offs.cpu().numpy(), r["row_offsets"], err_msg=key)
            np.testing.assert_array_equal(codes.cpu().numpy(), r["codes"], err_msg=key)


def test_out_tensors_and_stream(torch):
    labels = fields.random_labels((5, 9, 66), 3, seed=5)
    ref = oracle.marching(labels, 0)
    rows = plmss.marching_rows(labels.shape)
    codes = torch.full((rows * 65 * 6 + 2,), 0xAB, dtype=torch.uint8, device="cuda")
    offs = torch.full((rows + 1,), -1, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    d = _dev(torch, labels)
    torch.cuda.current_stream().synchronize()
    with torch.cuda.stream(s):
        c, o = plmss.marching_index(d, 0, out=(codes, offs), stream=s)
    s.synchronize()
    np.testing.assert_array_equal(o.cpu().numpy(), ref["row_offsets"])
    np.testing.assert_array_equal(c.cpu().numpy(), ref["codes"])
    assert codes[-2:].cpu().tolist() == [0xAB, 0xAB]  # nothing written past the cells


def test_full_size_sampled_rows(torch):
    """512^3 labels in the launch shape the measurement uses: every row's
    count equals the count of its own 2 x 2 x nx slab under the oracle on
    sampled rows (first, last, random), all codes are codes of the table, and
    the counts that the codes imply add up to the offsets everywhere."""
    with open(os.path.join(GOLDEN, "tet_binary_codes.json")) as fh:
        table = json.load(fh)
    n = 512
    labels = fields.region_labels((n, n, n), seed=9)
    rows = (n - 1) * (n - 1)
    rng = np.random.Generator(np.random.PCG64(12))
    sample = sorted(set([0, 1, n - 2, n - 1, rows - 1] + rng.integers(0, rows, size=48).tolist()))
    d = _dev(torch, labels)
    for mode in (0, 1):
        _say(f"marching 512^3 mode={mode}")
        codes, offs = plmss.marching_index(d, mode, with_codes=True)
        torch.cuda.synchronize()
        o = offs.cpu().numpy()
        c = codes.cpu().numpy().reshape(rows, n - 1, 6)
        assert o[0] == 0 and np.all(np.diff(o) >= 0)
        for r in sample:
            y, z = r % (n - 1), r // (n - 1)
            slab = oracle.marching(labels[z:z + 2, y:y + 2, :], mode)
            assert o[r + 1] - o[r] == slab["total"], r
            np.testing.assert_array_equal(c[r].ravel(), slab["codes"], err_msg=f"row {r}")
        # counts implied by the codes, with the table's own per-code figures
        # (a boundary triangle: two labels, one vertex apart)
        per_code = np.zeros(64, np.int8)
        for row in table["rows"]:
            lone = row["labels"] == 2 and row["separators"] == 1
            per_code[int(row["code"])] = int(row["separators"]) if mode == 0 else int(lone)
        valid = np.zeros(64, bool)
        valid[[int(row["code"]) for row in table["rows"]]] = True
        assert valid[c].all()
        implied = per_code[c].sum(axis=(1, 2), dtype=np.int64)
        np.testing.assert_array_equal(np.diff(o), implied)


# ---- geometry pass ------------------------------------------------------------------------

def _bits(a):
    return np.ascontiguousarray(a).view(np.int32)


def _compare_geo(torch, labels, mode, label=""):
    _say(f"geometry {label} shape={labels.shape} mode={mode}")
    ref = oracle.marching_geometry(labels, mode)
    xyz, sides, count = plmss.marching_geometry(_dev(torch, labels), mode)
    torch.cuda.synchronize()
    assert count == ref["count"], label
    np.testing.assert_array_equal(_bits(xyz.cpu().numpy()), _bits(ref["xyz"]), err_msg=f"{label} xyz")
    np.testing.assert_array_equal(sides.cpu().numpy(), ref["sides"], err_msg=f"{label} sides")
    return ref


@pytest.mark.parametrize("k", [2, 3, 4, 6])
@pytest.mark.parametrize("mode", [0, 1])
def test_geometry_random_labels(torch, k, mode):
    for i, shape in enumerate(SHAPES_3D[:6] + SHAPES_2D[:4]):
        _compare_geo(torch, fields.random_labels(shape, k, seed=300 * k + i), mode, f"k={k}")


@pytest.mark.parametrize("mode", [0, 1])
def test_geometry_region_and_segmentation_labels(torch, mode):
    for i, shape in enumerate([(40, 40, 40), (33, 65, 129), (1, 257, 255), (300, 301)]):
        _compare_geo(torch, fields.region_labels(shape, seed=50 + i), mode, f"regions {shape}")
    f = fields.smoothed_noise((24, 40, 70), 1.5, seed=11)
    ref = oracle.segment(f)
    out = plmss.segment(_dev(torch, f))
    torch.cuda.synchronize()
    for key in ("ms", "asc", "desc"):
        r = oracle.marching_geometry(ref[key], mode)
        xyz, sides, count = plmss.marching_geometry(out[key], mode)
        torch.cuda.synchronize()
        assert count == r["count"]
        np.testing.assert_array_equal(_bits(xyz.cpu().numpy()), _bits(r["xyz"]), err_msg=key)
        np.testing.assert_array_equal(sides.cpu().numpy(), r["sides"], err_msg=key)


def test_geometry_capacity_and_partial_outputs(torch):
    labels = fields.random_labels((5, 9, 66), 4, seed=6)
    ref = oracle.marching_geometry(labels, 0)
    n = ref["count"]
    d = _dev(torch, labels)
    _, offs = plmss.marching_index(d, 0)
    cap = n // 3
    xyz = torch.full((n, 3, 3), -7.0, dtype=torch.float32, device="cuda")
    sides = torch.full((n, 2), -7, dtype=torch.int32, device="cuda")
    plmss.marching_geometry(d, 0, row_offsets=offs, out=(xyz, sides, cap))
    torch.cuda.synchronize()
    x, s = xyz.cpu().numpy(), sides.cpu().numpy()
    np.testing.assert_array_equal(_bits(x[:cap]), _bits(ref["xyz"][:cap]))
    np.testing.assert_array_equal(s[:cap], ref["sides"][:cap])
    assert np.all(x[cap:] == -7.0) and np.all(s[cap:] == -7)
    only_xyz, none, _ = plmss.marching_geometry(d, 0, with_sides=False)
    none2, only_sides, _ = plmss.marching_geometry(d, 0, with_xyz=False)
    torch.cuda.synchronize()
    assert none is None and none2 is None
    np.testing.assert_array_equal(_bits(only_xyz.cpu().numpy()), _bits(ref["xyz"]))
    np.testing.assert_array_equal(only_sides.cpu().numpy(), ref["sides"])


def test_geometry_rejects_bad_out_tensors(torch):
    """Outputs smaller than the capacity, of the wrong type or layout, and
    row offsets of the wrong type or length are refused before any launch."""
    labels = _dev(torch, fields.random_labels((4, 5, 6), 3, seed=1))
    _, offs = plmss.marching_index(labels, 0)
    torch.cuda.synchronize()
    cap = 10
    ok_xyz = torch.empty((cap, 3, 3), dtype=torch.float32, device="cuda")
    ok_sides = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    bad = [
        dict(out=(torch.empty((cap - 1, 3, 3), dtype=torch.float32, device="cuda"), ok_sides, cap)),
        dict(out=(ok_xyz, torch.empty((cap - 1, 2), dtype=torch.int32, device="cuda"), cap)),
        dict(out=(ok_xyz.double(), ok_sides, cap)),
        dict(out=(ok_xyz, ok_sides.long(), cap)),
        dict(out=(ok_xyz.cpu(), ok_sides, cap)),
        dict(out=(torch.empty((3, 3, 2 * cap), dtype=torch.float32, device="cuda").transpose(0, 2), ok_sides, cap)),
        dict(out=(ok_xyz, ok_sides, -1)),
        dict(out=(ok_xyz, ok_sides, cap), row_offsets=offs.int()),
        dict(out=(ok_xyz, ok_sides, cap), row_offsets=offs[:-1]),
        dict(out=(ok_xyz, ok_sides, cap), row_offsets=offs.cpu()),
    ]
    for i, kw in enumerate(bad):
        kw.setdefault("row_offsets", offs)
        with pytest.raises(ValueError):
            plmss.marching_geometry(labels, 0, **kw)
            pytest.fail(f"case {i} was accepted")
    # a null output of either kind is allowed
    plmss.marching_geometry(labels, 0, row_offsets=offs, out=(None, ok_sides, cap))
    torch.cuda.synchronize()


def test_geometry_grids_without_cells(torch):
    for shape in [(1, 1, 1), (7,), (3, 4, 1), (4, 1, 4), (1, 6)]:
        labels = fields.random_labels(shape, 3, seed=2)
        xyz, sides, count = plmss.marching_geometry(_dev(torch, labels), 0)
        torch.cuda.synchronize()
        assert count == 0 and xyz.numel() == 0 and sides.numel() == 0


def _twelfths(a):
    k = np.rint(a.astype(np.float64) * 12).astype(np.int64)
    # every value is the float nearest to its twelfth
    np.testing.assert_array_equal(_bits(a), _bits((k / 12.0).astype(np.float32)))
    return k


@pytest.mark.parametrize("mode", [0, 1])
def test_geometry_full_size_sampled_rows(torch, mode):
    """512^3 region labels in the launch shape the measurement uses: the
    primitives of sampled rows equal the oracle's on the row's own
    2 x 2 x nx slab (shifted by the row's y, z; compared in exact twelfths,
    with every float checked to be the nearest to its twelfth)."""
    n = 512
    labels = fields.region_labels((n, n, n), seed=9)
    rows = (n - 1) * (n - 1)
    rng = np.random.Generator(np.random.PCG64(13))
    sample = sorted(set([0, n - 2, rows - 1] + rng.integers(0, rows, size=24).tolist()))
    d = _dev(torch, labels)
    _say(f"geometry 512^3 mode={mode}")
    _, offs = plmss.marching_index(d, mode)
    xyz, sides, count = plmss.marching_geometry(d, mode, row_offsets=offs)
    torch.cuda.synchronize()
    o = offs.cpu().numpy()
    assert count == o[-1]
    for r in sample:
        y, z = r % (n - 1), r // (n - 1)
        slab = oracle.marching_geometry(labels[z:z + 2, y:y + 2, :], mode)
        a, b = int(o[r]), int(o[r + 1])
        assert b - a == slab["count"], r
        got = xyz[a:b].cpu().numpy()
        want = _twelfths(slab["xyz"]) + 12 * np.array([0, y, z], np.int64)
        np.testing.assert_array_equal(_twelfths(got), want, err_msg=f"row {r}")
        np.testing.assert_array_equal(sides[a:b].cpu().numpy(), slab["sides"], err_msg=f"row {r}")


def test_extreme_label_values(torch):
    """Labels are compared for equality only: any int32 values, the extremes
    and negatives included, give the codes and primitives of their pattern."""
    vals = np.array([np.iinfo(np.int32).min, -1, 0, np.iinfo(np.int32).max], np.int32)
    for shape in [(4, 6, 70), (9, 65)]:
        labels = vals[fields.random_labels(shape, 4, seed=21)]
        for mode in (0, 1):
            _compare(torch, labels, mode, f"extremes {shape}")
            ref = _compare_geo(torch, labels, mode, f"extremes {shape}")
            assert set(np.unique(ref["sides"])) <= set(vals.tolist())


def test_geometry_long_rows_use_wide_coordinates(torch):
    """Rows longer than 2^27 vertices: twelfths of a coordinate no longer fit
    int32, the kernel takes its 64-bit path; labels vary only near the far end
    (a long 2-D strip, 2^27 + 200 vertices wide)."""
    nx = (1 << 27) + 200
    labels = np.zeros((2, nx), np.int32)
    labels[:, -150:] = fields.random_labels((2, 150), 3, seed=4)
    for mode in (0, 1):
        ref = oracle.marching_geometry(labels, mode)
        xyz, sides, count = plmss.marching_geometry(_dev(torch, labels), mode)
        torch.cuda.synchronize()
        assert count == ref["count"] > 0
        np.testing.assert_array_equal(_bits(xyz.cpu().numpy()), _bits(ref["xyz"]))
        np.testing.assert_array_equal(sides.cpu().numpy(), ref["sides"])
        assert ref["xyz"][:, :, 0].min() > (1 << 27) - 200


def test_geometry_union_of_ascending_and_descending(torch):
    f = fields.smoothed_noise((16, 30, 50), 1.5, seed=12)
    ref = oracle.segment(f)
    out = plmss.segment(_dev(torch, f))
    torch.cuda.synchronize()
    for mode in (0, 1):
        xyz, sides, ca, cd = plmss.marching_geometry_union(out["asc"], out["desc"], mode)
        torch.cuda.synchronize()
        ra, rd = oracle.marching_geometry(ref["asc"], mode), oracle.marching_geometry(ref["desc"], mode)
        assert (ca, cd) == (ra["count"], rd["count"])
        np.testing.assert_array_equal(_bits(xyz.cpu().numpy()), _bits(np.concatenate([ra["xyz"], rd["xyz"]])))
        np.testing.assert_array_equal(sides.cpu().numpy(), np.concatenate([ra["sides"], rd["sides"]]))
