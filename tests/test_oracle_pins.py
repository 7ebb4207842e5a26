"""Pins of the CPU oracle to facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: the paper's
worked examples (Fig. 1, Fig. 2), the cell totals printed in the caption of
Table 2, closed forms, and the independent brute force in ``bruteforce.py``.
"""
import ctypes
import json
import os

import numpy as np
import pytest

import oracle
from tests import bruteforce

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


# --- Fig. 1: the 4x4 worked example -------------------------------------------------

def test_fig1_wallmodes_labels():
    g = _golden("fig1_wallmodes.json")
    f = np.array(g["field"], np.float32).reshape(4, 4)
    r = oracle.segment(f)
    assert r["desc"].ravel().tolist() == g["desc"]
    assert r["asc"].ravel().tolist() == g["asc"]
    assert sorted(np.flatnonzero(r["desc"].ravel() == np.arange(16)).tolist()) == g["maxima"]
    assert sorted(np.flatnonzero(r["asc"].ravel() == np.arange(16)).tolist()) == g["minima"]
    assert r["n_min"] == 2 and r["n_max"] == 2 and r["K"] == g["K"]


def test_fig1_ms_partition_matches_figure_colours():
    g = _golden("fig1_wallmodes.json")
    f = np.array(g["field"], np.float32).reshape(4, 4)
    ms = oracle.segment(f)["ms"].ravel().tolist()
    # same region <=> same colour pair in panel (d)
    col = g["ms_colours"]
    for i in range(16):
        for j in range(16):
            assert (ms[i] == ms[j]) == (col[i] == col[j])
    assert ms == g["ms"]


def test_fig1_order_field_is_the_value_for_distinct_integers():
    g = _golden("fig1_wallmodes.json")
    f = np.array(g["field"], np.float32).reshape(4, 4)
    order, perm = oracle.order_field(f)
    assert order.ravel().tolist() == g["field"]  # values are a permutation of 0..15
    assert perm.tolist() == np.argsort(np.array(g["field"])).tolist()


# --- Fig. 2: path compression on a chain --------------------------------------------

def test_fig2_gradient_step_on_chain():
    g = _golden("fig2_path_compression.json")
    f = np.array(g["field"], np.float32)
    order, _ = oracle.order_field(f)
    up, dn = oracle.steepest(order)
    assert up.tolist() == g["gradient"]
    assert dn.tolist() == [0, 0, 1, 2, 3, 4, 5]


def test_fig2_iterations_and_converged_sets():
    g = _golden("fig2_path_compression.json")
    final, iters, hist = oracle.compress(np.array(g["gradient"]), descending=False, max_hist=8)
    assert iters == len(g["iterations"])
    assert [h.tolist() for h in hist] == g["iterations"]
    for h, conv in zip(hist, g["converged_after"]):
        got = [v for v in range(7) if h[v] == h[h[v]]]
        assert got == conv
    assert final.tolist() == [6] * 7


def test_fig2_decreasing_visit_order_finishes_in_one_iteration():
    g = _golden("fig2_path_compression.json")
    final, iters, _ = oracle.compress(np.array(g["gradient"]), descending=True)
    assert iters == g["descending_visit_iterations"]
    assert final.tolist() == [6] * 7


# --- Table 2 caption: cell totals of the triangulated grids -------------------------

@pytest.mark.parametrize("n,total", [(512, 3_473_956_851), (256, 432_287_731)])
def test_cell_totals_from_table2_caption(n, total):
    # Six tetrahedra per cube; a triangulated ball has Euler characteristic 1,
    # so V - E + F - T = 1 and V + E + F + T = 1 + 2E + 2T.
    t = 6 * (n - 1) ** 3
    two_e = total - 1 - 2 * t
    assert oracle.degree_sum(n, n, n) == two_e


def test_neighbourhood_matches_kuhn_simplices():
    for dims in [(4, 3, 5), (5, 4, 1), (6, 1, 1), (1, 5, 4), (3, 1, 4), (2, 2, 2)]:
        adj = bruteforce.kuhn_edges(*dims)
        for v in range(dims[0] * dims[1] * dims[2]):
            assert oracle.neighbours(*dims, v) == sorted(adj[v])
    assert max(len(oracle.neighbours(5, 5, 5, v)) for v in range(125)) == 14
    assert max(len(oracle.neighbours(5, 5, 1, v)) for v in range(25)) == 6


# --- brute force on tiny inputs ----------------------------------------------------

def _check_against_bruteforce(f):
    r = oracle.segment(f)
    asc, desc, ms, k = bruteforce.segment(f)
    np.testing.assert_array_equal(r["asc"], asc)
    np.testing.assert_array_equal(r["desc"], desc)
    np.testing.assert_array_equal(r["ms"], ms)
    assert r["K"] == k


def test_all_orderings_of_3x3_grid():
    perms, asc, desc, ms, k = bruteforce.grid3x3_all_orderings()
    # spot-check the vectorised brute force against the walking one
    for i in (0, 1, 1000, 123456, 362879):
        a2, d2, m2, k2 = bruteforce.segment(perms[i].astype(np.float32).reshape(3, 3))
        assert a2.ravel().tolist() == asc[i].tolist() and d2.ravel().tolist() == desc[i].tolist()
        assert m2.ravel().tolist() == ms[i].tolist() and k2 == k[i]
    for i in range(perms.shape[0]):
        r = oracle.segment(perms[i].astype(np.float32).reshape(3, 3))
        if (r["asc"].ravel() != asc[i]).any() or (r["desc"].ravel() != desc[i]).any() \
                or (r["ms"].ravel() != ms[i]).any() or r["K"] != k[i]:
            pytest.fail(f"ordering {perms[i].tolist()} differs")


@pytest.mark.parametrize("shape", [(3, 3, 3), (4, 3, 5), (5, 6, 4), (2, 7, 3), (8, 9, 10), (1, 6, 7), (9,), (5, 8)])
def test_random_fields_against_bruteforce(shape):
    rng = np.random.default_rng(sum(shape) * 7 + len(shape))
    _check_against_bruteforce(rng.standard_normal(shape).astype(np.float32))


def test_ties_against_bruteforce():
    rng = np.random.default_rng(11)
    for shape in [(4, 5, 6), (6, 7), (3, 3, 3), (20,)]:
        _check_against_bruteforce(rng.integers(0, 3, size=shape).astype(np.float32))
    _check_against_bruteforce(np.zeros((3, 4, 5), np.float32))


def test_signed_zero_subnormal_and_infinity_against_bruteforce():
    tiny = np.float32(1.4e-45)  # smallest subnormal
    vals = np.array([0.0, -0.0, tiny, -tiny, 2 * tiny, np.inf, -np.inf, 1.0, -1.0], np.float32)
    rng = np.random.default_rng(5)
    for shape in [(4, 5, 3), (7, 6), (3, 3, 3)]:
        _check_against_bruteforce(rng.choice(vals, size=shape))


# --- closed forms -------------------------------------------------------------------

@pytest.mark.parametrize("coef", [(1, 2, 3), (-1, 2, 0), (0, 0, 0), (0, -3, 1), (-2, -1, -1), (0, 1, 0)])
def test_linear_ramp_has_one_minimum_and_one_maximum(coef):
    nx, ny, nz = 7, 5, 4
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx]
    f = (coef[0] * x + coef[1] * y + coef[2] * z).astype(np.float32)  # small integers: exact
    r = oracle.segment(f)
    assert r["n_min"] == 1 and r["n_max"] == 1 and r["K"] == 1
    n = (nx, ny, nz)
    # highest corner: far end along rising axes and (by the index tie-break)
    # along flat ones; lowest corner symmetrically
    hi = [n[a] - 1 if coef[a] >= 0 else 0 for a in range(3)]
    lo = [0 if coef[a] >= 0 else n[a] - 1 for a in range(3)]
    vid = lambda p: p[0] + nx * (p[1] + ny * p[2])  # noqa: E731
    assert (r["desc"] == vid(hi)).all() and (r["asc"] == vid(lo)).all()


def test_constant_field():
    r = oracle.segment(np.full((3, 4, 5), 2.5, np.float32))
    assert (r["asc"] == 0).all() and (r["desc"] == 59).all() and r["K"] == 1


@pytest.mark.parametrize("dims,centre,sigma", [((17, 13), (7.3, 5.2), 4.0), ((11, 9, 8), (4.2, 3.7, 5.4), 3.0),
                                               ((9, 12, 10), (6.9, 2.3, 4.1), 5.0)])
def test_single_gaussian(dims, centre, sigma):
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in dims], indexing="ij")
    r2 = sum((g - c) ** 2 for g, c in zip(grids, centre))
    f = np.exp(-r2 / (2 * sigma * sigma)).astype(np.float32)
    assert f.min() > np.finfo(np.float32).tiny
    f = np.ascontiguousarray(np.transpose(f))  # axis order (.., y, x): x fastest
    r = oracle.segment(f)
    d = len(dims)
    near = [int(round(c)) for c in centre]
    strides = [1, dims[0], dims[0] * (dims[1] if d > 1 else 1)]
    near_id = sum(p * s for p, s in zip(near, strides))
    assert r["n_max"] == 1 and (r["desc"] == near_id).all()
    assert r["n_min"] == 2 ** d and r["K"] == 2 ** d
    corners = set()
    for bits in range(2 ** d):
        p = [(dims[a] - 1) if (bits >> a) & 1 else 0 for a in range(d)]
        corners.add(sum(pi * s for pi, s in zip(p, strides)))
    assert set(np.unique(r["asc"]).tolist()) == corners


@pytest.mark.parametrize("k,period", [((2, 3), 7), ((3, 3), 5), ((1, 2, 2), 7), ((2, 2, 2), 5), ((3, 1, 2), 9)])
def test_cosine_product_extremum_counts(k, period):
    axes = [np.cos(np.pi * np.arange(ki * period + 1) / period) for ki in k]
    f = axes[0]
    for a in axes[1:]:
        f = np.multiply.outer(f, a)
    f = np.ascontiguousarray(np.transpose(f)).astype(np.float32)
    r = oracle.segment(f)
    # extrema sit at the lattice points (m_1 P, m_2 P, ...); sign (-1)^(sum m)
    pts = list(np.ndindex(*[ki + 1 for ki in k]))
    n_pos = sum(1 for m in pts if sum(m) % 2 == 0)
    assert r["n_max"] == n_pos and r["n_min"] == len(pts) - n_pos


def test_monotone_line():
    for n in (1, 2, 7, 1000):
        r = oracle.segment(np.arange(n, dtype=np.float32))
        assert (r["asc"] == 0).all() and (r["desc"] == n - 1).all() and r["K"] == 1


def test_single_vertex():
    r = oracle.segment(np.array([3.0], np.float32))
    assert r["asc"].tolist() == [0] and r["desc"].tolist() == [0] and r["ms"].tolist() == [0] and r["K"] == 1


# --- invariants ---------------------------------------------------------------------

def _field(shape, seed):
    from paper_2303_15491_amd import fields
    return fields.smoothed_noise(shape, 1.5, seed)


@pytest.mark.parametrize("shape", [(12, 13, 14), (40, 37), (5, 1, 9)])
def test_invariants(shape):
    f = _field(shape, 21)
    r = oracle.segment(f)
    asc, desc, up, dn, ms = (r[k].ravel() for k in ("asc", "desc", "up", "dn", "ms"))
    assert (asc[asc] == asc).all() and (desc[desc] == desc).all()
    assert (desc == desc[up]).all() and (asc == asc[dn]).all()
    assert r["n_max"] == int((desc == np.arange(f.size)).sum())
    pairs = asc.astype(np.int64) * f.size + desc
    _, inv = np.unique(pairs, return_inverse=True)
    assert (inv.ravel() == ms).all()
    assert r["K"] <= r["n_min"] * r["n_max"]


def test_widening_scaling_and_negation():
    f = _field((10, 11, 12), 22)
    r = oracle.segment(f)
    r64 = oracle.segment(f.astype(np.float64))
    r2 = oracle.segment(f * np.float32(2))
    rn = oracle.segment(-f)
    assert len(np.unique(f)) == f.size  # tie-free
    for k in ("order", "asc", "desc", "ms"):
        np.testing.assert_array_equal(r[k], r64[k])
        np.testing.assert_array_equal(r[k], r2[k])
    np.testing.assert_array_equal(rn["asc"], r["desc"])
    np.testing.assert_array_equal(rn["desc"], r["asc"])


def test_degenerate_dims_agree():
    f2 = _field((9, 10), 23)
    a = oracle.segment(f2)
    b = oracle.segment(f2.reshape(1, 9, 10))
    for k in ("asc", "desc", "ms"):
        np.testing.assert_array_equal(a[k].ravel(), b[k].ravel())
    f1 = _field((30,), 24)
    c = oracle.segment(f1)
    d = oracle.segment(f1.reshape(1, 1, 30))
    for k in ("asc", "desc", "ms"):
        np.testing.assert_array_equal(c[k].ravel(), d[k].ravel())


def test_labels_equal_papers_path_compression_fixed_point():
    for seed, shape in [(31, (9, 8, 7)), (32, (25, 30)), (33, (100,))]:
        f = _field(shape, seed)
        r = oracle.segment(f)
        for desc_order in (False, True):
            d, _, _ = oracle.compress(r["up"], descending=desc_order)
            a, _, _ = oracle.compress(r["dn"], descending=desc_order)
            np.testing.assert_array_equal(d, r["desc"].ravel())
            np.testing.assert_array_equal(a, r["asc"].ravel())


def test_labels_equal_integral_line_walk():
    f = _field((14, 15, 16), 34)
    r = oracle.segment(f)
    rng = np.random.default_rng(0)
    for v in rng.integers(0, f.size, 200):
        mx, mn, _, _ = oracle.trace(f, int(v))
        assert mx == r["desc"].ravel()[v] and mn == r["asc"].ravel()[v]


def test_order_field_is_sorted_position():
    f = np.random.default_rng(3).integers(0, 5, size=(4, 5, 6)).astype(np.float32)
    order, perm = oracle.order_field(f)
    flat = f.ravel()
    expect = sorted(range(flat.size), key=lambda v: (float(flat[v]), v))
    assert perm.tolist() == expect
    assert (order.ravel()[perm] == np.arange(flat.size)).all()


# --- argument validation ------------------------------------------------------------

def test_nan_is_rejected():
    f = np.zeros((3, 3), np.float32)
    f[1, 2] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.segment(f)
    assert e.value.code == oracle.E_NAN


def test_bad_and_too_large_dims():
    lib = oracle._load()
    f = np.zeros(4, np.float32)
    out = [np.zeros(4, np.int32) for _ in range(3)]
    p = [o.ctypes.data_as(ctypes.c_void_p) for o in out]
    fp = f.ctypes.data_as(ctypes.c_void_p)
    assert lib.plmss_oracle_segment(fp, 0, 0, 1, 1, None, None, None, *p, None) == oracle.E_DIMS
    assert lib.plmss_oracle_segment(fp, 0, 2048, 2048, 513, None, None, None, *p, None) == oracle.E_TOO_LARGE
    assert lib.plmss_oracle_segment(fp, 2, 4, 1, 1, None, None, None, *p, None) == oracle.E_ARG
