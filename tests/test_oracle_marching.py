"""Pins of the oracle's multi-label marching index (Sec. "Multi-Label Marching
Triangles/Tetrahedra") against the paper's code table, decision tree and case
figures, closed forms and a row-by-row recount.  CPU only."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")
TET = json.load(open(os.path.join(GOLD, "tet_binary_codes.json")))
TRI = json.load(open(os.path.join(GOLD, "triangle_codes.json")))

# the six Kuhn tetrahedra of a cube: vertex positions along the axis order
PERMS3 = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def tet_vertices(perm):
    p = [0, 0, 0]
    out = [tuple(p)]
    for axis in perm:
        p[axis] += 1
        out.append(tuple(p))
    return out  # (x, y, z) offsets, increasing vertex id


def same_pattern(u, v):
    return all((u[i] == u[j]) == (v[i] == v[j]) for i in range(len(u)) for j in range(len(u)))


def table_row(labels4):
    rows = [r for r in TET["rows"] if same_pattern(r["abcd"], labels4)]
    assert len(rows) == 1, labels4
    return rows[0]


def test_table_rows_are_the_fifteen_patterns():
    # every equality pattern of four labels (the 15 set partitions) has one row
    pats = {tuple(r["abcd"]) for r in TET["rows"]}
    assert len(pats) == 15
    for lab in itertools.product(range(4), repeat=4):
        table_row(lab)


def test_cube_codes_and_counts_exhaustive():
    """Every labeling of one cube with labels 0..3: each tetrahedron's code is
    the table row of its equality pattern, and the totals are the figure's
    triangle counts (separators) and the three-of-a-kind tetrahedra
    (boundaries) summed over the six tetrahedra."""
    seen = set()
    for lab8 in itertools.product(range(4), repeat=8):
        cube = np.array(lab8, np.int32).reshape(2, 2, 2)  # [z][y][x]
        sep = oracle.marching(cube, 0)
        bnd = oracle.marching(cube, 1, with_codes=False)
        want_sep = want_bnd = 0
        for t, perm in enumerate(PERMS3):
            labels4 = [int(cube[z, y, x]) for (x, y, z) in tet_vertices(perm)]
            row = table_row(labels4)
            assert sep["codes"][t] == row["code"], (lab8, t)
            seen.add(row["code"])
            want_sep += row["separators"]
            counts = [labels4.count(v) for v in set(labels4)]
            want_bnd += 1 if sorted(counts) == [1, 3] else 0
        assert sep["total"] == want_sep and bnd["total"] == want_bnd, lab8
    assert seen == {r["code"] for r in TET["rows"]}


def tree_code(a, b, c):
    if a == b:
        return TRI["tree"]["a==b"]["a==c"] if a == c else TRI["tree"]["a==b"]["else"]
    if a == c:
        return TRI["tree"]["else"]["a==c"]
    return TRI["tree"]["else"]["else"]["b==c"] if b == c else TRI["tree"]["else"]["else"]["else"]


def test_square_codes_follow_the_decision_tree():
    for lab4 in itertools.product(range(3), repeat=4):
        sq = np.array(lab4, np.int32).reshape(2, 2)  # [y][x]
        out = oracle.marching(sq, 0)
        bnd = oracle.marching(sq, 1, with_codes=False)
        tris = [[(0, 0), (1, 0), (1, 1)], [(0, 0), (0, 1), (1, 1)]]  # x first, y first
        want = want_b = 0
        for t, verts in enumerate(tris):
            a, b, c = (int(sq[y, x]) for (x, y) in verts)
            code = tree_code(a, b, c)
            assert out["codes"][t] == code, (lab4, t)
            want += TRI["separators"][str(code)]
            want_b += 1 if len({a, b, c}) == 2 else 0
        assert out["total"] == want and bnd["total"] == want_b


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_step_interface_closed_form(axis):
    """A step in one axis crosses one layer of cubes; with the Kuhn cut every
    crossing cube holds two tetrahedra of each position of the step along
    its path: 2*1 + 2*2 + 2*1 = 8 separating triangles and 4 boundary
    triangles."""
    shape = (6, 5, 7)  # nz, ny, nx
    z, y, x = np.indices(shape)
    coord = (x, y, z)[axis]
    lab = (coord >= 3).astype(np.int32)
    n_other = np.prod([s - 1 for i, s in enumerate((7, 5, 6)) if i != axis])
    assert oracle.marching(lab, 0)["total"] == 8 * n_other
    assert oracle.marching(lab, 1)["total"] == 4 * n_other


def test_constant_and_all_distinct():
    shape = (4, 5, 6)
    cubes = 3 * 4 * 5
    assert oracle.marching(np.full(shape, 7, np.int32), 0)["total"] == 0
    ids = np.arange(np.prod(shape), dtype=np.int32).reshape(shape)
    assert oracle.marching(ids, 0)["total"] == 12 * 6 * cubes
    assert oracle.marching(ids, 1)["total"] == 0
    ids2 = np.arange(30, dtype=np.int32).reshape(5, 6)
    assert oracle.marching(ids2, 0)["total"] == 3 * 2 * 4 * 5


def test_degenerate_dims_have_no_cells():
    for shape in [(9,), (3, 1, 7), (4, 6, 1), (1, 5)]:
        out = oracle.marching(np.zeros(shape, np.int32), 0)
        assert out["rows"] == 0 and out["total"] == 0 and list(out["row_offsets"]) == [0]


def test_row_offsets_recount_rows_one_by_one():
    """Each row's count, recounted on the 2 x 2 x nx slab that holds it, gives
    the differences of row_offsets."""
    rng = np.random.default_rng(3)
    lab = rng.integers(0, 3, size=(4, 5, 9)).astype(np.int32)
    out = oracle.marching(lab, 0)
    offs = out["row_offsets"]
    nz, ny, nx = lab.shape
    for r in range(out["rows"]):
        y, z = r % (ny - 1), r // (ny - 1)
        slab = np.ascontiguousarray(lab[z:z + 2, y:y + 2, :])
        assert oracle.marching(slab, 0)["total"] == offs[r + 1] - offs[r]
