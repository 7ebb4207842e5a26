"""GPU parity of the batched path: many fields of different sizes and shapes
in one pass (and through replayable capacity plans) give, field by field, the
oracle's labels, bit for bit, whatever their neighbours in the batch."""
import sys

import numpy as np
import pytest

import oracle
import paper_2303_15491_amd as plmss
from paper_2303_15491_amd import fields
from tests import bruteforce

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


def _mixed_fields(seed=0):
    rng = np.random.default_rng(seed)
    shapes = [(20, 30, 70), (9, 8, 130), (50, 60), (300,), (16, 8, 64), (2, 2, 2), (1,), (1, 33), (33, 1, 17),
              (5, 77, 1), (3, 3), (40, 41, 42)]
    out = []
    for i, sh in enumerate(shapes):
        if len(sh) == 1 and sh[0] == 1:
            out.append(np.array([0.5], np.float32))
        else:
            out.append(fields.smoothed_noise(sh, float(rng.uniform(1.0, 2.5)), seed=100 + i))
    return out


def _check_one(f, o, label):
    ref = oracle.segment(f)
    info = o["info"].cpu().numpy()
    assert info[0] == 0, label
    for k in ("asc", "desc", "ms"):
        np.testing.assert_array_equal(o[k].cpu().numpy(), ref[k], err_msg=f"{label} {k}")
    assert (info[1], info[2], info[3]) == (ref["n_min"], ref["n_max"], ref["K"]), label


def test_batch_matches_oracle(torch):
    fs = _mixed_fields()
    _say(f"batch of {len(fs)} mixed fields")
    outs = plmss.segment_batch([torch.from_numpy(f).cuda() for f in fs])
    torch.cuda.synchronize()
    for i, (f, o) in enumerate(zip(fs, outs)):
        _check_one(f, o, f"field {i} {f.shape}")


@pytest.mark.parametrize("pair_stream", [0, 1])
def test_batch_pair_sort_cached_or_streamed(torch, pair_stream):
    """The batch's pair sort streams its loads by default; the cached form
    (and the forced streamed form) give the same labels."""
    saved = plmss.tune_get()
    try:
        plmss.tune_set(pair_stream=pair_stream)
        fs = _mixed_fields(seed=3)
        _say(f"batch pair_stream={pair_stream}")
        outs = plmss.segment_batch([torch.from_numpy(f).cuda() for f in fs])
        torch.cuda.synchronize()
        for i, (f, o) in enumerate(zip(fs, outs)):
            _check_one(f, o, f"pair_stream {pair_stream} field {i} {f.shape}")
    finally:
        plmss.tune_set(**saved)


def test_batch_isolation_position_and_neighbours(torch):
    fs = _mixed_fields(1)
    target = fields.smoothed_noise((24, 33, 65), 1.5, seed=7)
    alone = plmss.segment(torch.from_numpy(target).cuda())
    for pos in (0, 5, len(fs)):
        _say(f"isolation pos={pos}")
        batch = fs[:pos] + [target] + fs[pos:]
        outs = plmss.segment_batch([torch.from_numpy(f).cuda() for f in batch])
        torch.cuda.synchronize()
        for k in ("asc", "desc", "ms", "info"):
            assert torch.equal(outs[pos][k], alone[k]), (pos, k)


def test_batch_nan_stays_in_its_field(torch):
    fs = _mixed_fields(2)
    bad = fs[4].copy()
    bad.ravel()[17] = np.nan
    fs[4] = bad
    _say("batch with a NaN field")
    outs = plmss.segment_batch([torch.from_numpy(f).cuda() for f in fs])
    torch.cuda.synchronize()
    for i, (f, o) in enumerate(zip(fs, outs)):
        if i == 4:
            assert int(o["info"][0]) == plmss.E_NAN
        else:
            _check_one(f, o, f"field {i}")


def test_batch_float64(torch):
    fs = [f.astype(np.float64) for f in _mixed_fields(3)[:6]]
    _say("float64 batch")
    outs = plmss.segment_batch([torch.from_numpy(f).cuda() for f in fs])
    torch.cuda.synchronize()
    for i, (f, o) in enumerate(zip(fs, outs)):
        _check_one(f, o, f"f64 field {i}")


def test_uneven_batch_members(torch):
    shapes = fields.batch_shapes(64, seed=4, lo=32, hi=192)[:6]
    small = [tuple(max(8, s // 3) for s in sh) for sh in shapes]
    fs = [fields.gaussian_blobs(sh, seed=4 + j) for j, sh in enumerate(small)]
    _say(f"uneven batch {small}")
    outs = plmss.segment_batch([torch.from_numpy(f).cuda() for f in fs])
    torch.cuda.synchronize()
    for i, (f, o) in enumerate(zip(fs, outs)):
        _check_one(f, o, f"uneven {i} {f.shape}")


def test_plan_graph_replays_different_batches(torch):
    a = _mixed_fields(4)
    b = [fields.smoothed_noise((30, 20, 10), 1.5, seed=9), fields.smoothed_noise((64, 64), 2.0, seed=10),
         fields.smoothed_noise((7, 70, 9), 1.2, seed=11)]
    da = [torch.from_numpy(f).cuda() for f in a]
    db = [torch.from_numpy(f).cuda() for f in b]
    need = [max(x, y) for x, y in zip(plmss.batch_needs(da), plmss.batch_needs(db))]
    plan = plmss.Plan(need[0] + 1000, need[1] + 2, need[2] + 10, need[3] + 10)
    for rnd, (fs, ds) in enumerate([(a, da), (b, db), (a, da), (b, db)]):
        _say(f"plan replay {rnd}")
        outs = plan.set(ds)
        plan.launch(graph=True)
        torch.cuda.synchronize()
        for i, (f, o) in enumerate(zip(fs, outs)):
            _check_one(f, o, f"replay {rnd} field {i}")
        # eager work between replays
        plmss.segment(da[0])
        torch.cuda.synchronize()
    outs = plan.set(db)
    plan.launch(graph=False)
    torch.cuda.synchronize()
    for i, (f, o) in enumerate(zip(b, outs)):
        _check_one(f, o, f"eager plan field {i}")
    plan.close()


def test_plan_rejects_batches_beyond_capacity(torch):
    plan = plmss.Plan(1000, 2, 4, 4)
    with pytest.raises(plmss.PlmssError) as e:
        plan.set([torch.zeros(20, 20, 20, device="cuda")])
    assert e.value.code == plmss.E_TOO_LARGE
    plan.close()


def test_grid3x3_orderings_in_one_batch(torch):
    perms, asc, desc, ms, k = bruteforce.grid3x3_all_orderings()
    rng = np.random.default_rng(3)
    pick = rng.choice(perms.shape[0], 4000, replace=False)
    fs = [torch.from_numpy(perms[i].astype(np.float32).reshape(3, 3)).cuda() for i in pick]
    _say("3x3 orderings batch")
    outs = plmss.segment_batch(fs)
    torch.cuda.synchronize()
    for j, i in enumerate(pick):
        o = outs[j]
        assert o["asc"].cpu().numpy().ravel().tolist() == asc[i].tolist()
        assert o["desc"].cpu().numpy().ravel().tolist() == desc[i].tolist()
        assert o["ms"].cpu().numpy().ravel().tolist() == ms[i].tolist()
        assert int(o["info"][3]) == k[i]


def _oracle_all(host_fields):
    """Oracle segmentations of many fields, computed in parallel host threads
    (each oracle call runs in C without the interpreter lock)."""
    import concurrent.futures
    import os

    workers = max(1, min(16, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        return list(ex.map(oracle.segment, host_fields))


@pytest.mark.timeout(900)
def test_full_uneven_batch_graph_against_oracle(torch):
    """The whole 64-field uneven batch (sides 32..192, 16..256 Gaussians plus
    noise) through a capacity plan replayed as a hipGraph, with the persistent
    grid the batched measurement runs with, against the oracle field by field."""
    saved = plmss.tune_get()
    try:
        plmss.tune_set(persist_blocks=4096)
        _say("c4 generate")
        host = fields.batch_fields(64, seed=4)
        dev = [torch.from_numpy(f).cuda() for f in host]
        plan = plmss.Plan(*plmss.batch_needs(dev))
        _say("c4 plan launch (graph), twice")
        outs = plan.set(dev)
        plan.launch(graph=True)
        plan.set(dev, outs=outs)
        plan.launch(graph=True)
        torch.cuda.synchronize()
        _say("c4 oracle")
        refs = _oracle_all(host)
        for i, (ref, o) in enumerate(zip(refs, outs)):
            info = o["info"].cpu().numpy()
            assert info[0] == 0, i
            for k in ("asc", "desc", "ms"):
                np.testing.assert_array_equal(o[k].cpu().numpy(), ref[k], err_msg=f"c4 field {i} {k}")
            assert (info[1], info[2], info[3]) == (ref["n_min"], ref["n_max"], ref["K"]), i
        plan.close()
    finally:
        plmss.tune_set(**saved)


def _check_with_order(f, o, label):
    ref = oracle.segment(f)
    info = o["info"].cpu().numpy()
    assert info[0] == 0, label
    for k in ("asc", "desc", "ms", "order"):
        if k == "order" and o.get("order") is None:
            continue
        np.testing.assert_array_equal(o[k].cpu().numpy(), ref[k], err_msg=f"{label} {k}")
    assert (info[1], info[2], info[3]) == (ref["n_min"], ref["n_max"], ref["K"]), label


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_batch_order_fields_match_oracle(torch, dtype):
    """Order fields in a batch (Sec. "Preprocessing", per field): jobs with
    and without an order array side by side, of every shape class, with ties
    and special values in one field; each order field equals the oracle's."""
    fs = [f.astype(dtype) for f in _mixed_fields(5)]
    rng = np.random.default_rng(21)
    fs[2] = rng.integers(0, 3, size=fs[2].shape).astype(dtype)  # heavy ties
    fs[6] = np.array([np.inf], dtype)
    dev = [torch.from_numpy(f).cuda() for f in fs]
    outs = plmss._outs_for(dev, with_order=True)
    for i in (1, 4, 9):
        outs[i].pop("order")  # these jobs ask for no order field
    _say(f"batch with order fields {np.dtype(dtype).name}")
    plmss.segment_batch(dev, outs=outs)
    torch.cuda.synchronize()
    for i, (f, o) in enumerate(zip(fs, outs)):
        _check_with_order(f, o, f"order batch field {i} {f.shape}")


def test_batch_order_fields_many_fields(torch):
    """More than 256 fields: the field index takes two digits of the sort."""
    rng = np.random.default_rng(22)
    fs = []
    for i in range(300):
        sh = [(3, 3), (2, 3, 4), (5,), (4, 4)][i % 4]
        fs.append(rng.standard_normal(sh).astype(np.float32))
    dev = [torch.from_numpy(f).cuda() for f in fs]
    _say("batch of 300 fields with order")
    outs = plmss.segment_batch(dev, with_order=True)
    torch.cuda.synchronize()
    for i, (f, o) in enumerate(zip(fs, outs)):
        _check_with_order(f, o, f"many-field batch {i}")


def test_batch_order_nan_stays_in_its_field(torch):
    fs = _mixed_fields(6)
    bad = fs[3].copy()
    bad.ravel()[2] = np.nan
    fs[3] = bad
    _say("order batch with a NaN field")
    outs = plmss.segment_batch([torch.from_numpy(f).cuda() for f in fs], with_order=True)
    torch.cuda.synchronize()
    for i, (f, o) in enumerate(zip(fs, outs)):
        if i == 3:
            assert int(o["info"][0]) == plmss.E_NAN
        else:
            _check_with_order(f, o, f"order batch field {i}")


def test_plan_graph_with_order_fields(torch):
    """A plan that builds order fields, replayed through its hipGraph for two
    different batches in turn (A, B, A, B) with eager work in between."""
    a = _mixed_fields(7)
    b = [fields.smoothed_noise((30, 20, 10), 1.5, seed=19), fields.smoothed_noise((64, 64), 2.0, seed=20),
         fields.smoothed_noise((7, 70, 9), 1.2, seed=21)]
    da = [torch.from_numpy(f).cuda() for f in a]
    db = [torch.from_numpy(f).cuda() for f in b]
    need = [max(x, y) for x, y in zip(plmss.batch_needs(da), plmss.batch_needs(db))]
    plan = plmss.Plan(need[0] + 5000, need[1] + 2, need[2] + 10, need[3] + 10, with_order=True)
    for rnd, (fs, ds) in enumerate([(a, da), (b, db), (a, da), (b, db)]):
        _say(f"order plan replay {rnd}")
        outs = plan.set(ds)
        plan.launch(graph=True)
        torch.cuda.synchronize()
        for i, (f, o) in enumerate(zip(fs, outs)):
            _check_with_order(f, o, f"order replay {rnd} field {i}")
        plmss.segment(da[0], with_order=True)
        torch.cuda.synchronize()
    plan.close()
    plain = plmss.Plan(need[0], need[1], need[2], need[3])
    with pytest.raises(plmss.PlmssError) as e:
        plain.set(da, outs=plmss._outs_for(da, with_order=True))
    assert e.value.code == plmss.E_ARG
    plain.close()


def test_plan_beyond_2_30_vertices_takes_the_wide_id_path(torch):
    """A plan sized for more than 2^30 vertices numbers its launch's vertices
    with 31-bit ids, so its cross-tile chase addresses the pointer arrays with
    64-bit offsets (the path that launches below 2^30 vertices never take).
    Small fields through such a plan, graph-launched and eager, still give the
    oracle's labels bit for bit.  (Its workspace is tens of GB: sized for the
    capacity, not the batch.)"""
    fs = [fields.smoothed_noise((40, 33, 29), 1.5, seed=71), fields.smoothed_noise((17, 64), 1.2, seed=72),
          fields.smoothed_noise((300,), 2.0, seed=73), fields.gaussian_blobs((24, 40, 31), seed=74)]
    ds = [torch.from_numpy(f).cuda() for f in fs]
    need = plmss.batch_needs(ds)
    _say("plan with capacity 2^30 + 4096 vertices")
    plan = plmss.Plan((1 << 30) + 4096, need[1] + 2, need[2] + 10, need[3] + 10)
    try:
        for graph in (True, False):
            outs = plan.set(ds)
            plan.launch(graph=graph)
            torch.cuda.synchronize()
            for i, (f, o) in enumerate(zip(fs, outs)):
                _check_one(f, o, f"wide-id plan (graph={graph}) field {i} {f.shape}")
    finally:
        plan.close()
        del plan
        torch.cuda.empty_cache()
