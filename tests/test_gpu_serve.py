"""The serving loop: every request's labels are the same alone and in the
mix (tolerance 0), and admission never exceeds the memory budget."""
import sys

import numpy as np
import pytest

import paper_2303_15491_amd as plmss
from paper_2303_15491_amd import fields

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t

    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


# request sizes of the serving workload (2-D n^2, n in 128..2048; 3-D n^3, n
# in 64..384): its largest of each kind and some in between
SERVING_SIZES = [(2048, 2048), (384, 384, 384), (1024, 1024), (256, 256, 256), (128, 128), (64, 64, 64),
                 (700, 700), (160, 170, 180)]


def _oracle_all(host_fields):
    import concurrent.futures
    import os

    import oracle

    workers = max(1, min(16, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        return list(ex.map(oracle.segment, host_fields))


@pytest.mark.timeout(900)
def test_served_results_equal_alone_results(torch):
    """Small requests and requests of the serving workload's sizes, mixed
    and overlapping on the device: every served result equals the oracle's
    and the same field segmented alone (tolerance 0)."""
    from paper_2303_15491_amd.serve import Server, run_trace

    print("[gpu-case] serving mix", flush=True)
    sys.stdout.flush()
    rng = np.random.default_rng(8)
    reqs = []
    for i in range(40):
        if i % 2:
            n = int(rng.integers(16, 120))
            reqs.append(fields.smoothed_noise((n, n), float(rng.uniform(1.5, 4)), seed=300 + i))
        else:
            n = int(rng.integers(8, 40))
            reqs.append(fields.smoothed_noise((n, n + 3, n + 1), float(rng.uniform(1.5, 4)), seed=300 + i))
    for j, sh in enumerate(SERVING_SIZES):
        reqs.insert(3 + 4 * j, fields.smoothed_noise(sh, float(rng.uniform(1.5, 4)), seed=400 + j))
    nan_at = 11
    reqs[nan_at] = reqs[nan_at].copy()
    reqs[nan_at].ravel()[5] = np.nan
    trace = [{"t": 0.0005 * i} for i in range(len(reqs))]
    big = max(r.size for r in reqs)
    budget = 3 * big * 16
    server = Server(budget_bytes=budget, max_batch_vertices=big + (1 << 18), max_batch_fields=8,
                    keep_results=True)
    peak = [0]
    orig_admit = server._admit

    def admit():
        orig_admit()
        peak[0] = max(peak[0], server.resident)

    server._admit = admit
    done = run_trace(server, trace, lambda i, r: reqs[i], realtime=True)
    assert peak[0] <= budget
    assert len(server.done) == len(reqs)
    print("[gpu-case] serving mix: oracle", flush=True)
    refs = _oracle_all([r for i, r in enumerate(reqs) if i != nan_at])
    refs.insert(nan_at, None)
    for i, r in enumerate(done):
        alone = plmss.segment(torch.from_numpy(reqs[i]).cuda())
        torch.cuda.synchronize()
        if i == nan_at:
            assert int(r.out["info"][0]) == plmss.E_NAN
            continue
        for k in ("asc", "desc", "ms", "info"):
            assert torch.equal(r.out[k], alone[k]), (i, k)
        ref = refs[i]
        info = r.out["info"].cpu().numpy()
        assert info[0] == 0 and (info[1], info[2], info[3]) == (ref["n_min"], ref["n_max"], ref["K"]), i
        for k in ("asc", "desc", "ms"):
            np.testing.assert_array_equal(r.out[k].cpu().numpy(), ref[k], err_msg=f"request {i} {k}")
        r.out = None
        del alone
    st = server.stats()
    assert st["requests"] == len(reqs) and st["p99_ms"] >= st["p50_ms"] > 0
    server.close()
