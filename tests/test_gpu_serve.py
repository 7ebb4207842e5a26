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


def test_served_results_equal_alone_results(torch):
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
    reqs[11] = reqs[11].copy()
    reqs[11].ravel()[5] = np.nan
    trace = [{"t": 0.0005 * i} for i in range(len(reqs))]
    budget = 3 * max(r.size for r in reqs) * 16
    server = Server(budget_bytes=budget, max_batch_vertices=1 << 18, max_batch_fields=8, keep_results=True)
    peak = [0]
    orig_admit = server._admit

    def admit():
        orig_admit()
        peak[0] = max(peak[0], server.resident)

    server._admit = admit
    done = run_trace(server, trace, lambda i, r: reqs[i], realtime=True)
    assert peak[0] <= budget
    assert len(server.done) == len(reqs)
    for i, r in enumerate(done):
        alone = plmss.segment(torch.from_numpy(reqs[i]).cuda())
        torch.cuda.synchronize()
        if i == 11:
            assert int(r.out["info"][0]) == plmss.E_NAN
            continue
        for k in ("asc", "desc", "ms", "info"):
            assert torch.equal(r.out[k], alone[k]), (i, k)
    st = server.stats()
    assert st["requests"] == len(reqs) and st["p99_ms"] >= st["p50_ms"] > 0
    server.close()
