"""Autotuner: cache keys and storage on the CPU; on the GPU, every candidate
launch shape reproduces the labels exactly (the tuner checks each one)."""
import json

import numpy as np
import pytest

import paper_2303_15491_amd as plmss
from paper_2303_15491_amd import autotune, fields


def test_cache_key_buckets():
    assert autotune.cache_key("gfx950", "f32", "segment", 3, 512 ** 3) == "gfx950|f32|segment|3d|2^27"
    assert autotune.cache_key("gfx950", "f32", "batch", 3, 95_834_117).endswith("2^27")
    assert autotune.cache_key("gfx950", "f64", "segment", 2, 1) == "gfx950|f64|segment|2d|2^0"


def test_cache_store_lookup_apply(tmp_path, monkeypatch):
    monkeypatch.setenv("PLMSS_TUNE_CACHE", str(tmp_path / "tune.json"))
    saved = plmss.tune_get()
    try:
        assert autotune.lookup("k") is None and not autotune.apply("k")
        autotune._store("k", {"scan_depth": 8, "sort_workers": 512})
        autotune._store("j", {"persist_blocks": 4096})
        data = json.loads((tmp_path / "tune.json").read_text())
        assert set(data) == {"k", "j"}
        assert autotune.lookup("k") == {"scan_depth": 8, "sort_workers": 512}
        assert autotune.apply("k")
        assert plmss.tune_get()["scan_depth"] == 8 and plmss.tune_get()["sort_workers"] == 512
    finally:
        plmss.tune_set(**saved)


def test_search_space_is_valid():
    saved = plmss.tune_get()
    try:
        for knob, values in autotune.SPACE.items():
            for v in values:
                plmss.tune_set(**{knob: v})
    finally:
        plmss.tune_set(**saved)


@pytest.mark.gpu
def test_tuner_candidates_reproduce_labels(tmp_path, monkeypatch):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    monkeypatch.setenv("PLMSS_TUNE_CACHE", str(tmp_path / "tune.json"))
    saved = plmss.tune_get()
    try:
        print("[gpu-case] autotune segment 70x90x130 with order", flush=True)
        f = torch.from_numpy(fields.smoothed_noise((70, 90, 130), 1.5, seed=11)).cuda()
        r = autotune.tune_segment(f, with_order=True, reps=1)
        assert not r["cached"] and r["trials"] > 10
        assert autotune.tune_segment(f, with_order=True)["cached"]
        print("[gpu-case] autotune batch of 6", flush=True)
        batch = [torch.from_numpy(x).cuda() for x in fields.batch_fields(6, seed=9, lo=20, hi=70)]
        batch.append(torch.from_numpy(fields.gaussian_mix_2d(100, seed=3)).cuda())
        rb = autotune.tune_batch(batch, reps=1)
        assert rb["trials"] > 5
        for k, v in rb["knobs"].items():
            assert v in autotune.SPACE[k]
    finally:
        plmss.tune_set(**saved)
