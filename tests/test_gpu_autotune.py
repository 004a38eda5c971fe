"""The autotuner: every candidate gives identical masks, the winner is one of
them, and the cache is reused."""
import json

import numpy as np
import pytest

from paper_1903_12294_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_tune_plain_and_cache(tmp_path, monkeypatch):
    from paper_1903_12294_amd import autotune
    _need_gpu()
    monkeypatch.setenv("MF4D_TUNE_CACHE", str(tmp_path / "tune.json"))
    inst = synth.make_config(1, attr_mode="noise")
    res = autotune.tune_plain(inst, repeats=2)
    assert len(res["table"]) == len(autotune.PLAIN_SPACE)
    assert res["best"] in res["table"]
    cached = json.load(open(tmp_path / "tune.json"))
    assert len(cached) == 1
    again = autotune.tune_plain(inst, repeats=2)
    assert again == json.loads(json.dumps(res))


def test_tune_batched_identical_planes(tmp_path, monkeypatch):
    from paper_1903_12294_amd import autotune
    _need_gpu()
    monkeypatch.setenv("MF4D_TUNE_CACHE", str(tmp_path / "tune.json"))
    inst = synth.make_config(1)
    crit, qseeds = synth.make_queries(inst, Q=64, seed=5)
    res = autotune.tune_batched(inst, crit, qseeds, repeats=1)
    assert len(res["table"]) == len(autotune.BATCHED_SPACE)
