"""Autotuner: choices are valid, the JSON cache round-trips, a bad file is refused,
and batches planned with the tuned choices still give the plain path's words."""
import json

import pytest
import torch

from paper_1612_05778_amd import _native as nat
from paper_1612_05778_amd import api, synth

from .gpu_util import dev

pytestmark = pytest.mark.gpu


def test_tune_roundtrip_and_results(tmp_path):
    prods = synth.batch(4, 24, deg=(63, 1023), bits=(32, 512))
    items = [(dev(p.a), p.Na, dev(p.b), p.Nb) for p in prods]
    print(f"[tune] {len(items)} products", flush=True)
    ctx = api.Context(0)
    path = str(tmp_path / "tune.json")
    table = ctx.tune(items, cache_path=path)
    assert table, "no class tuned"
    for cls, (K, T) in table.items():
        assert K >= 2 and K & (K - 1) == 0 and K <= 64
        assert T in (8, 16, 32)
    doc = json.load(open(path))
    assert doc["version"] == nat.zpm_version()
    assert {int(c): tuple(v) for c, v in doc["classes"].items()} == table

    got = ctx.mul_batch(items, graph=True)
    torch.cuda.synchronize()
    ref = [ctx.mul(a, Na, b, Nb) for (a, Na, b, Nb) in items]
    torch.cuda.synchronize()
    for k, (g, r) in enumerate(zip(got, ref)):
        assert torch.equal(g, r), f"product {k} differs after tuning"

    ctx2 = api.Context(0)
    ctx2.tune_load(path)
    assert ctx2.tune_table() == table
    bad = tmp_path / "bad.json"
    bad.write_text(json.dumps({"version": nat.zpm_version(), "classes": {"2821": [3, 16]}}))
    with pytest.raises(nat.ZpmError) as e:
        ctx2.tune_load(str(bad))
    assert e.value.code == nat.ZPM_EINVAL
    assert ctx2.tune_table() == table
    old = tmp_path / "old.json"
    old.write_text(json.dumps({"version": -1, "classes": {}}))
    with pytest.raises(nat.ZpmError):
        ctx2.tune_load(str(old))
    ctx2.close()
    ctx.close()
