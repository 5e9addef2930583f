"""The autotuner on first run and its JSON cache across processes: each case
runs a fresh Python process (the process-wide table and the cache file are
read once per process)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import torch
from paper_2303_16999_amd import spmm, synth
b, n = 16, 384
mb = kb = 96
mask = synth.block_mask(mb, kb, 1 / 8, 5)
nnz = int(mask.sum())
vals = torch.from_numpy(synth.to_storage(synth.normal((nnz, b, b), 6), "f16")).cuda()
X = torch.from_numpy(synth.to_storage(synth.normal((kb * b, n), 7), "f16")).cuda()
plan = spmm.StaticPlan(mb * b, kb * b, b, mask, "f16")
plan.set_values(vals)
before = plan.variant_for(n)
Y = torch.empty((mb * b, n), dtype=torch.float16, device="cuda")
plan.run(X, Y)
torch.cuda.synchronize()
after = plan.variant_for(n)
ref = spmm.StaticPlan(mb * b, kb * b, b, mask, "f16", variant=after or 8 + 256)  # the variant that ran
ref.set_values(vals)
Yr = torch.empty_like(Y)
ref.run(X, Yr)
torch.cuda.synchronize()
print(json.dumps({"before": before, "after": after, "same": bool(torch.equal(Y, Yr))}), flush=True)
"""


def _child(env_extra):
    env = dict(os.environ)
    env.pop("SPMM_AUTOTUNE", None)
    env.pop("SPMM_AUTOTUNE_CACHE", None)
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], env=env, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_first_run_tunes_and_cache_carries_the_choice(tmp_path):
    cache = str(tmp_path / "tune.json")
    first = _child({"SPMM_AUTOTUNE_CACHE": cache})
    assert first["before"] == 0 and first["after"] != 0 and first["same"]
    doc = json.load(open(cache))
    assert doc["format"] == "spmm-autotune-2" and doc["device"].startswith("gfx")
    assert any(e["b"] == 16 and e["variant"] == first["after"] for e in doc["entries"])
    second = _child({"SPMM_AUTOTUNE_CACHE": cache})
    assert second["before"] == first["after"] == second["after"] and second["same"]


def test_autotune_off_keeps_the_rule(tmp_path):
    cache = str(tmp_path / "tune.json")
    r = _child({"SPMM_AUTOTUNE": "0", "SPMM_AUTOTUNE_CACHE": cache})
    assert r["before"] == 0 and r["after"] == 0 and r["same"]
    assert not os.path.exists(cache)


@pytest.mark.parametrize("content", ["not json at all", '{"format": "spmm-autotune-2", "device": "other/1", '
                                     '"hip_runtime": 1, "entries": [{"b": 16, "w": 1, "x": 1, "y": 1, '
                                     '"density_class": 3, "n_class": 9, "dense": 0, "variant": 520}]}'])
def test_foreign_or_broken_cache_is_ignored_and_rewritten(tmp_path, content):
    cache = tmp_path / "tune.json"
    cache.write_text(content)
    r = _child({"SPMM_AUTOTUNE_CACHE": str(cache)})
    assert r["before"] == 0 and r["after"] != 0 and r["same"]
    doc = json.loads(cache.read_text())
    assert doc["device"] != "other/1" and any(e["variant"] == r["after"] for e in doc["entries"])
