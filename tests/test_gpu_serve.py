"""GPU tests of the serving loop: each request's result is the same alone and
in the mix (continuous batching), equal to the plain path, and matches the
FP64 oracle chain."""
import time

import numpy as np
import pytest
import torch

from oracle import spmm_ref as O
from paper_2303_16999_amd import spmm, synth
from gpu_cases import dev

pytestmark = pytest.mark.gpu

DIMS = [256, 512, 256, 512, 256]
RELU = [1, 0, 1, 0]
B = 16


def _layers(seed=0, d=0.25):
    layers = []
    for l in range(len(DIMS) - 1):
        k, m = DIMS[l], DIMS[l + 1]
        mask = synth.block_mask(m // B, k // B, d, seed + 10 * l)
        rows, cols = synth.mask_coo(mask)
        vals = synth.to_storage(synth.normal((len(rows), B, B), seed + 10 * l + 1) * 0.25, "f16")
        plan = spmm.StaticPlan(m, k, B, mask, "f16")
        plan.set_values(dev(vals))
        layers.append((plan, rows, cols, synth.storage_to_f64(vals, "f16")))
    torch.cuda.synchronize()
    return layers


def _oracle_chain(layers, x64):
    """FP64 products; activations rounded to FP16 after every layer as stored."""
    v = x64
    for l, (_, rows, cols, vals) in enumerate(layers):
        v = O.spmm_blockwise(DIMS[l + 1], DIMS[l], B, rows, cols, vals, v)
        if RELU[l]:
            v = np.maximum(v, 0.0)
        v = torch.from_numpy(v).to(torch.float16).to(torch.float64).numpy()
    return v


def _requests(count, seed):
    g = np.random.default_rng(seed)
    ns = [int(v) for v in g.integers(1, 120, count)]
    xs = [synth.to_storage(synth.normal((DIMS[0], n), seed + 100 + i), "f16") for i, n in enumerate(ns)]
    return ns, xs


def _serve(layers, ns, xs, mode, manual, max_active=64, stagger=False):
    srv = spmm.Server([p for p, *_ in layers], DIMS, relu=RELU, mem_budget_bytes=64 << 20, max_active=max_active,
                      mode=mode, manual=manual)
    ys = [np.full((DIMS[-1], n), np.nan, np.float16) for n in ns]
    half = len(ns) // 2
    for i in range(len(ns)):
        if stagger and i == half:
            time.sleep(0.002)  # the second half arrives while the first is in flight
        srv.submit(i, ns[i], np.ascontiguousarray(xs[i]), ys[i])
    srv.drain()
    done = srv.poll()
    stats = srv.stats()
    srv.close()
    assert sorted(d["id"] for d in done) == list(range(len(ns)))
    return ys, stats


def test_alone_equals_in_mix_equals_plain_and_oracle():
    layers = _layers()
    ns, xs = _requests(12, seed=5)
    alone = []
    for i in range(len(ns)):
        ys, _ = _serve(layers, [ns[i]], [xs[i]], spmm.SERVE_CONTINUOUS, manual=True)
        alone.append(ys[0])
    mix, st = _serve(layers, ns, xs, spmm.SERVE_CONTINUOUS, manual=False, max_active=4, stagger=True)
    assert st["peak_active"] <= 4 and st["requests_done"] == len(ns)
    plain, _ = _serve(layers, ns, xs, spmm.SERVE_PLAIN, manual=False)
    for i in range(len(ns)):
        assert np.array_equal(alone[i], mix[i]), i
        assert np.array_equal(alone[i], plain[i]), i
        ref = _oracle_chain(layers, synth.storage_to_f64(xs[i], "f16"))
        assert O.rel_fro(mix[i].astype(np.float64), ref) <= 5e-3, i


def test_manual_continuous_steps_batch_requests_at_different_layers():
    layers = _layers(seed=3)
    ns, xs = _requests(6, seed=9)
    srv = spmm.Server([p for p, *_ in layers], DIMS, relu=RELU, mem_budget_bytes=64 << 20, max_active=8,
                      mode=spmm.SERVE_CONTINUOUS, manual=True)
    ys = [np.zeros((DIMS[-1], n), np.float16) for n in ns]
    srv.submit(0, ns[0], xs[0], ys[0])
    srv.step()
    srv.step()
    for i in range(1, len(ns)):
        srv.submit(i, ns[i], xs[i], ys[i])
    srv.step()  # request 0 at its third layer, the rest at their first: one launch
    st = srv.stats()
    assert st["active"] == len(ns) and st["problems_run"] == 2 + len(ns)
    srv.drain()
    assert sorted(d["id"] for d in srv.poll()) == list(range(len(ns)))
    for i in range(len(ns)):
        ref = _oracle_chain(layers, synth.storage_to_f64(xs[i], "f16"))
        assert O.rel_fro(ys[i].astype(np.float64), ref) <= 5e-3, i
    srv.close()
