"""Serving at the serving model's own dimensions: 8 layers of
(W1 16384 x 4096, ReLU, W2 4096 x 16384), b = 16, density 1/16, FP16 weights
scaled by 1/sqrt(k d) (W1) and sqrt(2)/sqrt(k d) (W2) so that activations
stay O(1). A few requests of n <= 64 go through continuous batching; each one
is replayed layer by layer on the device (one grouped launch per layer, ReLU
fused as in the server), its output equals the server's bit for bit, and
every layer is checked against the FP64 layer oracle on the device's own FP16
input to that layer (relative Frobenius error and every element within its
rounding bound)."""
import math

import numpy as np
import pytest
import torch

from oracle import spmm_ref as O
from paper_2303_16999_amd import spmm, synth
from gpu_cases import assert_elementwise, dev

pytestmark = pytest.mark.gpu

D_IN, D_HID, B, D = 4096, 16384, 16, 1 / 16
LAYERS = 16  # 8 x (W1, W2)


def _model():
    layers = []
    for l in range(LAYERS):
        k, m = (D_IN, D_HID) if l % 2 == 0 else (D_HID, D_IN)
        mask = synth.block_mask(m // B, k // B, D, 500 + 2 * l)
        rows, cols = synth.mask_coo(mask)
        scale = (1.0 if l % 2 == 0 else math.sqrt(2.0)) / math.sqrt(k * D)
        vals = synth.to_storage(synth.normal((len(rows), B, B), 501 + 2 * l) * scale, "f16")
        plan = spmm.StaticPlan(m, k, B, mask, "f16", n_hint=64)
        plan.set_values(dev(vals))
        layers.append({"plan": plan, "rows": rows, "cols": cols, "vals64": synth.storage_to_f64(vals, "f16"),
                       "m": m, "k": k, "relu": l % 2 == 0})
    torch.cuda.synchronize()
    return layers


def test_serving_model_dims_layer_oracle():
    layers = _model()
    dims = [D_IN] + [L["m"] for L in layers]
    relu = [1 if L["relu"] else 0 for L in layers]
    ns = [1, 19, 64]
    n8 = [-(-n // 8) * 8 for n in ns]
    xs = [synth.to_storage(synth.normal((D_IN, n), 900 + i), "f16") for i, n in enumerate(ns)]
    # the server: continuous batching of the three requests
    srv = spmm.Server([L["plan"] for L in layers], dims, relu=relu, mem_budget_bytes=1 << 30, max_active=8,
                      mode=spmm.SERVE_CONTINUOUS)
    ys = [np.full((D_IN, w), np.nan, np.float16) for w in n8]
    xh = [np.zeros((D_IN, w), np.float16) for w in n8]
    for i, n in enumerate(ns):
        xh[i][:, :n] = xs[i]
        srv.submit(i, n, xh[i], ys[i])
    srv.drain()
    assert sorted(d["id"] for d in srv.poll()) == [0, 1, 2]
    srv.close()
    # the same requests layer by layer, all three side by side in one buffer
    # (columns are independent), each layer against the FP64 layer oracle
    offs = np.concatenate([[0], np.cumsum(n8)])
    cur = torch.zeros((D_IN, int(offs[-1])), dtype=torch.float16, device="cuda")
    for i, n in enumerate(ns):
        cur[:, offs[i]: offs[i] + n] = dev(xs[i])
    used = np.concatenate([np.arange(offs[i], offs[i] + n) for i, n in enumerate(ns)])
    g = spmm.Group(1)
    for l, L in enumerate(layers):
        out = torch.full((L["m"], cur.shape[1]), float("nan"), dtype=torch.float16, device="cuda")
        g.run([L["plan"]], [cur], [out], relu=[relu[l]])
        torch.cuda.synchronize()
        x64 = cur.cpu().numpy().astype(np.float64)[:, used]
        ref = O.spmm_blockwise(L["m"], L["k"], B, L["rows"], L["cols"], L["vals64"], x64)
        A = O.spmm_blockwise(L["m"], L["k"], B, L["rows"], L["cols"], np.abs(L["vals64"]), np.abs(x64))
        if L["relu"]:
            ref = np.maximum(ref, 0.0)
        got = out.cpu().numpy().astype(np.float64)[:, used]
        err = O.rel_fro(got, ref)
        assert err <= 5e-3, (l, err)
        assert_elementwise(got, ref, A, L["k"], "f16")
        assert np.abs(got).max() < 1e3, l  # the scaling keeps activations O(1)
        cur = out
    g.close()
    final = cur.cpu().numpy()
    for i, n in enumerate(ns):
        assert np.array_equal(ys[i][:, :n], final[:, offs[i]: offs[i] + n]), i
    for L in layers:
        L["plan"].close()
