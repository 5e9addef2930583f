"""GPU tests of the tile variants, the autotuner and the grouped launch in both
its forms (one workgroup per unit; persistent workgroups walking the units on a static schedule)."""
import numpy as np
import pytest
import torch

from oracle import spmm_ref as O
from paper_2303_16999_amd import spmm
from gpu_cases import Case, round_like, y_f64

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("b,w,y", [(16, "f16", "f16"), (32, "bf16", "f32"), (4, "f16", "f16"), (8, "bf16", "bf16"),
                                   (1, "f16", "f32")])
def test_variants_agree_bitwise_and_match_oracle(b, w, y):
    # the variants change the column tiling only, never the order of the sums
    c = Case(23 * b + 3, 17 * b + 1, 301, b, 0.3, w=w, y=y, seed=50 + b)
    variants = (2, 4, 8) if b >= 16 else (4, 8)
    outs = []
    for v in variants:
        plan = spmm.StaticPlan(c.m, c.k, b, c.mask, w, y=y, variant=v)
        vals, X, _ = c.device_inputs()
        plan.set_values(vals)
        Y = c.new_Y()
        plan.run(X, Y, n=c.n)
        torch.cuda.synchronize()
        outs.append(Y)
        plan.close()
    for Y in outs[1:]:
        assert torch.equal(outs[0][:, : c.n], Y[:, : c.n])
    assert O.rel_fro(y_f64(outs[0], c), c.oracle()) <= 5e-3


@pytest.mark.parametrize("b,w", [(16, "f16"), (8, "f16"), (4, "bf16"), (32, "bf16")])
def test_autotune_picks_a_variant_and_keeps_results(b, w):
    c = Case(64 * b, 48 * b, 96, b, 1 / 8, w=w, seed=61)
    plan, Y0 = c.run_static()
    vals, X, _ = c.device_inputs()
    Y1 = c.new_Y()
    v, times = plan.autotune(X, Y1, n=c.n)
    # candidates: tile widths x kernel forms (form 2: pipelined row kernel for
    # b = 16/32, LDS-staged kernel for b = 1/4/8)
    want = {16: [2, 4, 8, 514, 516, 520, 1024], 32: [2, 4, 8, 514, 516, 520], 8: [4, 8, 512], 4: [4, 8, 512]}[b]
    want = sorted(x + 256 if x < 256 else x for x in want)
    assert sorted(times) == want and v in times and all(t > 0 for t in times.values())
    assert plan.variant_for(c.n) == v
    Y2 = c.new_Y()
    plan.run(X, Y2, n=c.n)  # now on the tuned variant
    torch.cuda.synchronize()
    assert torch.equal(Y1[:, : c.n], Y2[:, : c.n])
    # every candidate forced through the plan options: the same bits as the
    # tuned run where the kernel form sums in the same order (tile widths; the
    # pipelined row kernel), else within the FP16 bound of the oracle (the b = 4
    # LDS-staged kernel and the split rows of form 4 add in another order)
    ref = c.oracle()

    def order_class(var):
        form = var >> 8
        return "split" if form == 4 else ("lds" if (b < 16 and form == 2) else "rows")

    for var in times:
        pv = spmm.StaticPlan(c.m, c.k, b, c.mask, w, variant=var)
        pv.set_values(vals)
        Y3 = c.new_Y()
        pv.run(X, Y3, n=c.n)
        torch.cuda.synchronize()
        if order_class(var) == order_class(v):
            assert torch.equal(Y1[:, : c.n], Y3[:, : c.n]), var
        assert O.rel_fro(y_f64(Y3, c), ref) <= 5e-3, var
        pv.close()


def test_autotune_widths_reports_best_per_tile_width():
    c = Case(64 * 16, 48 * 16, 200, 16, 1 / 8, w="f16", seed=62)
    plan, Y0 = c.run_static()
    _, X, _ = c.device_inputs()
    Y1 = c.new_Y()
    v, widths = plan.autotune_widths(X, Y1, n=c.n)
    # forms without a width of their own (split rows: ns = 0) show only in v
    assert sorted(widths) == [2, 4, 8] and ((v & 0xFF) in widths or (v >> 8) == 4)
    ref = c.oracle()
    for Y in (Y0, Y1):  # each run's tuning may settle on another form: both within the bound
        assert O.rel_fro(y_f64(Y, c), ref) <= 5e-3


def _group_cases(b, w, y, ns, seed):
    cases = []
    for i, n in enumerate(ns):
        m = (5 + 3 * i) * b + (i % 3)
        k = (7 + 2 * i) * b + (i % 2)
        cases.append(Case(m, k, max(n, 1), b, 0.15 + 0.05 * i, w=w, y=y, seed=seed + i))
    return cases


@pytest.mark.parametrize("persist", ["0", "1"])
@pytest.mark.parametrize("b,w,y", [(16, "f16", "f16"), (32, "bf16", "f32"), (16, "bf16", "bf16")])
def test_group_matches_single_launches_and_oracle(b, w, y, persist, monkeypatch):
    monkeypatch.setenv("SPMM_GROUP_PERSIST", persist)
    ns = [1, 17, 64, 200, 513, 0, 33]
    cases = _group_cases(b, w, y, ns, seed=70)
    relu = [i % 2 for i in range(len(cases))]
    plans, Xs, Ys, ref_single = [], [], [], []
    for c in cases:
        plan, Ys_single = c.run_static()
        vals, X, _ = c.device_inputs()
        plans.append(plan)
        Xs.append(X)
        Ys.append(c.new_Y())
        ref_single.append(Ys_single)
    g = spmm.Group(16)
    g.run(plans, Xs, Ys, ns=ns, relu=relu)
    torch.cuda.synchronize()
    for i, c in enumerate(cases):
        if ns[i] == 0:
            assert torch.isnan(Ys[i]).all().item()  # skipped problem left untouched
            continue
        single = ref_single[i][:, : c.n]
        if relu[i]:
            single = torch.clamp(single, min=0)
        assert torch.equal(Ys[i][:, : c.n], single), i
        ref = c.oracle()
        if relu[i]:
            ref = np.maximum(ref, 0.0)
        assert O.rel_fro(y_f64(Ys[i], c), ref) <= 5e-3, i


@pytest.mark.parametrize("graph", ["1", "0"])
def test_group_graph_replays_with_new_tables(graph, monkeypatch):
    """Replay the captured graph (or, with SPMM_GROUP_GRAPH=0, launch directly)
    many times with different n, X and Y; eager work and synchronisations
    between the calls; every call checked."""
    monkeypatch.setenv("SPMM_GROUP_GRAPH", graph)
    b = 16
    cases = _group_cases(b, "f16", "f16", [40, 300, 7, 129], seed=90)
    plans = [c.run_static()[0] for c in cases]
    singles = {}
    g = spmm.Group(8)
    rng = np.random.default_rng(0)
    for rep in range(6):
        sel = [int(i) for i in rng.permutation(len(cases))[: 2 + rep % 3]]
        ns = [int(rng.integers(1, cases[i].n + 1)) for i in sel]
        Xs = [cases[i].device_inputs()[1] for i in sel]
        Ys = [cases[i].new_Y() for i in sel]
        g.run([plans[i] for i in sel], Xs, Ys, ns=ns)
        torch.cuda.synchronize()
        junk = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        for j, i in enumerate(sel):
            key = (i, ns[j])
            if key not in singles:
                Yr = cases[i].new_Y()
                plans[i].run(Xs[j], Yr, n=ns[j])
                torch.cuda.synchronize()
                singles[key] = Yr[:, : ns[j]].clone()
            assert torch.equal(Ys[j][:, : ns[j]], singles[key]), (rep, i)
        del junk


def test_group_rejects_mixed_plans():
    a = Case(64, 64, 32, 16, 0.5, w="f16", seed=1)
    bcase = Case(64, 64, 32, 32, 0.5, w="f16", seed=2)
    pa, _ = a.run_static()
    pb, _ = bcase.run_static()
    g = spmm.Group(4)
    Xa, Xb = a.device_inputs()[1], bcase.device_inputs()[1]
    with pytest.raises(spmm.SpmmError) as e:
        g.run([pa, pb], [Xa, Xb], [a.new_Y(), bcase.new_Y()])
    assert e.value.status == spmm.ERR_INVALID_ARG
    with pytest.raises(spmm.SpmmError) as e:
        g.run([pa] * 5, [Xa] * 5, [a.new_Y() for _ in range(5)])
    assert e.value.status == spmm.ERR_INVALID_ARG


@pytest.mark.parametrize("persist", ["0", "1"])
def test_group_device_table_form_matches_single_launches(persist, monkeypatch):
    """More problems than fit in the kernel arguments: the table goes through device memory."""
    monkeypatch.setenv("SPMM_GROUP_PERSIST", persist)
    b = 16
    cases = [Case((3 + i % 5) * b, (4 + i % 3) * b + i % 2, 1 + (i * 37) % 150, b, 0.3, w="f16", seed=200 + i)
             for i in range(40)]
    plans, Xs, singles = [], [], []
    for c in cases:
        plan, Ys = c.run_static()
        plans.append(plan)
        Xs.append(c.device_inputs()[1])
        singles.append(Ys[:, : c.n].clone())
    g = spmm.Group(64)
    for rep in range(3):  # several calls walk the ring of tables
        Ys = [c.new_Y() for c in cases]
        g.run(plans, Xs, Ys, ns=[c.n for c in cases])
        torch.cuda.synchronize()
        for i, c in enumerate(cases):
            assert torch.equal(Ys[i][:, : c.n], singles[i]), (rep, i)


# argument table, device table, graph; then both tables in the persistent form
@pytest.mark.parametrize("count,graph,persist", [(3, "0", "0"), (40, "0", "0"), (3, "1", "0"), (3, "0", "1"),
                                                 (40, "0", "1")])
def test_group_back_to_back_calls_keep_their_own_tables(count, graph, persist, monkeypatch):
    """Calls issued without synchronising in between, each with other n, X and Y:
    every output must be the one its own call asked for. With
    SPMM_GROUP_GRAPH=1 the captured graph's node is updated while the previous
    replay of the same executable may still be running."""
    monkeypatch.setenv("SPMM_GROUP_GRAPH", graph)
    monkeypatch.setenv("SPMM_GROUP_PERSIST", persist)
    b = 16
    cases = [Case((3 + i % 4) * b, (5 + i % 3) * b, 64 + 8 * (i % 7), b, 0.3, w="f16", seed=300 + i)
             for i in range(count)]
    plans = [c.run_static()[0] for c in cases]
    g = spmm.Group(64)
    calls = []
    for rep in range(6):
        ns = [1 + (rep * 13 + 5 * i) % c.n for i, c in enumerate(cases)]
        Xs = [torch.randn((c.k, c.ldx), device="cuda").half() for c in cases]
        Ys = [c.new_Y() for c in cases]
        g.run(plans, Xs, Ys, ns=ns)
        calls.append((ns, Xs, Ys))
    torch.cuda.synchronize()
    for ns, Xs, Ys in calls:
        for i, c in enumerate(cases):
            Yr = c.new_Y()
            plans[i].run(Xs[i], Yr, n=ns[i])
            torch.cuda.synchronize()
            assert torch.equal(Ys[i][:, : ns[i]], Yr[:, : ns[i]]), i


def test_group_persistent_form_large_and_small_calls_in_turn(monkeypatch):
    """The persistent form's grid follows each call: a call with many units per
    workgroup, one with fewer units than workgroups, then the first again,
    unsynchronised, all equal to single launches."""
    monkeypatch.setenv("SPMM_GROUP_PERSIST", "1")
    b = 16
    big = [Case(256 * b // 4, 128 * b // 4, 4096, b, 1 / 8, w="f16", seed=400 + i) for i in range(3)]
    small = [Case(3 * b, 5 * b, 9, b, 0.5, w="f16", seed=410)]
    g = spmm.Group(8)
    calls = []
    for cases in (big, small, big, small):
        plans = [c.run_static()[0] for c in cases]
        Xs = [c.device_inputs()[1] for c in cases]
        Ys = [c.new_Y() for c in cases]
        g.run(plans, Xs, Ys, ns=[c.n for c in cases])
        calls.append((cases, plans, Xs, Ys))
    torch.cuda.synchronize()
    for cases, plans, Xs, Ys in calls:
        for i, c in enumerate(cases):
            Yr = c.new_Y()
            plans[i].run(Xs[i], Yr, n=c.n)
            torch.cuda.synchronize()
            assert torch.equal(Ys[i][:, : c.n], Yr[:, : c.n]), i
