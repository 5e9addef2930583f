"""The serving scheduler (host C++) without a device: admission by memory and
slots, continuous batching, completion after the last layer, FIFO order,
rejection, and pool reuse. Runs the library's simulate mode."""
import pytest

from paper_2303_16999_amd import spmm

DIMS = [4096, 16384, 4096, 16384, 4096]  # 4 layers, W1/W2 alternating
L = len(DIMS) - 1


def _bytes(n, dims=DIMS):
    ld = -(-n // 8) * 8
    side0 = max(dims[l] if l % 2 == 0 else dims[l + 1] for l in range(len(dims) - 1))
    side1 = max(dims[l + 1] if l % 2 == 0 else dims[l] for l in range(len(dims) - 1))
    r = lambda b: -(-b // 256) * 256
    return r(side0 * ld * 2) + r(side1 * ld * 2)


def _server(**kw):
    args = dict(mem_budget_bytes=1 << 30, max_active=64, mode=spmm.SERVE_CONTINUOUS, manual=True, simulate=True)
    args.update(kw)
    return spmm.Server([None] * L, DIMS, relu=[1, 0] * (L // 2), **args)


def test_single_request_completes_after_one_step_per_layer():
    s = _server()
    s.submit(7, 33)
    for i in range(L - 1):
        assert s.step() == 1
        assert s.poll() == []
    assert s.step() == 0
    done = s.poll()
    assert [d["id"] for d in done] == [7] and done[0]["n"] == 33
    st = s.stats()
    assert st["steps"] == L and st["problems_run"] == L and st["tokens_done"] == 33


def test_continuous_batching_admits_while_others_are_in_flight():
    s = _server()
    s.submit(1, 8)
    s.step()             # request 1 at layer 1
    s.submit(2, 8)
    s.step()             # 2 admitted now, not after 1 finishes
    assert s.stats()["active"] == 2
    for _ in range(L - 2):
        s.step()
    assert [d["id"] for d in s.poll()] == [1]
    s.step()
    assert [d["id"] for d in s.poll()] == [2]
    assert s.stats()["steps"] == L + 1


def test_max_active_bounds_the_batch():
    s = _server(max_active=3)
    for i in range(10):
        s.submit(i, 16)
    s.step()
    st = s.stats()
    assert st["active"] == 3 and st["pending"] == 7
    s.drain()
    st = s.stats()
    assert st["peak_active"] == 3 and st["requests_done"] == 10 and st["active"] == 0


def test_memory_budget_binds_and_is_released():
    per = _bytes(8)
    s = _server(mem_budget_bytes=int(per * 2.5))
    for i in range(5):
        s.submit(i, 8)
    s.step()
    assert s.stats()["active"] == 2
    s.drain()
    st = s.stats()
    assert st["peak_pool_bytes"] <= int(per * 2.5) and st["peak_active"] == 2
    # the pool coalesced back: a request of two slots' worth fits now
    s.submit(99, 16)
    s.step()
    assert s.stats()["active"] == 1


def test_fifo_head_of_line_and_completion_order():
    per_small, per_big = _bytes(8), _bytes(64)
    s = _server(mem_budget_bytes=per_big + per_small)
    s.submit(1, 64)
    s.submit(2, 64)   # does not fit beside 1: waits at the head
    s.submit(3, 8)    # would fit beside 1, but stays behind 2
    s.step()
    st = s.stats()
    assert st["active"] == 1 and st["pending"] == 2
    s.drain()
    done = s.poll()
    assert [d["id"] for d in done] == [1, 2, 3]
    assert done[2]["admit_s"] >= done[0]["done_s"]


def test_rejects_requests_larger_than_the_pool_and_bad_n():
    s = _server(mem_budget_bytes=_bytes(8))
    with pytest.raises(spmm.SpmmError) as e:
        s.submit(1, 64)
    assert e.value.status == spmm.ERR_REJECTED
    with pytest.raises(spmm.SpmmError) as e:
        s.submit(2, 0)
    assert e.value.status == spmm.ERR_INVALID_ARG
    s.submit(3, 8)
    s.drain()
    assert [d["id"] for d in s.poll()] == [3]


def test_plain_mode_runs_one_request_at_a_time_in_order():
    s = _server(mode=spmm.SERVE_PLAIN)
    for i in range(4):
        s.submit(10 + i, 5 + i)
    for i in range(4):
        s.step()
        assert [d["id"] for d in s.poll()] == [10 + i]
    st = s.stats()
    assert st["steps"] == 4 and st["peak_active"] == 1 and st["problems_run"] == 4 * L


def test_worker_thread_drains_everything_once():
    s = _server(manual=False, max_active=8)
    ids = list(range(200))
    for i in ids:
        s.submit(i, 1 + (i * 37) % 500)
    s.drain()
    done = []
    while True:
        got = s.poll(64)
        if not got:
            break
        done += got
    assert sorted(d["id"] for d in done) == ids
    assert all(d["submit_s"] <= d["admit_s"] <= d["done_s"] for d in done)
    assert s.stats()["peak_active"] <= 8
    s.close()


def test_token_budget_limits_admission_but_never_blocks_a_lone_request():
    s = _server(max_tokens=100)
    s.submit(1, 60)
    s.submit(2, 60)   # 60 + 60 > 100: waits for 1
    s.submit(3, 30)   # FIFO: stays behind 2
    s.step()
    st = s.stats()
    assert st["active"] == 1 and st["pending"] == 2
    for _ in range(L - 1):
        s.step()
    assert [d["id"] for d in s.poll()] == [1]
    s.step()          # 2 and 3 fit together now (90 tokens)
    assert s.stats()["active"] == 2
    s.drain()
    assert [d["id"] for d in s.poll()] == [2, 3]
    big = _server(max_tokens=16)
    big.submit(7, 500)  # larger than the budget, admitted alone
    big.step()
    assert big.stats()["active"] == 1
