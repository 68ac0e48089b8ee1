"""The served form: results in the mix equal results alone, continuous
batching overlaps batches, the HBM budget evicts least recently used
graphs and rejects requests that can never fit."""
import sys

import numpy as np
import pytest

import oracle
from helpers import assert_same
from paper_1503_07881_amd import ringo, serve, workloads


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_server_rejects_bad_config():
    import ctypes
    L = serve._lib()
    h = ctypes.c_void_p()
    for cfg in (serve.ServerConfig(0, 1, 1, 1), serve.ServerConfig(1 << 30, 0, 1, 1),
                serve.ServerConfig(1 << 30, 1, 0, 1), serve.ServerConfig(1 << 30, 17, 1, 1)):
        assert L.ringo_server_create(ctypes.byref(cfg), ctypes.byref(h)) == 1


def pinned_tables(specs):
    import torch
    out = []
    for s in specs:
        hs, hd = workloads.generate_host(s)
        ps = torch.from_numpy(hs).pin_memory().numpy()
        pd = torch.from_numpy(hd).pin_memory().numpy()
        out.append((ps, pd))
    return out


@pytest.mark.gpu
def test_mix_equals_alone(cuda):
    import torch
    specs = [workloads.mixed_table(55, i, 1, 200_000) for i in range(24)]
    tables = pinned_tables(specs)
    say("serve: 24 requests in one burst, 3 workers")
    with serve.Server(budget_bytes=8 << 30, num_streams=3, max_batch_tables=4) as srv:
        ids = [srv.submit(s, d) for s, d in tables]
        got = []
        for rid in ids:
            rc, _, lat = srv.wait(rid)
            assert rc == 0 and lat is not None and lat > 0
            got.append(srv.graph(rid, cuda))
        st = srv.stats()
        assert st["completed"] == 24 and st["failed"] == 0 and st["evicted"] == 0
        assert st["batches"] >= 6  # at most 4 requests per batch
    for i, (s, d) in enumerate(tables):
        alone = ringo.to_graph(torch.from_numpy(s).to(cuda), torch.from_numpy(d).to(cuda))
        torch.cuda.synchronize()
        for f in ("node_ids", "out_offsets", "out_nbrs", "in_offsets", "in_nbrs"):
            assert torch.equal(getattr(got[i], f), getattr(alone, f)), f"request {i}: {f} differs"
        if i % 6 == 0:
            assert_same(got[i], oracle.table_to_graph(s, d), f"request {i} vs oracle: ")


@pytest.mark.gpu
def test_poisson_replay_overlaps(cuda):
    specs = [workloads.mixed_table(56, i, 1_000, 2_000_000) for i in range(60)]
    tables = pinned_tables(specs)
    arrivals = np.cumsum(np.full(len(tables), 0.0005))  # 2000 requests/s: faster than service
    say("serve: 60 requests at 2000/s, 2 workers")
    with serve.Server(budget_bytes=64 << 30, num_streams=2, max_batch_tables=8) as srv:
        res = serve.replay(srv, tables, arrivals, warmup=5)
        ov = serve.device_overlap(srv.batches())
    s = res.summary()
    say("serve:", s)
    say("serve: device overlap", ov)
    assert s["requests"] == 55 and s["failed"] == 0
    assert res.stats["max_concurrent_batches"] == 2  # two batches admitted at once
    # and their device work overlapped: intervals between events recorded on
    # the two worker streams intersect
    assert ov["max_batches_at_once"] == 2 and ov["device_overlap_ms"] > 0
    assert s["p99_ms"] >= s["p50_ms"] > 0


@pytest.mark.gpu
def test_budget_evicts_lru_and_rejects_oversized(cuda):
    specs = [workloads.TableSpec("uniform", 100_000, seed=57, table=i, pool=10_000) for i in range(30)]
    tables = pinned_tables(specs)
    say("serve: 30 requests under a 30 MB budget")
    with serve.Server(budget_bytes=30 << 20, num_streams=1, max_batch_tables=1) as srv:
        ids = []
        for s, d in tables:
            ids.append(srv.submit(s, d))
            srv.wait(ids[-1])  # one at a time, never released
        states = [srv.poll(r)[0] for r in ids]
        assert states[-1] == 0
        assert ringo.STATUS_EVICTED in states[:10], states
        evicted_first = states.index(ringo.STATUS_EVICTED)
        assert all(st == 0 for st in states[evicted_first + 1:][-5:])
        assert srv.stats()["evicted"] >= 1
        big = workloads.generate_host(workloads.TableSpec("uniform", 400_000, seed=58, pool=1000))
        rid = srv.submit(*big)
        rc, _, _ = srv.wait(rid)
        assert rc == 3  # RINGO_ERR_OUT_OF_MEMORY: its footprint exceeds the whole budget


@pytest.mark.gpu
def test_batched_budget_frees_what_it_counts(cuda):
    """Batches of up to 6 requests under a budget that binds: every graph
    holds blocks of its own, so once the server is idle the bytes it counts
    as resident are exactly the live blocks a caller's allocator handed out;
    evictions happened; a graph pinned all along was never evicted, and its
    view, read on the client's stream while other graphs were evicted,
    equals the oracle's graph.  The budget (32 MB) lies just above the
    largest request's admission footprint (28.5 MB for 143,444 rows), and
    that request comes last: the graphs resident by then (about 15 MB) and
    its footprint exceed the budget, so the server must evict however its
    batches overlapped, while the pinned graph and it still fit."""
    import torch
    from test_gpu_alloc import CountingAllocator
    specs = [workloads.mixed_table(60, i, 3_000, 150_000) for i in range(40)]
    tables = pinned_tables(specs)
    big = max(range(1, len(specs)), key=lambda i: specs[i].n)
    budget = 32 << 20
    al = CountingAllocator(cuda)
    al.install()
    try:
        with serve.Server(budget_bytes=budget, num_streams=2, max_batch_tables=6,
                          max_batch_rows=400_000) as srv:
            first = srv.submit(*tables[0])
            assert srv.wait(first)[0] == 0
            rc, view = srv.pin(first)
            assert rc == 0
            say("serve: 39 more requests under a 32 MB budget, first graph pinned, the largest last")
            ids = [first] + [None] * (len(tables) - 1)
            for i in [i for i in range(1, len(tables)) if i != big] + [big]:
                ids[i] = srv.submit(*tables[i])
            for rid in ids:
                rc, _, _ = srv.wait(rid)
                assert rc in (0, ringo.STATUS_EVICTED), rc
            # the pinned view, read on the client's stream
            g = ringo.view_graph(view, cuda)
            got = {f: getattr(g, f).cpu().numpy() for f in ("node_ids", "out_offsets", "out_nbrs",
                                                            "in_offsets", "in_nbrs")}
            torch.cuda.synchronize()
            assert_same(got, oracle.table_to_graph(*tables[0]), "pinned graph: ")
            assert srv.poll(first)[0] == 0, "a pinned graph was evicted"
            st = srv.stats()
            states = [srv.poll(r)[0] for r in ids]
            say("serve: stats", st, "evicted", states.count(ringo.STATUS_EVICTED))
            assert st["completed"] == 40 and st["failed"] == 0
            assert st["evicted"] >= 1 and states.count(ringo.STATUS_EVICTED) == st["evicted"]
            assert st["resident_bytes"] <= budget
            torch.cuda.synchronize()
            live = sum(al.live.values())
            assert st["resident_bytes"] == live, (st["resident_bytes"], live)
            assert srv.release(first) == ringo.STATUS_PENDING  # still pinned
            assert srv.unpin(first) == 0
            assert srv.unpin(first) == 1  # no pin left
            # resident graphs read back correctly after the evictions
            for i, rid in enumerate(ids):
                if states[i] == 0 and i % 5 == 0:
                    assert_same(srv.graph(rid, cuda), oracle.table_to_graph(*tables[i]), f"request {i}: ")
            for rid in ids:
                srv.release(rid)
            assert srv.stats()["resident_bytes"] == 0
    finally:
        assert ringo.lib().ringo_set_allocator(None, None, None) == 0
    assert not al.live, "blocks left after the server released every graph"
