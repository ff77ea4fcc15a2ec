"""GPU: the serving loop.  Each request's bits are the same alone and in the
mix, equal the plain per-request path, and equal the oracle on a sample;
hipGraph replays agree with direct launches across many steps."""
import threading

import numpy as np
import pytest

import oracle
from paper_1108_3126_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SMALL = dict(hbm_budget=1 << 30, step_bytes=16 << 20, step_strings=1 << 16, step_requests=64, slots=2,
             program_slots=64)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def requests():
    reqs = [W.serving_request(3, i, max_strings=600) for i in range(40)]
    # a repeated program (cache hit) and an empty request
    reqs.append((reqs[0][0], W.pack([b"abc", b""])))
    reqs.append((reqs[1][0], W.pack([])))
    return reqs


def _oracle_sample(prog, s, k=40):
    if s.n == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.uint8)
    idx = np.unique(np.linspace(0, s.n - 1, min(k, s.n)).astype(np.int64))
    return idx, oracle.match(prog.ast, prog.root, prog.classes, prog.search, s.data, s.offsets, index=idx)


def test_alone_vs_mix_vs_plain_vs_oracle(dev, requests):
    from paper_1108_3126_amd import server

    with server.Server(use_graph=True, **SMALL) as srv:
        alone = []
        for prog, s in requests:
            alone.append(srv.wait(srv.submit(prog, s.data, s.offsets)))
        ids = [srv.submit(prog, s.data, s.offsets) for prog, s in requests]
        mix = [srv.wait(r) for r in ids]
        st = srv.stats()
    print("server stats:", {k: st[k] for k in ("steps", "graph_steps", "cache_hits", "cache_misses", "p50_us",
                                               "p99_us")}, flush=True)
    assert st["completed"] == 2 * len(requests) and st["steps"] < 2 * len(requests)  # the mix was batched
    assert st["cache_hits"] > 0
    for (prog, s), a, b in zip(requests, alone, mix):
        assert np.array_equal(a, b)
        assert np.array_equal(server.plain_match(prog, s.data, s.offsets), a)
        idx, want = _oracle_sample(prog, s)
        assert np.array_equal(a[idx], want)


def test_graph_replays_agree_with_direct_launches(dev, requests):
    from paper_1108_3126_amd import server

    outs = []
    for use_graph in (False, True):
        with server.Server(use_graph=use_graph, **SMALL) as srv:
            res = []
            for rep in range(3):  # many steps: the graph is replayed with new parameters each time
                ids = [srv.submit(prog, s.data, s.offsets) for prog, s in requests[rep::3]]
                res += [srv.wait(r) for r in ids]
                torch.cuda.synchronize()
            st = srv.stats()
            assert (st["graph_steps"] > 0) == use_graph
            outs.append(res)
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_concurrent_clients(dev, requests):
    from paper_1108_3126_amd import server

    with server.Server(use_graph=True, **SMALL) as srv:
        want = {i: srv.wait(srv.submit(p, s.data, s.offsets)) for i, (p, s) in enumerate(requests)}
        got, errs = {}, []

        def client(k):
            try:
                for i in range(k, len(requests), 4):
                    p, s = requests[i]
                    got[i] = srv.wait(srv.submit(p, s.data, s.offsets))
            except Exception as e:  # pragma: no cover
                errs.append(e)

        ts = [threading.Thread(target=client, args=(k,)) for k in range(4)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        assert not errs
        for i in want:
            assert np.array_equal(got[i], want[i])


def test_admission_errors(dev):
    from paper_1108_3126_amd import rx, server

    with server.Server(use_graph=False, **SMALL) as srv:
        prog = W.small_program(0)
        big = W.Strings(np.zeros(17 << 20, np.uint8), np.array([0, 17 << 20], np.int64))
        with pytest.raises(rx.RxError) as ei:
            srv.submit(prog, big.data, big.offsets)
        assert ei.value.code == rx.RX_ETOOBIG
        bad = W.Program(np.array([(3, 0, 0, 0, 0)], dtype=W.AST_DTYPE), 0, np.zeros((0, 4), np.uint64), False)
        with pytest.raises(rx.RxError) as ei:
            srv.submit(bad, np.zeros(1, np.uint8), np.array([0, 1], np.int64))
        assert ei.value.code == rx.RX_EINVAL
        with pytest.raises(rx.RxError):
            srv.wait(12345)
        assert srv.stats()["rejected"] == 1


def test_more_distinct_programs_than_resident_slots(dev):
    """Four resident program slots, two step slots, 24 distinct programs submitted at once: every
    request completes (a step takes at most program_slots / slots distinct programs) and its bits
    equal the oracle's; evictions happen."""
    from paper_1108_3126_amd import server

    reqs = [W.serving_request(5, i, max_strings=200) for i in range(24)]
    cfg = dict(SMALL, program_slots=4, slots=2)
    with server.Server(use_graph=True, **cfg) as srv:
        ids = [srv.submit(p, s.data, s.offsets) for p, s in reqs]
        got = [srv.wait(r, timeout_us=60_000_000) for r in ids]
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["cache_evictions"] > 0
    for (p, s), g in zip(reqs, got):
        idx, want = _oracle_sample(p, s)
        assert np.array_equal(g[idx], want)


def test_plain_context_equals_plain_path(dev, requests):
    """The preallocated plain path (one stream, buffers made once) gives the plain path's bits."""
    from paper_1108_3126_amd import rx, server

    with server.PlainContext(16 << 20, 1 << 16) as ctx:
        for prog, s in requests:
            assert np.array_equal(ctx.match(prog, s.data, s.offsets), server.plain_match(prog, s.data, s.offsets))
        big = W.Strings(np.zeros(17 << 20, np.uint8), np.array([0, 17 << 20], np.int64))
        with pytest.raises(rx.RxError) as ei:
            ctx.match(requests[0][0], big.data, big.offsets)
        assert ei.value.code == rx.RX_ETOOBIG
