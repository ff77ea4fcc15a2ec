"""GPU parity of batched matching (many programs, uneven lengths, one
persistent launch with device-side length bucketing) against the oracle, and
determinacy across bucket edges and launch shapes."""
import numpy as np
import pytest

import oracle
from paper_1108_3126_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _oracle_all(progs, s):
    return np.stack([oracle.match(p.ast, p.root, p.classes, p.search, s.data, s.offsets) for p in progs])


@pytest.fixture(scope="module")
def multi_case():
    progs = W.multi_programs(seed=2, count=8, lo=16, hi=300)
    s = W.multi_lines(seed=2, n=3000, hi=1500)
    return progs, s, _oracle_all(progs, s)


def test_multi_matches_oracle(dev, multi_case):
    from paper_1108_3126_amd import rx

    progs, s, want = multi_case
    ps = [rx.compile(p.ast, p.root, p.classes, p.search).upload(dev) for p in progs]
    d, o = torch.from_numpy(s.data).to(dev), torch.from_numpy(s.offsets).to(dev)
    got = rx.match_multi(ps, d, o).cpu().numpy()
    print("multi: accepted per program", want.sum(axis=1).tolist(), flush=True)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("edges,block,grid", [([], 64, 1), ([100], 128, 7), ([4, 64, 65, 200, 1000], 256, 0),
                                              ([0], 256, 3), (list(range(100, 1600, 100)), 64, 0)])
def test_multi_bucketing_is_determinate(dev, multi_case, edges, block, grid):
    from paper_1108_3126_amd import rx

    progs, s, want = multi_case
    ps = [rx.compile(p.ast, p.root, p.classes, p.search).upload(dev) for p in progs[:4]]
    d, o = torch.from_numpy(s.data).to(dev), torch.from_numpy(s.offsets).to(dev)
    got = rx.match_multi(ps, d, o, config=rx.multi_config(edges, block, grid)).cpu().numpy()
    assert np.array_equal(got, want[:4])


def test_multi_edge_cases(dev):
    from paper_1108_3126_amd import rx

    progs = W.multi_programs(seed=40, count=3, lo=8, hi=40)
    strs = [b"", b" ", b"e" * 5000, b"the quick", b""] + [bytes([i % 256]) * (i % 37) for i in range(300)]
    s = W.pack(strs)
    ps = [rx.compile(p.ast, p.root, p.classes, p.search).upload(dev) for p in progs]
    want = _oracle_all(progs, s)
    d, o = torch.from_numpy(s.data).to(dev), torch.from_numpy(s.offsets).to(dev)
    assert np.array_equal(rx.match_multi(ps, d, o).cpu().numpy(), want)
    # an anchored program alongside searched ones
    small = W.small_program(3)
    ps2 = ps + [rx.compile(small.ast, small.root, small.classes, False).upload(dev)]
    want2 = np.concatenate([want, _oracle_all([small], s)])
    assert np.array_equal(rx.match_multi(ps2, d, o).cpu().numpy(), want2)
    # zero strings
    z = rx.match_multi(ps, torch.zeros(1, dtype=torch.uint8, device=dev), torch.zeros(1, dtype=torch.int64, device=dev))
    assert z.shape == (3, 0)


# -- plane form: the bit-sliced circuit over length-sorted slabs -----------------
def _planes(rx, ps):
    rx.prepare_multi(ps)
    return rx.multi_config(form=rx.FORM_PLANES)


def test_planes_match_oracle(dev, multi_case):
    from paper_1108_3126_amd import rx

    progs, s, want = multi_case
    ps = [rx.compile(p.ast, p.root, p.classes, p.search).upload(dev) for p in progs]
    cfg = _planes(rx, ps)
    d, o = torch.from_numpy(s.data).to(dev), torch.from_numpy(s.offsets).to(dev)
    got = rx.match_multi(ps, d, o, config=cfg).cpu().numpy()
    assert np.array_equal(got, want)


def test_planes_many_slabs_match_oracle(dev):
    """More slabs than the longest few that run first: the rest go through planes and circuits in parts
    of about equal ticks (the planes of one part made while the circuits of the one before run); every
    (program, line) bit equals the oracle's, over 98 slabs of log-normal lengths."""
    from paper_1108_3126_amd import rx

    progs = W.multi_programs(seed=2, count=6, lo=16, hi=300)
    s = W.multi_lines(seed=7, n=200_000, hi=2000)
    want = np.stack([oracle.match(p.ast, p.root, p.classes, p.search, s.data, s.offsets, threads=8) for p in progs])
    ps = [rx.compile(p.ast, p.root, p.classes, p.search).upload(dev) for p in progs]
    cfg = _planes(rx, ps)
    d, o = torch.from_numpy(s.data).to(dev), torch.from_numpy(s.offsets).to(dev)
    for _ in range(2):
        got = rx.match_multi(ps, d, o, config=cfg).cpu().numpy()
        bad = np.nonzero(got != want)
        assert bad[0].size == 0, list(zip(bad[0][:5], bad[1][:5]))


def test_planes_edge_cases(dev):
    """Empty strings, one-byte strings, lengths around the slab and sort limits (8190 sorts, 8191 and
    longer run in table form), a partial last slab, unaligned offsets, anchored and searched."""
    from paper_1108_3126_amd import rx

    progs = W.multi_programs(seed=41, count=3, lo=8, hi=60) + [W.small_program(5)]
    rng = np.random.default_rng(9)
    strs = [b"", b"a", b"ab", b"e" * 8190, b"e" * 8191, b"the quick brown" * 700, b""]
    strs += [bytes(rng.integers(32, 127, size=int(rng.integers(0, 90)), dtype=np.uint8)) for _ in range(4200)]
    strs += [b"ab" * int(k) for k in rng.integers(0, 40, size=300)]
    s = W.pack(strs)
    want = _oracle_all(progs, s)
    ps = [rx.compile(p.ast, p.root, p.classes, p.search).upload(dev) for p in progs]
    cfg = _planes(rx, ps)
    # the strings one byte into the buffer: every offset unaligned
    buf = np.concatenate([np.zeros(1, np.uint8), s.data])
    d = torch.from_numpy(buf).to(dev)
    o = torch.from_numpy(s.offsets + 1).to(dev)
    got = rx.match_multi(ps, d, o, config=cfg).cpu().numpy()
    bad = np.nonzero(got != want)
    assert bad[0].size == 0, list(zip(bad[0][:5], bad[1][:5]))
    # the table form agrees
    assert np.array_equal(rx.match_multi(ps, d, o).cpu().numpy(), want)
    # one string; no strings
    one = W.pack([b"xyz"])
    got1 = rx.match_multi(ps, torch.from_numpy(one.data).to(dev), torch.from_numpy(one.offsets).to(dev),
                          config=cfg).cpu().numpy()
    assert np.array_equal(got1, _oracle_all(progs, one))
    z = rx.match_multi(ps, torch.zeros(1, dtype=torch.uint8, device=dev), torch.zeros(1, dtype=torch.int64, device=dev),
                       config=cfg)
    assert z.shape == (4, 0)


def test_planes_needs_a_prepared_list(dev, multi_case):
    from paper_1108_3126_amd import rx

    progs, s, want = multi_case
    ps = [rx.compile(p.ast, p.root, p.classes, p.search).upload(dev) for p in progs[:2]]
    d, o = torch.from_numpy(s.data).to(dev), torch.from_numpy(s.offsets).to(dev)
    with pytest.raises(rx.RxError) as ei:
        rx.match_multi(ps, d, o, config=rx.multi_config(form=rx.FORM_PLANES))
    assert ei.value.code == rx.RX_EINVAL
    rx.prepare_multi(ps)
    # a different order is another list
    with pytest.raises(rx.RxError):
        rx.match_multi(ps[::-1], d, o, config=rx.multi_config(form=rx.FORM_PLANES))
    got = rx.match_multi(ps, d, o, config=rx.multi_config(form=rx.FORM_PLANES)).cpu().numpy()
    assert np.array_equal(got, want[:2])


def test_planes_repeat_calls_share_workspace(dev, multi_case):
    """The same workspace for two calls in a row, the second smaller: every counter is cleared by the
    call's own kernels."""
    from paper_1108_3126_amd import rx

    progs, s, want = multi_case
    ps = [rx.compile(p.ast, p.root, p.classes, p.search).upload(dev) for p in progs[:3]]
    cfg = _planes(rx, ps)
    d, o = torch.from_numpy(s.data).to(dev), torch.from_numpy(s.offsets).to(dev)
    work = torch.empty(1 << 26, dtype=torch.uint8, device=dev)
    a = rx.match_multi(ps, d, o, config=cfg, work=work).cpu().numpy()
    o2 = torch.from_numpy(s.offsets[:1001].copy()).to(dev)
    b = rx.match_multi(ps, d, o2, config=cfg, work=work).cpu().numpy()
    assert np.array_equal(a, want[:3]) and np.array_equal(b, want[:3, :1000])


# -- captured graphs: the same launches replayed ---------------------------------
@pytest.mark.parametrize("form", ["table", "planes"])
def test_graph_replay_equals_direct(dev, multi_case, form):
    """cfg.graph = 1: the first call instantiates, an identical call replays, a call on other buffers and
    fewer strings updates (or re-instantiates) the graph; every replay equals the oracle, with eager work
    and synchronisation between the replays."""
    from paper_1108_3126_amd import rx

    progs, s, want = multi_case
    ps = [rx.compile(p.ast, p.root, p.classes, p.search).upload(dev) for p in progs[:4]]
    fm = rx.FORM_PLANES if form == "planes" else rx.FORM_TABLE
    if form == "planes":
        rx.prepare_multi(ps)
    d, o = torch.from_numpy(s.data).to(dev), torch.from_numpy(s.offsets).to(dev)
    cfg = rx.multi_config(form=fm, max_bytes=d.numel(), graph=True)
    direct = rx.multi_config(form=fm, max_bytes=d.numel())
    need = rx.lib().rx_match_multi_workspace(s.n, 4, rx.ctypes.byref(cfg))
    work = torch.empty(int(need) + 256, dtype=torch.uint8, device=dev)
    out = torch.empty((4, s.n), dtype=torch.uint8, device=dev)
    c0 = rx.multi_graph_counts()
    for rep in range(3):
        out.fill_(7)
        rx.match_multi(ps, d, o, out=out, config=cfg, work=work)
        torch.cuda.synchronize()
        print(f"graph {form} replay {rep}: counts {rx.multi_graph_counts()}", flush=True)
        assert np.array_equal(out.cpu().numpy(), want[:4]), rep
        # eager work between replays: a direct call on the same workspace, then a torch op
        assert np.array_equal(rx.match_multi(ps, d, o, config=direct, work=work).cpu().numpy(), want[:4])
        torch.cuda.synchronize()
    c1 = rx.multi_graph_counts()
    assert c1[2] - c0[2] == 1 and c1[0] - c0[0] == 2, (c0, c1)
    # other buffers, fewer strings: updated in place or instantiated again
    o2 = torch.from_numpy(s.offsets[:1201].copy()).to(dev)
    out2 = torch.empty((4, 1200), dtype=torch.uint8, device=dev)
    for rep in range(2):
        out2.fill_(7)
        rx.match_multi(ps, d, o2, out=out2, config=cfg, work=work)
        torch.cuda.synchronize()
        assert np.array_equal(out2.cpu().numpy(), want[:4, :1200]), rep
    c2 = rx.multi_graph_counts()
    assert (c2[1] - c1[1]) + (c2[2] - c1[2]) == 1 and c2[0] - c1[0] == 1, (c1, c2)
    # and back to the first call's arguments
    out.fill_(7)
    rx.match_multi(ps, d, o, out=out, config=cfg, work=work)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want[:4])
