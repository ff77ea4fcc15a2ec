"""GPU parity at the workloads' full sizes, in the launch configurations the
benchmark times: sampled outputs against the oracle one by one, and
properties that hold at any size (planted strings match; closed forms of the
nested-star families; every result the same alone and in the mix)."""
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


@pytest.mark.timeout(300)
def test_single_program_1m_x_256(dev):
    """1M strings of 256 bytes, ~200-node expression searched, default launch (the bench's)."""
    from paper_1108_3126_amd import rx

    prog = W.single_program(1)
    s, planted = W.single_strings(prog, seed=1, n=1_000_000, length=256)
    p = rx.compile(prog.ast, prog.root, prog.classes, True).upload(dev).jit()
    print("full single: staging", p.jit_staging(), flush=True)
    d = torch.from_numpy(s.data).to(dev)
    out = rx.match_fixed(p, d, 256, s.n)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert got[planted].all()
    # every one of the 1M results against the oracle (about 10 s on the host's cores)
    want_all = oracle.match(prog.ast, prog.root, prog.classes, True, s.data, s.offsets)
    bad = np.nonzero(got != want_all)[0]
    assert bad.size == 0, bad[:10]
    rng = np.random.default_rng(2024)
    idx = np.unique(np.concatenate([rng.choice(s.n, 3000, replace=False), np.arange(0, s.n, 2048),
                                    np.arange(2047, s.n, 2048), [s.n - 1], planted[:300]])).astype(np.int64)
    # the same batch through the table-form kernel: every string, bit for bit
    out2 = rx.match_fixed(p, d, 256, s.n, launch=(rx.VARIANT_LANE, 0, 0, 0))
    torch.cuda.synchronize()
    assert np.array_equal(out2.cpu().numpy(), got)
    # earliest accepting prefix, sliced form: accepted iff the bit is set; a sample on every prefix
    first = rx.match_first_fixed(p, d, 256, s.n)
    torch.cuda.synchronize()
    first = first.cpu().numpy()
    assert np.array_equal((first >= 0).astype(np.uint8), got) and first.max() <= 256
    sub = np.unique(np.concatenate([idx[::40], planted[:20], [s.n - 1]]))
    pre = []
    for i in sub:
        w = bytes(s.data[i * 256:(i + 1) * 256])
        pre += [w[:k] for k in range(257)]
    ps = W.pack(pre)
    acc = oracle.match(prog.ast, prog.root, prog.classes, True, ps.data, ps.offsets).reshape(len(sub), 257)
    want_first = np.where(acc.any(axis=1), acc.argmax(axis=1), -1)
    assert np.array_equal(first[sub], want_first)


@pytest.mark.timeout(400)
def test_multi_16_programs_4m_lines(dev):
    """16 programs x 4M log-normal lines in one batched launch, default and tuned configurations."""
    from paper_1108_3126_amd import autotune, rx

    progs = W.multi_programs(2)
    lines = W.multi_lines(2)
    ps = [rx.compile(q.ast, q.root, q.classes, True).upload(dev) for q in progs]
    d = torch.from_numpy(lines.data).to(dev)
    o = torch.from_numpy(lines.offsets).to(dev)
    out = rx.match_multi(ps, d, o)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    cfg, info = autotune.tune_multi(ps, d, o, budget_runs=12, use_cache=False)
    print("full multi: tuned", info, flush=True)
    out2 = rx.match_multi(ps, d, o, config=cfg)
    torch.cuda.synchronize()
    assert np.array_equal(out2.cpu().numpy(), got)
    # the plane form (the benchmark's): every one of the 64M results equals the table form's
    rx.prepare_multi(ps)
    out3 = rx.match_multi(ps, d, o, config=rx.multi_config(form=rx.FORM_PLANES))
    torch.cuda.synchronize()
    bad = np.argwhere(out3.cpu().numpy() != got)
    assert bad.size == 0, bad[:10]
    # a seeded subsample of 200,000 (line, program) pairs plus every line longer than 1 KiB against
    # every program, through the oracle
    rng = np.random.default_rng(7)
    pair_line = rng.integers(0, lines.n, 200_000)
    pair_prog = rng.integers(0, len(progs), 200_000)
    lens = np.diff(lines.offsets)
    long_ids = np.nonzero(lens > 1024)[0]
    assert long_ids.size > 10_000
    for k, q in enumerate(progs):
        idx = np.unique(np.concatenate([pair_line[pair_prog == k], long_ids, [0, lines.n - 1]])).astype(np.int64)
        want = oracle.match(q.ast, q.root, q.classes, True, lines.data, lines.offsets, index=idx)
        bad = np.nonzero(got[k][idx] != want)[0]
        assert bad.size == 0, (k, idx[bad[:10]])


@pytest.mark.parametrize("family,k", [("nested", 819), ("altstar", 585)])
def test_pathological_long_strings(dev, family, k):
    """4,096-node programs on 256 strings of length 10^4 and 10^5: the closed form a^n rejected, a^(n-1) t accepted."""
    from paper_1108_3126_amd import rx

    prog = W.pathological_program(family, k)
    p = rx.compile(prog.ast, prog.root).upload(dev)
    for n_len in (10_000, 100_000):
        s = W.pathological_strings(family, n_len, count=256)
        print(f"pathological {family} n={n_len}", flush=True)
        out = rx.match_fixed(p, torch.from_numpy(s.data).to(dev), n_len, s.n)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert got[:128].sum() == 0 and got[128:].all()


def test_serving_full_distribution(dev):
    """Requests drawn from the serving distribution (up to 10^4 strings of up to 8 KB): alone, in
    the mix and through the plain path give the same bits; a sample equals the oracle."""
    from paper_1108_3126_amd import server

    reqs = [W.serving_request(3, i) for i in range(60)]
    with server.Server(use_graph=True) as srv:
        alone = [srv.wait(srv.submit(p, s.data, s.offsets)) for p, s in reqs]
        ids = [srv.submit(p, s.data, s.offsets) for p, s in reqs]
        mix = [srv.wait(r) for r in ids]
        st = srv.stats()
    print("full serving:", {k: st[k] for k in ("steps", "graph_steps", "p50_us", "p99_us")}, flush=True)
    assert st["steps"] < 2 * len(reqs)
    for (p, s), a, b in zip(reqs, alone, mix):
        assert np.array_equal(a, b)
        assert np.array_equal(server.plain_match(p, s.data, s.offsets), a)
        if s.n:
            idx = np.unique(np.linspace(0, s.n - 1, min(12, s.n)).astype(np.int64))
            want = oracle.match(p.ast, p.root, p.classes, p.search, s.data, s.offsets, index=idx)
            assert np.array_equal(a[idx], want)
