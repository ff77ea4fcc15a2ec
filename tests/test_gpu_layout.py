"""rx_match on equal-length consecutive strings: a check on the device sends them
to the bit-sliced kernel (the program's circuit compiled) and the table-form
launch does nothing; any other layout takes the table form.  Every case is
compared with the oracle, and with the table form forced (rx_match_ex, lane
kernel) on the same buffers."""
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


@pytest.fixture(scope="module")
def prog(dev):
    from paper_1108_3126_amd import rx

    p = W.single_program(1)
    P = rx.compile(p.ast, p.root, p.classes, True)
    P.jit()
    return p, P.upload(dev)


def _table(rx, P, d, o):
    return rx.match(P, d, o, launch=(rx.VARIANT_LANE, 0, 0, 0)).cpu().numpy()


def _uniform(p, n, length, seed):
    s, _ = W.single_strings(p, seed=seed, n=n, length=length, plant_frac=0.1)
    return s


@pytest.mark.parametrize("n,length", [(16384, 64), (20000, 256), (40001, 48)])
def test_uniform_layout_matches_oracle(dev, prog, n, length):
    from paper_1108_3126_amd import rx

    p, P = prog
    s = _uniform(p, n, length, seed=n)
    d, o = torch.from_numpy(s.data).to(dev), torch.from_numpy(s.offsets).to(dev)
    got = rx.match(P, d, o).cpu().numpy()
    want = oracle.match(p.ast, p.root, p.classes, True, s.data, s.offsets, threads=8)
    assert want.sum() > 0 and np.array_equal(got, want)
    assert np.array_equal(_table(rx, P, d, o), want)


def test_uniform_layout_at_an_offset(dev, prog):
    """The first string 256 bytes into the buffer (still 16-byte aligned): the sliced kernel reads from there."""
    from paper_1108_3126_amd import rx

    p, P = prog
    s = _uniform(p, 18000, 128, seed=3)
    buf = np.concatenate([np.full(256, 0x7a, np.uint8), s.data])
    d, o = torch.from_numpy(buf).to(dev), torch.from_numpy(s.offsets + 256).to(dev)
    want = oracle.match(p.ast, p.root, p.classes, True, s.data, s.offsets, threads=8)
    assert np.array_equal(rx.match(P, d, o).cpu().numpy(), want)


@pytest.mark.parametrize("flaw", ["one_longer", "unaligned", "length_40", "gap_at_end"])
def test_other_layouts_take_the_table_form(dev, prog, flaw):
    from paper_1108_3126_amd import rx

    p, P = prog
    n = 17000
    if flaw == "one_longer":
        # string 9000 one byte longer: every later offset moves
        strs = [bytes(x) for x in np.split(_uniform(p, n, 64, seed=5).data, n)]
        strs[9000] = strs[9000] + b"q"
        s = W.pack(strs)
        buf, offs = s.data, s.offsets
    elif flaw == "unaligned":
        s = _uniform(p, n, 64, seed=6)
        buf, offs = np.concatenate([np.zeros(1, np.uint8), s.data]), s.offsets + 1
    elif flaw == "length_40":
        s = _uniform(p, n, 40, seed=7)
        buf, offs = s.data, s.offsets
    else:
        # equal strides but the last string ends early
        s = _uniform(p, n, 64, seed=8)
        buf, offs = s.data, s.offsets.copy()
        offs[-1] -= 3
    d, o = torch.from_numpy(buf).to(dev), torch.from_numpy(offs).to(dev)
    want = oracle.match(p.ast, p.root, p.classes, True, buf, offs, threads=8)
    got = rx.match(P, d, o).cpu().numpy()
    assert np.array_equal(got, want)


def test_slots_wrap_over_many_calls(dev, prog):
    """More calls than layout slots, alternating equal-length and uneven batches, on one stream: every
    result equals the oracle's."""
    from paper_1108_3126_amd import rx

    p, P = prog
    n = 16384
    a = _uniform(p, n, 16, seed=11)
    strs = [bytes(x) for x in np.split(_uniform(p, n, 16, seed=12).data, n)]
    strs[5] = strs[5][:7]
    b = W.pack(strs)
    want_a = oracle.match(p.ast, p.root, p.classes, True, a.data, a.offsets, threads=8)
    want_b = oracle.match(p.ast, p.root, p.classes, True, b.data, b.offsets, threads=8)
    da, oa = torch.from_numpy(a.data).to(dev), torch.from_numpy(a.offsets).to(dev)
    db, ob = torch.from_numpy(b.data).to(dev), torch.from_numpy(b.offsets).to(dev)
    calls = 4200
    out = torch.empty((calls, n), dtype=torch.uint8, device=dev)
    for k in range(calls):
        if k % 2 == 0:
            rx.match(P, da, oa, out=out[k])
        else:
            rx.match(P, db, ob, out=out[k])
    got = out.cpu().numpy()
    assert np.array_equal(got[0::2], np.broadcast_to(want_a, got[0::2].shape))
    assert np.array_equal(got[1::2], np.broadcast_to(want_b, got[1::2].shape))


def test_equal_lengths_take_the_sliced_kernel(dev, prog):
    """200,000 strings of 256 bytes: the sliced path is several times faster than the table form (the
    kernel that ran is seen by its speed; both give the oracle's bits on a sample)."""
    from paper_1108_3126_amd import rx

    p, P = prog
    s = _uniform(p, 200000, 256, seed=21)
    d, o = torch.from_numpy(s.data).to(dev), torch.from_numpy(s.offsets).to(dev)
    out = torch.empty(s.n, dtype=torch.uint8, device=dev)

    def timed(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_auto = timed(lambda: rx.match(P, d, o, out=out))
    got = out.cpu().numpy()
    t_table = timed(lambda: rx.match(P, d, o, out=out, launch=(rx.VARIANT_LANE, 0, 0, 0)))
    print(f"rx_match equal lengths: {t_auto:.3f} ms, table form forced: {t_table:.3f} ms", flush=True)
    idx = np.random.default_rng(0).choice(s.n, size=3000, replace=False).astype(np.int64)
    want = oracle.match(p.ast, p.root, p.classes, True, s.data, s.offsets, index=idx)
    assert np.array_equal(got[idx], want)
    assert np.array_equal(out.cpu().numpy(), got)
    assert t_auto * 2 < t_table
