"""GPU: the allocation-free chunk-parallel entry point (rx_match_long_noalloc)
gives rx_match_long's result, on two calls in a row (the second one smaller),
called through the C interface; an explicit chunk count whose rows exceed the
static workspace is refused."""
import ctypes

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


def _noalloc(rx, p, d, length, chunks, out):
    stream = torch.cuda.current_stream()
    return rx.lib().rx_match_long_noalloc(p.handle, ctypes.c_void_p(d.data_ptr()), int(length), int(chunks),
                                          ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream))


def test_noalloc_equals_workspace_form_twice(dev):
    from paper_1108_3126_amd import rx

    prog = W.single_program(1)
    p = rx.compile(prog.ast, prog.root, prog.classes, True).upload(dev)
    member, _ = W.single_strings(prog, seed=41, n=1, length=256, plant_frac=1.0)
    rng = np.random.default_rng(5)
    text = rng.integers(97, 123, size=1 << 20, dtype=np.uint8)
    text[-256:] = member.data            # a member in the last 256 bytes: every chunk matters
    d = torch.from_numpy(text).to(dev)
    out = torch.full((1,), 7, dtype=torch.uint8, device=dev)
    # first call: 1 MiB, default chunk count; second call: a shorter prefix with an explicit count
    for length, chunks in ((text.size, 0), (300_000, 37), (5_000, 0)):
        print(f"noalloc: length {length} chunks {chunks}", flush=True)
        assert _noalloc(rx, p, d, length, chunks, out) == rx.RX_OK, rx.lib().rx_last_error()
        got = int(out.cpu().numpy()[0])
        want = int(rx.match_long(p, d, length, chunks).cpu().numpy()[0])
        assert got == want
        if length <= 5_000:
            o = oracle.match(prog.ast, prog.root, prog.classes, True, text[:length], np.array([0, length]))
            assert got == int(o[0])
    assert int(out.cpu().numpy()[0]) in (0, 1)


def test_noalloc_pathological_and_errors(dev):
    from paper_1108_3126_amd import rx

    prog = W.pathological_program("altstar", 585)   # 4,096 nodes: wavefront rows, large sets
    p = rx.compile(prog.ast, prog.root).upload(dev)
    s = W.pathological_strings("altstar", 20_000, count=2)
    for k, want in ((0, 0), (1, 1)):          # a^n is rejected, a^(n-1) c accepted
        d = torch.from_numpy(s.data[k * 20_000:(k + 1) * 20_000].copy()).to(dev)
        out = torch.empty(1, dtype=torch.uint8, device=dev)
        assert _noalloc(rx, p, d, 20_000, 0, out) == rx.RX_OK, rx.lib().rx_last_error()
        assert int(out.cpu().numpy()[0]) == want
    # an explicit count whose rows do not fit the 16 MiB array
    need = ctypes.c_size_t()
    assert rx.lib().rx_match_long_workspace(p.handle, 20_000, 4000, ctypes.byref(need)) == rx.RX_OK
    assert need.value > 16 << 20
    out = torch.empty(1, dtype=torch.uint8, device=dev)
    assert _noalloc(rx, p, d, 20_000, 4000, out) == rx.RX_ETOOBIG
