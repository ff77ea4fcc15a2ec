"""Host side of chunk-parallel matching: the workspace size follows the chunk rule (the requested count,
at most 4096 and at most one chunk per byte, every chunk non-empty; by default about sqrt(length / 2) for lane
rows and sqrt(length / 20) for wavefront rows)."""
import ctypes

import pytest

from paper_1108_3126_amd import rx
from paper_1108_3126_amd import workloads as W


def expect(p, C):
    """Sets of 1 + (C - 1)(L + 1) rows (u32 words, padded to 8 bytes), then one int64 per row."""
    rows = 1 + (C - 1) * (p.info.n_leaves + 1)
    return ((rows * p.info.words * 4 + 7) // 8) * 8 + 8 * rows


def ws(p, length, chunks):
    n = ctypes.c_size_t()
    rc = rx.lib().rx_match_long_workspace(p.handle, length, chunks, ctypes.byref(n))
    if rc:
        raise rx.RxError(rc, "workspace")
    return n.value


@pytest.mark.parametrize("search", [False, True])
def test_workspace_rule(search):
    prog = W.single_program(1)
    p = rx.compile(prog.ast, prog.root, prog.classes, search)
    assert ws(p, 0, 0) == expect(p, 1)                  # one chunk, row 0 only
    assert ws(p, 1000, 1) == expect(p, 1)
    assert ws(p, 1000, 10) == expect(p, 10)
    assert ws(p, 10, 100) == expect(p, 10)              # at most one chunk per byte
    assert ws(p, 1001, 10) == expect(p, 10)             # chunks of 101 bytes: 10 non-empty
    assert ws(p, 1000, 7) == expect(p, 7)               # chunks of 143 bytes: 7
    assert ws(p, 20_000, 0) == expect(p, 100)           # default for lane rows: sqrt(20000 / 2) = 100
    assert ws(p, 1 << 40, 0) == expect(p, 4096)         # capped at 4096
    with pytest.raises(rx.RxError):
        ws(p, -1, 0)


def test_workspace_rule_wavefront_rows():
    big = W.pathological_program("nested", 819)
    p = rx.compile(big.ast, big.root)
    assert p.info.words > 16
    assert ws(p, 200_000, 0) == expect(p, 100)   # sqrt(200000 / 20) = 100


@pytest.mark.parametrize("fn", ["match_long", "match_first_long"])
def test_length_beyond_the_tensor_is_refused_before_any_launch(fn):
    # the row kernels read bytes [0, length): a length past the tensor is refused on the host
    import torch

    prog = W.single_program(1)
    p = rx.compile(prog.ast, prog.root, prog.classes, True)
    data = torch.zeros(100, dtype=torch.uint8)
    for bad in (101, -1, 1 << 40):
        with pytest.raises(ValueError):
            getattr(rx, fn)(p, data, bad)
    with pytest.raises(TypeError):   # a host tensor never reaches a launch either
        getattr(rx, fn)(p, data, 100)
