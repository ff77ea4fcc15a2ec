"""Host side of chunk-parallel matching: the workspace size follows the chunk rule (the requested count,
at most 4096 and at most one chunk per byte, every chunk non-empty; by default about sqrt(length / 2) for lane
rows and sqrt(length / 20) for wavefront rows)."""
import ctypes

import pytest

from paper_1108_3126_amd import rx
from paper_1108_3126_amd import workloads as W


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
    L, Wd = p.info.n_leaves, p.info.words
    row = 4 * Wd
    assert ws(p, 0, 0) == row                      # one chunk, row 0 only
    assert ws(p, 1000, 1) == row
    assert ws(p, 1000, 10) == (1 + 9 * (L + 1)) * row
    assert ws(p, 10, 100) == (1 + 9 * (L + 1)) * row   # at most one chunk per byte
    assert ws(p, 1001, 10) == (1 + 9 * (L + 1)) * row  # chunks of 101 bytes: 10 non-empty
    assert ws(p, 1000, 7) == (1 + 6 * (L + 1)) * row   # chunks of 143 bytes: 7
    assert ws(p, 20_000, 0) == (1 + 99 * (L + 1)) * row   # default for lane rows: sqrt(20000 / 2) = 100
    assert ws(p, 1 << 40, 0) == (1 + 4095 * (L + 1)) * row  # capped at 4096
    with pytest.raises(rx.RxError):
        ws(p, -1, 0)


def test_workspace_rule_wavefront_rows():
    big = W.pathological_program("nested", 819)
    p = rx.compile(big.ast, big.root)
    L, Wd = p.info.n_leaves, p.info.words
    assert Wd > 16
    assert ws(p, 200_000, 0) == (1 + 99 * (L + 1)) * 4 * Wd   # sqrt(200000 / 20) = 100
