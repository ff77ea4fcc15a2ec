"""The device image of the node-per-thread machine: header, one record per node of d[] (kind | label
<< 8, c0, c1, cont) matching rx_program_nodes, and the classes as 256-bit masks."""
import struct

import numpy as np

from paper_1108_3126_amd import rx
from paper_1108_3126_amd import workloads as W


def test_node_image_matches_node_array():
    for search in (False, True):
        prog = W.single_program(1)
        p = rx.compile(prog.ast, prog.root, prog.classes, search)
        img = p.node_image()
        m, ncls = struct.unpack_from("<ii", img, 0)
        nodes = p.nodes()
        assert m == len(nodes) and len(img) == 16 + 16 * m + 32 * ncls
        for i, (kind, c0, c1, label, cont) in enumerate(nodes):
            kl, r0, r1, rc = struct.unpack_from("<iiii", img, 16 + 16 * i)
            assert (kl & 0xFF, r0, r1, rc) == (kind, c0, c1, cont)
            if kind in (rx.BYTE, rx.CLASS):
                assert kl >> 8 == label
        # the caller's classes first, as 256-bit masks in little-endian 32-bit words
        for k, words in enumerate(prog.classes):
            got = np.frombuffer(img, np.uint32, 8, 16 + 16 * m + 32 * k)
            want = np.frombuffer(np.asarray(words, np.uint64).tobytes(), np.uint32)
            assert np.array_equal(got, want)
        assert ncls == len(prog.classes) + (1 if search else 0)


def test_node_image_short_buffer():
    import ctypes

    p = rx.compile_regex(b"a*b")
    n = ctypes.c_size_t()
    assert rx.lib().rx_program_node_image(p.handle, None, 0, ctypes.byref(n)) == 0
    buf = ctypes.create_string_buffer(n.value)
    assert rx.lib().rx_program_node_image(p.handle, buf, n.value - 1, ctypes.byref(n)) == rx.RX_EINVAL
