"""Python handle on the C++ serving loop (rx_server_*): submit requests from
any thread, wait for their bits, read latency percentiles.  Strings are host
numpy arrays; the server copies them, batches them with whatever else is
pending and runs them on the device."""
from __future__ import annotations

import ctypes

import numpy as np

from . import rx


def _ast_classes(prog):
    a = rx.as_ast(prog.ast)
    c = rx.as_classes(prog.classes)
    return a, c


class Server:
    def __init__(self, hbm_budget=0, step_bytes=0, step_strings=0, step_requests=0, slots=0, use_graph=True,
                 block=0, grid=0, program_slots=0):
        cfg = rx.rx_server_config(int(hbm_budget), int(step_bytes), int(step_strings), int(step_requests),
                                  int(slots), int(bool(use_graph)), int(block), int(grid), int(program_slots))
        h = ctypes.c_void_p()
        rx._check(rx.lib().rx_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._n = {}

    def close(self):
        if self._h is not None and self._h.value:
            rx.lib().rx_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, prog, data, offsets) -> int:
        """prog: a workloads.Program (AST, root, classes, search); data/offsets: host arrays."""
        a, c = _ast_classes(prog)
        data = np.ascontiguousarray(data, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        n = len(offsets) - 1
        rid = ctypes.c_int64()
        rx._check(rx.lib().rx_server_submit(self._h, a.ctypes.data, len(a), int(prog.root),
                                            c.ctypes.data if len(c) else None, len(c),
                                            rx.RX_SEARCH if prog.search else 0,
                                            data.ctypes.data if data.size else None, offsets.ctypes.data, n,
                                            ctypes.byref(rid)))
        self._n[rid.value] = n
        return rid.value

    def wait(self, rid: int, timeout_us: int = -1) -> np.ndarray:
        n = self._n.get(rid, 0)
        out = np.zeros(max(n, 1), np.uint8)
        rx._check(rx.lib().rx_server_wait(self._h, int(rid), out.ctypes.data, int(timeout_us)))
        self._n.pop(rid, None)
        return out[:n]

    def stats(self) -> dict:
        s = rx.rx_server_counters()
        rx._check(rx.lib().rx_server_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in s._fields_}

    def reset_stats(self):
        rx._check(rx.lib().rx_server_reset_stats(self._h))


def plain_match(prog, data, offsets) -> np.ndarray:
    """The per-request plain path (compile, upload, copy in, launch, copy out, sync, free)."""
    a, c = _ast_classes(prog)
    data = np.ascontiguousarray(data, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n = len(offsets) - 1
    out = np.zeros(max(n, 1), np.uint8)
    rx._check(rx.lib().rx_plain_match(a.ctypes.data, len(a), int(prog.root), c.ctypes.data if len(c) else None,
                                      len(c), rx.RX_SEARCH if prog.search else 0,
                                      data.ctypes.data if data.size else None, offsets.ctypes.data, n,
                                      out.ctypes.data))
    return out[:n]


class PlainContext:
    """The plain path with its stream and device buffers made once (rx_plain_*): per request it
    compiles, uploads, copies in, launches once, copies out and synchronises."""

    def __init__(self, max_bytes: int, max_strings: int):
        h = ctypes.c_void_p()
        rx._check(rx.lib().rx_plain_create(int(max_bytes), int(max_strings), ctypes.byref(h)))
        self._h = h

    def match(self, prog, data, offsets) -> np.ndarray:
        a, c = _ast_classes(prog)
        data = np.ascontiguousarray(data, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        n = len(offsets) - 1
        out = np.zeros(max(n, 1), np.uint8)
        rx._check(rx.lib().rx_plain_run(self._h, a.ctypes.data, len(a), int(prog.root),
                                        c.ctypes.data if len(c) else None, len(c),
                                        rx.RX_SEARCH if prog.search else 0,
                                        data.ctypes.data if data.size else None, offsets.ctypes.data, n,
                                        out.ctypes.data))
        return out[:n]

    def close(self):
        if self._h is not None and self._h.value:
            rx.lib().rx_plain_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
