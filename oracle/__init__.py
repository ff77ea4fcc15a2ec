"""CPU oracle package (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  It shares no code with the HIP library in
``paper_1108_3126_amd``; neither imports the other.

* ``pwpi``      -- pure-Python engines written from the paper (big-step, EKW,
                   PW-pi, generic and sequential lockstep) for tiny inputs.
* ``rx_oracle.c`` -- the C twin of the PW-pi backtracking oracle, threaded over
                   strings, used for parity at real sizes.  ``build()``
                   compiles it with gcc; ``match()`` calls it through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rx_oracle.c")
LIB = os.path.join(HERE, "librx_oracle.so")

AST_DTYPE = np.dtype(
    [("kind", np.uint8), ("byte", np.uint8), ("cls", np.uint16), ("c0", np.int32), ("c1", np.int32)]
)

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, pthreads) into oracle/librx_oracle.so."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-Wall", "-o", tmp, SRC]
        )
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        lib.rxo_match.restype = ctypes.c_int
        lib.rxo_match.argtypes = [
            ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
            ctypes.c_int,
        ]
        lib.rxo_heap_cont.restype = ctypes.c_int
        lib.rxo_heap_cont.argtypes = [
            ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_int,
        ]
        _lib = lib
    return _lib


def as_ast(ast) -> np.ndarray:
    """Accept a structured array or a list of (kind, byte, cls, c0, c1) tuples."""
    if isinstance(ast, np.ndarray) and ast.dtype == AST_DTYPE:
        return np.ascontiguousarray(ast)
    return np.array([tuple(int(v) for v in a) for a in ast], dtype=AST_DTYPE)


def as_classes(classes) -> np.ndarray:
    """Classes as an (n, 4) uint64 array.  The encoding of each entry comes from its type (as in
    ``pwpi._class_set``): an int is a 256-bit mask, ``pwpi.Words`` or a numpy uint64 row holds
    four 64-bit words, any other iterable lists the member bytes."""
    from .pwpi import _class_set

    if isinstance(classes, np.ndarray) and classes.dtype == np.uint64:
        return np.ascontiguousarray(classes.reshape(-1, 4))
    out = np.zeros((max(len(classes), 1), 4), dtype=np.uint64)
    for i, c in enumerate(classes):
        for b in _class_set(c):
            out[i, b >> 6] |= np.uint64(1) << np.uint64(b & 63)
    return out


def default_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def match(ast, root, classes, search, data, offsets, index=None, threads=None) -> np.ndarray:
    """out[k] = 1 iff string k (or index[k]) is matched, by the C PW-pi oracle."""
    lib = _load()
    ast = as_ast(ast)
    cls = as_classes(classes)
    data = np.ascontiguousarray(np.frombuffer(bytes(data), np.uint8) if isinstance(data, (bytes, bytearray)) else data, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n_all = len(offsets) - 1
    if index is not None:
        index = np.ascontiguousarray(index, dtype=np.int64)
        if index.size and (index.min() < 0 or index.max() >= n_all):
            raise IndexError("string index out of range")
        n = len(index)
    else:
        n = n_all
    out = np.zeros(max(n, 1), dtype=np.uint8)
    if data.size == 0:
        data = np.zeros(1, np.uint8)
    rc = lib.rxo_match(
        ast.ctypes.data, len(ast), int(root), cls.ctypes.data, len(classes), int(bool(search)),
        data.ctypes.data, offsets.ctypes.data, index.ctypes.data if index is not None else None,
        n, out.ctypes.data, int(threads or default_threads()),
    )
    if rc == -1:
        raise ValueError("malformed AST")
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return out[:n]


def heap_cont(ast, root, classes=(), search=False) -> list:
    """The oracle heap's cont table (null = -1), including PLUS companions at the end."""
    lib = _load()
    ast = as_ast(ast)
    cls = as_classes(classes)
    cap = len(ast) + 16 + int(np.sum(ast["kind"] == 6))
    buf = np.zeros(cap, dtype=np.int32)
    m = lib.rxo_heap_cont(ast.ctypes.data, len(ast), int(root), cls.ctypes.data, len(classes), int(bool(search)), buf.ctypes.data, cap)
    if m < 0:
        raise ValueError("malformed AST")
    return buf[:m].tolist()
