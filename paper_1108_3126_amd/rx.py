"""Python binding of the C interface in include/rx.h (ctypes; argument
marshalling only -- every step of matching runs in the HIP library).

PyTorch supplies device memory and streams: strings, offsets and results are
torch tensors on the GPU, and calls are enqueued on the current torch stream.
The library must have been built (``python -m paper_1108_3126_amd.build``);
importing this module fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librx.so")

RX_OK, RX_EINVAL, RX_ETOOBIG, RX_ENOTUPLOADED, RX_EHIP, RX_EBUSY, RX_ENOMEM, RX_EJIT, RX_ETIMEOUT = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
EPS, BYTE, CLASS, CAT, ALT, STAR, PLUS, OPT, PLUSLOOP = range(9)
RX_SEARCH = 1
VARIANT_AUTO, VARIANT_LANE, VARIANT_WAVE, VARIANT_SLICED, VARIANT_CHUNKS = range(5)

AST_DTYPE = np.dtype(
    [("kind", np.uint8), ("byte", np.uint8), ("cls", np.uint16), ("c0", np.int32), ("c1", np.int32)]
)


class RxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rx error {code}: {msg}")
        self.code = code


class rx_info(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int32), ("n_leaves", ctypes.c_int32), ("words", ctypes.c_int32),
        ("nullable", ctypes.c_int32), ("suffix_any", ctypes.c_int32), ("search", ctypes.c_int32),
        ("table_bytes", ctypes.c_int64), ("depth", ctypes.c_int32), ("n_classes", ctypes.c_int32),
    ]


class rx_node(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("c0", ctypes.c_int32), ("c1", ctypes.c_int32),
                ("label", ctypes.c_int32), ("cont", ctypes.c_int32)]


class rx_multi_config(ctypes.Structure):
    _fields_ = [("n_edges", ctypes.c_int32), ("edges", ctypes.c_int32 * 15), ("block", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("form", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("max_bytes", ctypes.c_int64)]


FORM_TABLE, FORM_PLANES = 0, 1


def multi_config(edges=None, block=0, grid=0, form=FORM_TABLE, max_bytes=0, graph=False) -> "rx_multi_config":
    c = rx_multi_config()
    if edges:
        c.n_edges = len(edges)
        for i, e in enumerate(edges):
            c.edges[i] = int(e)
    c.block, c.grid = int(block), int(grid)
    c.form, c.max_bytes, c.graph = int(form), int(max_bytes), int(bool(graph))
    return c


class rx_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_int64), ("step_bytes", ctypes.c_int64), ("step_strings", ctypes.c_int64),
                ("step_requests", ctypes.c_int32), ("slots", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("block", ctypes.c_int32), ("grid", ctypes.c_int32), ("program_slots", ctypes.c_int32)]


class rx_server_counters(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "rejected", "queued", "max_queue", "steps",
                                               "graph_steps", "strings", "bytes", "cache_hits", "cache_misses",
                                               "cache_evictions")] + \
               [(k, ctypes.c_double) for k in ("p50_us", "p99_us", "mean_us", "max_us", "wall_s", "pack_ms",
                                                "device_ms")]


class rx_launch(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("block", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("unroll", ctypes.c_int32)]


_VP, _I32, _I64, _U32, _SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t

# name -> (restype, argtypes); every symbol include/rx.h declares
SIGNATURES = {
    "rx_compile": (ctypes.c_int, [_VP, _I32, _I32, _VP, _I32, _U32, ctypes.POINTER(_VP)]),
    "rx_program_free": (None, [_VP]),
    "rx_program_info": (ctypes.c_int, [_VP, ctypes.POINTER(rx_info)]),
    "rx_program_nodes": (ctypes.c_int, [_VP, _VP, _I32, ctypes.POINTER(_I32)]),
    "rx_program_sets": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "rx_program_upload": (ctypes.c_int, [_VP, _VP, _SZ, _VP]),
    "rx_match": (ctypes.c_int, [_VP, _VP, _VP, _I64, _VP, _VP]),
    "rx_match_ex": (ctypes.c_int, [_VP, _VP, _VP, _I64, _VP, ctypes.POINTER(rx_launch), _VP]),
    "rx_match_fixed": (ctypes.c_int, [_VP, _VP, _I64, _I64, _VP, _VP]),
    "rx_match_fixed_ex": (ctypes.c_int, [_VP, _VP, _I64, _I64, _VP, ctypes.POINTER(rx_launch), _VP]),
    "rx_program_jit": (ctypes.c_int, [_VP, ctypes.c_char_p]),
    "rx_program_jit_source": (ctypes.c_int, [_VP, ctypes.c_char_p, _SZ, ctypes.POINTER(_SZ)]),
    "rx_program_jit_stats": (ctypes.c_int, [_VP, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "rx_program_jit_staging": (ctypes.c_int, [_VP, ctypes.POINTER(_I32)]),
    "rx_program_jit_guard": (ctypes.c_int, [_VP, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "rx_program_jit_selfcheck": (ctypes.c_int, [_VP, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "rx_match_multi_prepare": (ctypes.c_int, [ctypes.POINTER(_VP), _I32, ctypes.c_char_p, ctypes.POINTER(_I32)]),
    "rx_program_jit_planes_source": (ctypes.c_int, [_VP, ctypes.c_char_p, _SZ, ctypes.POINTER(_SZ)]),
    "rx_isa_check_staging": (ctypes.c_int, [ctypes.c_char_p, _SZ, ctypes.c_char_p, ctypes.c_char_p,
                                            ctypes.POINTER(_I32)]),
    "rx_match_first": (ctypes.c_int, [_VP, _VP, _VP, _I64, _VP, _VP]),
    "rx_match_first_fixed": (ctypes.c_int, [_VP, _VP, _I64, _I64, _VP, _VP]),
    "rx_program_node_image": (ctypes.c_int, [_VP, _VP, _SZ, ctypes.POINTER(_SZ)]),
    "rx_match_long_workspace": (ctypes.c_int, [_VP, _I64, _I32, ctypes.POINTER(_SZ)]),
    "rx_trace_enabled": (ctypes.c_int, []),
    "rx_match_first_long": (ctypes.c_int, [_VP, _VP, _I64, _I32, _VP, _SZ, _VP, _VP]),
    "rx_match_long": (ctypes.c_int, [_VP, _VP, _I64, _I32, _VP, _SZ, _VP, _VP]),
    "rx_match_long_noalloc": (ctypes.c_int, [_VP, _VP, _I64, _I32, _VP, _VP]),
    "rx_match_nodes": (ctypes.c_int, [_VP, _VP, _VP, _VP, _I64, _VP, _VP]),
    "rx_parse": (ctypes.c_int, [ctypes.c_char_p, _SZ, _VP, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32), _VP, _I32,
                                ctypes.POINTER(_I32)]),
    "rx_match_multi_workspace": (ctypes.c_int64, [_I64, _I32, ctypes.POINTER(rx_multi_config)]),
    "rx_multi_graph_counts": (ctypes.c_int, [ctypes.POINTER(_I64)]),
    "rx_match_multi": (ctypes.c_int, [ctypes.POINTER(_VP), _I32, _VP, _VP, _I64, _VP, _VP, _SZ,
                                      ctypes.POINTER(rx_multi_config), _VP]),
    "rx_autotune": (ctypes.c_int, [_VP, _VP, _VP, _I64, _I64, _VP, _I32, ctypes.POINTER(rx_launch),
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I32), _VP]),
    "rx_autotune_multi": (ctypes.c_int, [ctypes.POINTER(_VP), _I32, _VP, _VP, _I64, _VP, _VP, _SZ, _I32,
                                         ctypes.POINTER(rx_multi_config), ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(_I32), _VP]),
    "rx_server_create": (ctypes.c_int, [ctypes.POINTER(rx_server_config), ctypes.POINTER(_VP)]),
    "rx_server_destroy": (None, [_VP]),
    "rx_server_submit": (ctypes.c_int, [_VP, _VP, _I32, _I32, _VP, _I32, _U32, _VP, _VP, _I64,
                                        ctypes.POINTER(_I64)]),
    "rx_server_wait": (ctypes.c_int, [_VP, _I64, _VP, _I64]),
    "rx_server_stats": (ctypes.c_int, [_VP, ctypes.POINTER(rx_server_counters)]),
    "rx_server_reset_stats": (ctypes.c_int, [_VP]),
    "rx_plain_match": (ctypes.c_int, [_VP, _I32, _I32, _VP, _I32, _U32, _VP, _VP, _I64, _VP]),
    "rx_plain_create": (ctypes.c_int, [_I64, _I64, ctypes.POINTER(_VP)]),
    "rx_plain_run": (ctypes.c_int, [_VP, _VP, _I32, _I32, _VP, _I32, _U32, _VP, _VP, _I64, _VP]),
    "rx_plain_destroy": (None, [_VP]),
    "rx_stream_copy": (ctypes.c_int, [_VP, _VP, _I64, _VP]),
    "rx_last_error": (ctypes.c_char_p, []),
    "rx_version": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """The loaded librx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_1108_3126_amd.build")
        # torch brings its own HIP runtime and hiprtc; loading it first makes the
        # library bind to those, so the process holds one HIP runtime whose
        # device pointers and streams both sides share
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != RX_OK:
        raise RxError(rc, lib().rx_last_error().decode(errors="replace"))
    return rc


def as_ast(ast) -> np.ndarray:
    if isinstance(ast, np.ndarray) and ast.dtype == AST_DTYPE:
        return np.ascontiguousarray(ast)
    if isinstance(ast, np.ndarray) and ast.dtype.names == AST_DTYPE.names:
        return np.ascontiguousarray(ast.astype(AST_DTYPE))
    return np.array([tuple(int(v) for v in a) for a in ast], dtype=AST_DTYPE)


def as_classes(classes) -> np.ndarray:
    if classes is None:
        return np.zeros((0, 4), np.uint64)
    if isinstance(classes, np.ndarray) and classes.dtype == np.uint64:
        return np.ascontiguousarray(classes.reshape(-1, 4))
    # each entry's encoding comes from its type: an int is a 256-bit mask, a numpy uint64 row is the
    # four words of rx_class, any other iterable lists member bytes
    out = np.zeros((len(classes), 4), dtype=np.uint64)
    for i, c in enumerate(classes):
        if isinstance(c, (int, np.integer)) and not isinstance(c, bool):
            c = int(c)
            if not 0 <= c < (1 << 256):
                raise ValueError("a 256-bit class mask is out of range")
            for w in range(4):
                out[i, w] = (c >> (64 * w)) & ((1 << 64) - 1)
        elif isinstance(c, np.ndarray) and c.dtype == np.uint64:
            if c.size != 4:
                raise ValueError("a word-encoded class is four uint64 words")
            out[i] = c.reshape(4)
        else:
            for b in c:
                b = int(b)
                if not 0 <= b <= 255:
                    raise ValueError("class members are bytes 0..255")
                out[i, b >> 6] |= np.uint64(1) << np.uint64(b & 63)
    return out


def _keep_for_stream(t, stream):
    """A temporary freed on return is reused by torch only after `stream` has passed this point."""
    if stream is not None:
        t.record_stream(stream)


def _stream_handle(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Program:
    """A compiled program (rx_compile) plus, once uploaded, its device tables."""

    def __init__(self, ast, root, classes=None, search=False):
        a = as_ast(ast)
        c = as_classes(classes)
        h = ctypes.c_void_p()
        _check(lib().rx_compile(a.ctypes.data, len(a), int(root), c.ctypes.data if len(c) else None, len(c),
                                RX_SEARCH if search else 0, ctypes.byref(h)))
        self._h = h
        self._dev_buf = None
        self.info = rx_info()
        _check(lib().rx_program_info(h, ctypes.byref(self.info)))

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.rx_program_free(h)
            self._h = None

    # -- introspection -------------------------------------------------
    def nodes(self) -> list:
        m = ctypes.c_int32()
        _check(lib().rx_program_nodes(self._h, None, 0, ctypes.byref(m)))
        arr = (rx_node * m.value)()
        _check(lib().rx_program_nodes(self._h, arr, m.value, ctypes.byref(m)))
        return [(n.kind, n.c0, n.c1, n.label, n.cont) for n in arr]

    def sets(self):
        """(first[W], follow[L, W], bytemask[256, W], leaf_node[L]) as numpy arrays."""
        W, L = self.info.words, self.info.n_leaves
        first = np.zeros(W, np.uint32)
        follow = np.zeros((max(L, 1), W), np.uint32)
        mask = np.zeros((256, W), np.uint32)
        leaf = np.zeros(max(L, 1), np.int32)
        _check(lib().rx_program_sets(self._h, first.ctypes.data, follow.ctypes.data, mask.ctypes.data, leaf.ctypes.data))
        return first, follow[:L], mask, leaf[:L]

    # -- bit-sliced circuit -------------------------------------------------
    def jit(self, arch=None):
        """Generate and compile the bit-sliced circuit kernel (hiprtc)."""
        _check(lib().rx_program_jit(self._h, arch.encode() if arch else None))
        return self

    def jit_planes_source(self) -> str:
        n = ctypes.c_size_t()
        _check(lib().rx_program_jit_planes_source(self._h, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value + 1)
        _check(lib().rx_program_jit_planes_source(self._h, buf, n.value + 1, ctypes.byref(n)))
        return buf.value.decode()

    def jit_source(self) -> str:
        n = ctypes.c_size_t()
        _check(lib().rx_program_jit_source(self._h, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value + 1)
        _check(lib().rx_program_jit_source(self._h, buf, n.value + 1, ctypes.byref(n)))
        return buf.value.decode()

    def jit_stats(self):
        r, s, o = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().rx_program_jit_stats(self._h, ctypes.byref(r), ctypes.byref(s), ctypes.byref(o)))
        return {"ready": r.value, "state_words": s.value, "ops": o.value}

    def node_image(self) -> bytes:
        """Device image of d[] for the node-per-thread machine (header, 16 bytes per node, classes)."""
        n = _SZ()
        _check(lib().rx_program_node_image(self._h, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().rx_program_node_image(self._h, buf, n.value, ctypes.byref(n)))
        return buf.raw[: n.value]

    def jit_staging(self):
        """[default mode, 1/0 for staging modes 1..5, earliest-accept form]: which sliced kernels run."""
        st = (ctypes.c_int32 * 7)()
        _check(lib().rx_program_jit_staging(self._h, st))
        return list(st)

    def jit_guard(self):
        """The static check of the register-staged kernels: {"ran", "violations" (per kernel), "dropped"}."""
        ran, dropped = ctypes.c_int32(), ctypes.c_int32()
        v = (ctypes.c_int32 * 8)()
        _check(lib().rx_program_jit_guard(self._h, ctypes.byref(ran), v, ctypes.byref(dropped)))
        return {"ran": ran.value, "violations": list(v)[:7], "dropped": dropped.value}

    def jit_selfcheck(self):
        """The run-time check of the bit-sliced kernels against the table step: {"ran", "dropped"}."""
        ran, dropped = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().rx_program_jit_selfcheck(self._h, ctypes.byref(ran), ctypes.byref(dropped)))
        return {"ran": ran.value, "dropped": dropped.value}

    # -- device -----------------------------------------------------------
    def upload(self, device=None, stream=None):
        import torch

        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        nbytes = int(self.info.table_bytes)
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        off = (-buf.data_ptr()) % 256
        view = buf[off:off + nbytes]
        with torch.cuda.device(dev):
            _check(lib().rx_program_upload(self._h, ctypes.c_void_p(view.data_ptr()), nbytes, _stream_handle(stream)))
        self._dev_buf = buf
        return self


def compile(ast, root, classes=None, search=False) -> Program:
    return Program(ast, root, classes, search)


def parse(pattern):
    """Regular-expression text (str or bytes; see rx_parse) -> (ast, root, classes) for compile()."""
    pat = pattern.encode("latin-1") if isinstance(pattern, str) else bytes(pattern)
    n_ast, root, n_cls = _I32(), _I32(), _I32()
    rc = lib().rx_parse(pat, len(pat), None, 0, ctypes.byref(n_ast), ctypes.byref(root), None, 0, ctypes.byref(n_cls))
    if rc not in (RX_OK, RX_ETOOBIG) or (rc == RX_ETOOBIG and n_ast.value == 0):
        _check(rc)
    ast = np.zeros(n_ast.value, dtype=AST_DTYPE)
    classes = np.zeros((n_cls.value, 4), dtype=np.uint64)
    _check(lib().rx_parse(pat, len(pat), ast.ctypes.data_as(ctypes.c_void_p), n_ast.value, ctypes.byref(n_ast),
                          ctypes.byref(root), classes.ctypes.data_as(ctypes.c_void_p), n_cls.value,
                          ctypes.byref(n_cls)))
    return ast, root.value, classes


def compile_regex(pattern, search=False) -> Program:
    """compile(parse(pattern)): whole-string matching, or any substring with search=True."""
    ast, root, classes = parse(pattern)
    return Program(ast, root, classes, search)


def match(prog: Program, data, offsets, out=None, launch=None, stream=None):
    """Match every string against ``prog``: returns a uint8 tensor of 0/1 on the device."""
    import torch

    if prog._dev_buf is None:
        prog.upload(device=data.device if data.numel() else offsets.device, stream=stream)
    if data.dtype != torch.uint8 or offsets.dtype != torch.int64:
        raise TypeError("data must be uint8 and offsets int64")
    if not (data.is_cuda and offsets.is_cuda):
        raise TypeError("data and offsets must be device tensors")
    data = data.contiguous()
    offsets = offsets.contiguous()
    n = offsets.numel() - 1
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.uint8, device=offsets.device)
    sh = _stream_handle(stream)
    dptr = ctypes.c_void_p(data.data_ptr() if data.numel() else offsets.data_ptr())
    if launch is None:
        _check(lib().rx_match(prog.handle, dptr, ctypes.c_void_p(offsets.data_ptr()), n,
                              ctypes.c_void_p(out.data_ptr()), sh))
    else:
        L = launch if isinstance(launch, rx_launch) else rx_launch(*launch)
        _check(lib().rx_match_ex(prog.handle, dptr, ctypes.c_void_p(offsets.data_ptr()), n,
                                 ctypes.c_void_p(out.data_ptr()), ctypes.byref(L), sh))
    return out


def match_first(prog: Program, data, offsets, out=None, stream=None):
    """Earliest accepting prefix length per string (int64 tensor, -1 where no prefix matches)."""
    import torch

    if prog._dev_buf is None:
        prog.upload(device=data.device if data.numel() else offsets.device, stream=stream)
    if data.dtype != torch.uint8 or offsets.dtype != torch.int64:
        raise TypeError("data must be uint8 and offsets int64")
    if not (data.is_cuda and offsets.is_cuda):
        raise TypeError("data and offsets must be device tensors")
    data = data.contiguous()
    offsets = offsets.contiguous()
    n = offsets.numel() - 1
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.int64, device=offsets.device)
    dptr = ctypes.c_void_p(data.data_ptr() if data.numel() else offsets.data_ptr())
    _check(lib().rx_match_first(prog.handle, dptr, ctypes.c_void_p(offsets.data_ptr()), n,
                                ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def match_long(prog: Program, data, length: int = None, chunks: int = 0, out=None, stream=None):
    """Chunk-parallel matching of one long string data[:length]: a 1-element uint8 tensor (0/1)."""
    import torch

    if data.dtype != torch.uint8:
        raise TypeError("data must be a uint8 tensor")
    if length is None:
        length = data.numel()
    # checked before anything runs: the kernels read bytes [0, length) of the tensor
    if not 0 <= int(length) <= data.numel():
        raise ValueError(f"length {length} outside the data tensor's {data.numel()} bytes")
    if not data.is_cuda:
        raise TypeError("data must be a device tensor")
    if prog._dev_buf is None:
        prog.upload(device=data.device, stream=stream)
    data = data.contiguous()
    need = _SZ()
    _check(lib().rx_match_long_workspace(prog.handle, int(length), int(chunks), ctypes.byref(need)))
    work = torch.empty(max(int(need.value), 4), dtype=torch.uint8, device=data.device)
    _keep_for_stream(work, stream)
    if out is None:
        out = torch.empty(1, dtype=torch.uint8, device=data.device)
    dptr = ctypes.c_void_p(data.data_ptr() if data.numel() else work.data_ptr())
    _check(lib().rx_match_long(prog.handle, dptr, int(length), int(chunks), ctypes.c_void_p(work.data_ptr()),
                               work.numel(), ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def match_first_long(prog: Program, data, length: int = None, chunks: int = 0, out=None, stream=None):
    """Earliest accepting prefix of one long string data[:length], in chunks: a 1-element int64 tensor (-1: none)."""
    import torch

    if data.dtype != torch.uint8:
        raise TypeError("data must be a uint8 tensor")
    if length is None:
        length = data.numel()
    # checked before anything runs: the kernels read bytes [0, length) of the tensor
    if not 0 <= int(length) <= data.numel():
        raise ValueError(f"length {length} outside the data tensor's {data.numel()} bytes")
    if not data.is_cuda:
        raise TypeError("data must be a device tensor")
    if prog._dev_buf is None:
        prog.upload(device=data.device, stream=stream)
    data = data.contiguous()
    need = _SZ()
    _check(lib().rx_match_long_workspace(prog.handle, int(length), int(chunks), ctypes.byref(need)))
    work = torch.empty(max(int(need.value), 8), dtype=torch.uint8, device=data.device)
    _keep_for_stream(work, stream)
    if out is None:
        out = torch.empty(1, dtype=torch.int64, device=data.device)
    dptr = ctypes.c_void_p(data.data_ptr() if data.numel() else work.data_ptr())
    _check(lib().rx_match_first_long(prog.handle, dptr, int(length), int(chunks), ctypes.c_void_p(work.data_ptr()),
                                     work.numel(), ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def match_nodes(prog: Program, data, offsets, out=None, stream=None):
    """The node-per-thread machine (one thread per node of d[], stamp vectors c and n): uint8 0/1 per string."""
    import torch

    if data.dtype != torch.uint8 or offsets.dtype != torch.int64:
        raise TypeError("data must be uint8 and offsets int64")
    if not (data.is_cuda and offsets.is_cuda):
        raise TypeError("data and offsets must be device tensors")
    img = getattr(prog, "_node_dev", None)
    if img is None or img.device != offsets.device:
        host = prog.node_image()
        img = torch.frombuffer(bytearray(host), dtype=torch.uint8).to(offsets.device)
        prog._node_dev = img
    data = data.contiguous()
    offsets = offsets.contiguous()
    n = offsets.numel() - 1
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.uint8, device=offsets.device)
    dptr = ctypes.c_void_p(data.data_ptr() if data.numel() else offsets.data_ptr())
    _check(lib().rx_match_nodes(prog.handle, ctypes.c_void_p(img.data_ptr()), dptr, ctypes.c_void_p(offsets.data_ptr()),
                                n, ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def match_first_fixed(prog: Program, data, length: int, n: int = None, out=None, stream=None):
    """match_first for fixed-length strings (string i = data[i*length:(i+1)*length])."""
    import torch

    if prog._dev_buf is None:
        prog.upload(device=data.device, stream=stream)
    if data.dtype != torch.uint8 or not data.is_cuda:
        raise TypeError("data must be a uint8 device tensor")
    data = data.contiguous()
    if n is None:
        n = data.numel() // length if length else 0
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.int64, device=data.device)
    _check(lib().rx_match_first_fixed(prog.handle, ctypes.c_void_p(data.data_ptr()), int(length), int(n),
                                      ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def match_fixed(prog: Program, data, length: int, n: int = None, out=None, launch=None, stream=None):
    """Match n fixed-length strings (string i = data[i*length:(i+1)*length])."""
    import torch

    if prog._dev_buf is None:
        prog.upload(device=data.device, stream=stream)
    if data.dtype != torch.uint8 or not data.is_cuda:
        raise TypeError("data must be a uint8 device tensor")
    data = data.contiguous()
    if n is None:
        n = data.numel() // length if length else 0
    if n * length > data.numel():
        raise ValueError("data holds fewer than n * length bytes")
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.uint8, device=data.device)
    sh = _stream_handle(stream)
    if launch is None:
        _check(lib().rx_match_fixed(prog.handle, ctypes.c_void_p(data.data_ptr()), int(length), int(n),
                                    ctypes.c_void_p(out.data_ptr()), sh))
    else:
        L = launch if isinstance(launch, rx_launch) else rx_launch(*launch)
        _check(lib().rx_match_fixed_ex(prog.handle, ctypes.c_void_p(data.data_ptr()), int(length), int(n),
                                       ctypes.c_void_p(out.data_ptr()), ctypes.byref(L), sh))
    return out


def prepare_multi(progs, arch=None) -> int:
    """Compile and load the plane-form module of this program list (rx_match_multi_prepare); returns the
    per-lane spill bytes the device compiler chose (0 when every state word fits in registers)."""
    handles = (ctypes.c_void_p * len(progs))(*[p.handle.value for p in progs])
    sp = ctypes.c_int32()
    _check(lib().rx_match_multi_prepare(handles, len(progs), arch.encode() if arch else None, ctypes.byref(sp)))
    return sp.value


def match_multi(progs, data, offsets, out=None, config=None, work=None, stream=None):
    """Every string against every program in one batched launch: returns a (P, n) uint8 tensor."""
    import torch

    n = offsets.numel() - 1
    P = len(progs)
    for p in progs:
        if p._dev_buf is None:
            p.upload(device=offsets.device, stream=stream)
    cfg = config if config is not None else rx_multi_config()
    if cfg.form == FORM_PLANES and cfg.max_bytes < data.numel():
        # the plane workspace is sized by a bound on the total string bytes: the buffer's size
        cfg = multi_config(list(cfg.edges)[:cfg.n_edges], cfg.block, cfg.grid, FORM_PLANES, data.numel(), cfg.graph)
    need = lib().rx_match_multi_workspace(n, P, ctypes.byref(cfg))
    if need < 0:
        _check(int(need))
    if work is None or work.numel() < need + 256:
        work = torch.empty(int(need) + 256, dtype=torch.uint8, device=offsets.device)
        _keep_for_stream(work, stream)
    wptr = work.data_ptr() + ((-work.data_ptr()) % 256)
    if out is None:
        out = torch.empty((P, max(n, 0)), dtype=torch.uint8, device=offsets.device)
    handles = (ctypes.c_void_p * P)(*[p.handle.value for p in progs])
    dptr = data.data_ptr() if data.numel() else offsets.data_ptr()
    _check(lib().rx_match_multi(handles, P, ctypes.c_void_p(dptr), ctypes.c_void_p(offsets.data_ptr()), n,
                                ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(wptr), int(need),
                                ctypes.byref(cfg), _stream_handle(stream)))
    return out


def multi_graph_counts():
    """(replays, in-place updates, instantiations) of rx_match_multi's graphs so far."""
    c = (ctypes.c_int64 * 3)()
    _check(lib().rx_multi_graph_counts(c))
    return tuple(int(x) for x in c)


def stream_copy(dst, src, nbytes=None, stream=None):
    """Measurement-only coalesced copy between two device tensors."""
    nbytes = int(nbytes if nbytes is not None else src.numel() * src.element_size())
    _check(lib().rx_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                                _stream_handle(stream)))


def version() -> str:
    return lib().rx_version().decode()
