"""Exact simulation (ES) of AIG miters on AMD MI355X (gfx950).

A thin ctypes binding over the C ABI declared in include/fastlec_es.h
(``libfastlec_es.so``, built in-tree by ``paper_2512_06627_amd.build``).
Every step of the simulation runs in the library's HIP kernels; this module
only marshals arguments.  PyTorch, when given, supplies the stream
(``torch.cuda.current_stream()``) and optional caller-owned device scratch.

The library must be built: importing works without it, but every entry point
raises ``LibraryMissing`` when ``libfastlec_es.so`` is absent.  There is no
fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libfastlec_es.so")

FASTLEC_OK = 0
FASTLEC_ERR_PARSE = -1
FASTLEC_ERR_UNSUPPORTED = -2
FASTLEC_ERR_NOMEM = -3
FASTLEC_ERR_DEVICE = -4
FASTLEC_ERR_INVALID = -5
FASTLEC_CANCELLED = -6
FASTLEC_TIMEOUT = -7
FASTLEC_REJECTED = -8
FASTLEC_EQUIVALENT = 0
FASTLEC_NONEQUIVALENT = 1
FASTLEC_KERNEL_AUTO = 0
FASTLEC_KERNEL_INTERP = 1
FASTLEC_KERNEL_SPECIALIZED = 2
FASTLEC_KERNEL_INTERP_HBM = 3

KERNELS = {"auto": 0, "interp": 1, "specialized": 2, "interp_hbm": 3}


class LibraryMissing(RuntimeError):
    pass


class EsError(RuntimeError):
    def __init__(self, code, msg, result=None):
        super().__init__(f"fastlec_es error {code}: {msg}")
        self.code = code
        self.result = result


class fastlec_es_info(ctypes.Structure):
    _fields_ = [("num_pis", ctypes.c_uint32), ("num_ands", ctypes.c_uint32),
                ("num_ands_tfi", ctypes.c_uint32), ("num_outputs", ctypes.c_uint32),
                ("peak_live_slots", ctypes.c_uint32), ("num_instrs", ctypes.c_uint32),
                ("levels", ctypes.c_uint32), ("num_xors", ctypes.c_uint32), ("interp_rows", ctypes.c_uint32)]


class fastlec_es_options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("hip_stream", ctypes.c_void_p),
                ("words_per_thread", ctypes.c_uint32), ("tile_words", ctypes.c_uint32),
                ("wg_size", ctypes.c_uint32), ("kernel", ctypes.c_int),
                ("begin_word", ctypes.c_uint64), ("end_word", ctypes.c_uint64),
                ("deadline_s", ctypes.c_double), ("cancel_flag", ctypes.POINTER(ctypes.c_int)),
                ("dev_scratch", ctypes.c_void_p), ("dev_scratch_bytes", ctypes.c_size_t)]


class fastlec_es_result(ctypes.Structure):
    _fields_ = [("verdict", ctypes.c_int32), ("reserved", ctypes.c_uint32), ("cex", ctypes.c_uint64),
                ("patterns_evaluated", ctypes.c_uint64), ("next_word", ctypes.c_uint64),
                ("plan_ms", ctypes.c_double), ("compile_ms", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("queued_ms", ctypes.c_double), ("latency_ms", ctypes.c_double), ("predicted_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class fastlec_es_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("steps", ctypes.c_uint64), ("active", ctypes.c_uint64), ("queued", ctypes.c_uint64),
                ("charge_in_use_bytes", ctypes.c_uint64), ("budget_bytes", ctypes.c_uint64),
                ("peak_charge_bytes", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64),
                ("max_active", ctypes.c_uint64), ("busy_ms", ctypes.c_double),
                ("specialized_slices", ctypes.c_uint64)]


# (name, restype, argtypes) of every symbol in include/fastlec_es.h
_P = ctypes.c_void_p
SIGNATURES = [
    ("fastlec_es_options_init", None, [ctypes.POINTER(fastlec_es_options)]),
    ("fastlec_es_load_aig", ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(_P)]),
    ("fastlec_es_load_aig_file", ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(_P)]),
    ("fastlec_es_info_get", ctypes.c_int, [_P, ctypes.POINTER(fastlec_es_info)]),
    ("fastlec_es_check", ctypes.c_int, [_P, ctypes.POINTER(fastlec_es_options), ctypes.POINTER(fastlec_es_result)]),
    ("fastlec_es_check_batch", ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_size_t, ctypes.POINTER(fastlec_es_options),
                                              ctypes.POINTER(fastlec_es_result)]),
    ("fastlec_es_check_noalloc", ctypes.c_int, [_P, ctypes.POINTER(fastlec_es_options),
                                                ctypes.POINTER(fastlec_es_result)]),
    ("fastlec_es_free", None, [_P]),
    ("fastlec_es_last_error", ctypes.c_char_p, []),
    ("fastlec_es_server_create", ctypes.c_int, [ctypes.POINTER(fastlec_es_options), ctypes.c_size_t, ctypes.POINTER(_P)]),
    ("fastlec_es_server_submit", ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_uint64)]),
    ("fastlec_es_server_poll", ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(fastlec_es_result), ctypes.c_int]),
    ("fastlec_es_server_stats_get", ctypes.c_int, [_P, ctypes.POINTER(fastlec_es_server_stats)]),
    ("fastlec_es_server_destroy", None, [_P]),
    ("fastlec_es_compile_specialized", ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                                      ctypes.POINTER(ctypes.c_size_t)]),
    ("fastlec_es_compile_specialized_many", ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_size_t, ctypes.c_int,
                                                           ctypes.POINTER(ctypes.c_double)]),
    ("fastlec_es_specialized_source", ctypes.c_size_t, [_P, ctypes.c_int, ctypes.c_char_p, ctypes.c_size_t]),
    ("fastlec_es_host_replay", ctypes.c_int, [_P, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                              ctypes.POINTER(ctypes.c_uint32)]),
    ("fastlec_es_host_replay_specialized", ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_uint64,
                                                          ctypes.POINTER(ctypes.c_uint32)]),
    ("fastlec_es_simulate", ctypes.c_int, [_P, _P, ctypes.c_uint64, _P, ctypes.POINTER(fastlec_es_options),
                                           ctypes.POINTER(ctypes.c_double)]),
    ("fastlec_es_signature_hash", ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_uint64, _P, _P,
                                                 ctypes.POINTER(fastlec_es_options), ctypes.POINTER(ctypes.c_double)]),
    ("fastlec_es_classes", ctypes.c_int, [ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint64,
                                          ctypes.POINTER(ctypes.c_uint32)]),
    ("fastlec_es_memory_get", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_uint64),
                                             ctypes.POINTER(ctypes.c_uint64)]),
    ("fastlec_es_valu_probe", ctypes.c_int, [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    ("fastlec_es_predict", ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    ("fastlec_es_submiter_aag", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint8),
                                               ctypes.c_uint64, ctypes.c_uint32, ctypes.c_char_p, ctypes.c_size_t,
                                               ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_uint32),
                                               ctypes.POINTER(ctypes.c_uint32)]),
]

_lib = None


def lib():
    """The loaded C library; raises LibraryMissing when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(f"{LIB_PATH} not built: run paper_2512_06627_amd.build.build()")
        # PyTorch ships its own HIP and HSA runtimes; loaded after this library has initialised
        # the system ROCm runtime, it finds no GPU.  Loading it first lets both work in one process.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _raise(code, result=None):
    msg = lib().fastlec_es_last_error().decode(errors="replace")
    raise EsError(code, msg, result)


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream  # torch.cuda.Stream


def options(device=0, stream=None, words_per_thread=0, tile_words=0, wg_size=0, kernel="auto",
            begin_word=0, end_word=0, deadline_s=0.0, cancel_flag=None, scratch=None):
    o = fastlec_es_options()
    lib().fastlec_es_options_init(ctypes.byref(o))
    o.device = device
    o.hip_stream = _stream_handle(stream)
    o.words_per_thread = words_per_thread
    o.tile_words = tile_words
    o.wg_size = wg_size
    o.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    o.begin_word = begin_word
    o.end_word = end_word
    o.deadline_s = deadline_s
    if cancel_flag is not None:
        o.cancel_flag = ctypes.cast(ctypes.addressof(cancel_flag), ctypes.POINTER(ctypes.c_int))
    if scratch is not None:  # a torch tensor on the device
        o.dev_scratch = scratch.data_ptr()
        o.dev_scratch_bytes = scratch.numel() * scratch.element_size()
    return o


class Circuit:
    """A loaded, planned circuit (handle of fastlec_es_load_aig)."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        return self._h

    def info(self):
        i = fastlec_es_info()
        rc = lib().fastlec_es_info_get(self._h, ctypes.byref(i))
        if rc:
            _raise(rc)
        return {f: getattr(i, f) for f, _ in i._fields_ if f != "reserved"}

    def close(self):
        if self._h and self._h.value:
            lib().fastlec_es_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fastlec_es_load_aig(data: bytes) -> Circuit:
    h = ctypes.c_void_p()
    rc = lib().fastlec_es_load_aig(data, len(data), ctypes.byref(h))
    if rc:
        _raise(rc)
    return Circuit(h.value)


def fastlec_es_load_aig_file(path: str) -> Circuit:
    h = ctypes.c_void_p()
    rc = lib().fastlec_es_load_aig_file(path.encode(), ctypes.byref(h))
    if rc:
        _raise(rc)
    return Circuit(h.value)


def fastlec_es_check(circuit: Circuit, **opts) -> dict:
    """Exact simulation of one circuit; returns the result fields as a dict."""
    o = options(**opts)
    r = fastlec_es_result()
    rc = lib().fastlec_es_check(circuit.handle, ctypes.byref(o), ctypes.byref(r))
    if rc:
        _raise(rc, r.as_dict())
    return r.as_dict()


def fastlec_es_check_noalloc(circuit: Circuit, **opts) -> dict:
    """fastlec_es_check on the interpreter, with the library's static device array instead of
    device allocations; returns the result fields as a dict."""
    o = options(**opts)
    r = fastlec_es_result()
    rc = lib().fastlec_es_check_noalloc(circuit.handle, ctypes.byref(o), ctypes.byref(r))
    if rc:
        _raise(rc, r.as_dict())
    return r.as_dict()


def fastlec_es_check_batch(circuits, **opts) -> list:
    """Exact simulation of several circuits in one persistent launch."""
    k = len(circuits)
    arr = (ctypes.c_void_p * k)(*[c.handle.value for c in circuits])
    res = (fastlec_es_result * k)()
    o = options(**opts)
    rc = lib().fastlec_es_check_batch(arr, k, ctypes.byref(o), res)
    if rc:
        _raise(rc, [r.as_dict() for r in res])
    return [r.as_dict() for r in res]


def fastlec_es_compile_specialized(circuit: Circuit, waves_per_eu: int = 2):
    ms = ctypes.c_double()
    size = ctypes.c_size_t()
    rc = lib().fastlec_es_compile_specialized(circuit.handle, waves_per_eu, ctypes.byref(ms), ctypes.byref(size))
    if rc:
        _raise(rc)
    return {"compile_ms": ms.value, "code_bytes": size.value}


def fastlec_es_compile_specialized_many(circuits, waves_per_eu: int = 3) -> float:
    """Compile the specialized kernels of several circuits as few hipRTC programs; returns the
    compile time paid (ms)."""
    arr = (ctypes.c_void_p * len(circuits))(*[c.handle.value for c in circuits])
    ms = ctypes.c_double()
    rc = lib().fastlec_es_compile_specialized_many(arr, len(circuits), waves_per_eu, ctypes.byref(ms))
    if rc:
        _raise(rc)
    return ms.value


def fastlec_es_specialized_source(circuit: Circuit, waves_per_eu: int = 2) -> str:
    n = lib().fastlec_es_specialized_source(circuit.handle, waves_per_eu, None, 0)
    buf = ctypes.create_string_buffer(n)
    lib().fastlec_es_specialized_source(circuit.handle, waves_per_eu, buf, n)
    return buf.value.decode()


def fastlec_es_host_replay(circuit: Circuit, bundle: int, hw: int, count: int):
    out = (ctypes.c_uint32 * count)()
    rc = lib().fastlec_es_host_replay(circuit.handle, bundle, hw, count, out)
    if rc:
        _raise(rc)
    return list(out)


def fastlec_es_host_replay_specialized(circuit: Circuit, hw: int, count: int):
    out = (ctypes.c_uint32 * count)()
    rc = lib().fastlec_es_host_replay_specialized(circuit.handle, hw, count, out)
    if rc:
        _raise(rc)
    return list(out)


def _device_ptr(x):
    """Device address of a torch tensor (or an integer address)."""
    return x if isinstance(x, int) else x.data_ptr()


def fastlec_es_simulate(circuit: Circuit, pi_words, num_words: int, sig, **opts) -> float:
    """Value of every variable on num_words columns of input words (device buffers: pi_words
    n x num_words uint32, sig (max_var + 1) x num_words uint32); returns the kernel time in ms."""
    o = options(**opts)
    ms = ctypes.c_double()
    rc = lib().fastlec_es_simulate(circuit.handle, _device_ptr(pi_words) if pi_words is not None else None,
                                   num_words, _device_ptr(sig), ctypes.byref(o), ctypes.byref(ms))
    if rc:
        _raise(rc)
    return ms.value


def fastlec_es_signature_hash(sig, rows: int, num_words: int, hash, ones, **opts) -> float:
    """Complement-normalised hash and number of ones of every row (device buffers); returns
    the kernel time in ms."""
    o = options(**opts)
    ms = ctypes.c_double()
    rc = lib().fastlec_es_signature_hash(_device_ptr(sig), rows, num_words, _device_ptr(hash), _device_ptr(ones),
                                         ctypes.byref(o), ctypes.byref(ms))
    if rc:
        _raise(rc)
    return ms.value


def fastlec_es_classes(hashes):
    """numpy uint32 array: the lowest row with the same hash as each row (host arrays)."""
    import numpy as np
    h = np.ascontiguousarray(np.asarray(hashes, dtype=np.uint64))
    out = np.zeros(h.size, dtype=np.uint32)
    rc = lib().fastlec_es_classes(h.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), h.size,
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    if rc:
        _raise(rc)
    return out


def fastlec_es_predict(circuit: Circuit, begin_word: int = 0, end_word: int = 0) -> dict:
    """Predicted kernel times (ms) of a plain check: interpreter, specialized kernel, compile."""
    i, s, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    rc = lib().fastlec_es_predict(circuit.handle, begin_word, end_word, ctypes.byref(i), ctypes.byref(s),
                                  ctypes.byref(c))
    if rc:
        _raise(rc)
    return {"interp_ms": i.value, "specialized_ms": s.value, "compile_ms": c.value}


def fastlec_es_submiter_aag(circuit: Circuit, class_of, polarity, target: int):
    """(ASCII AIGER bytes of the sub-miter of pair (target, class_of[target]), original input
    index of each of its inputs).  class_of, polarity: host arrays of max_var + 1 entries."""
    import numpy as np
    cls = np.ascontiguousarray(np.asarray(class_of, dtype=np.uint32))
    pol = np.ascontiguousarray(np.asarray(polarity, dtype=np.uint8))
    if cls.size != pol.size:
        raise ValueError("class_of and polarity must have the same length")
    L = lib()
    cp = cls.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    pp = pol.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    need = ctypes.c_size_t()
    k = ctypes.c_uint32()
    rc = L.fastlec_es_submiter_aag(circuit.handle, cp, pp, cls.size, target, None, 0, ctypes.byref(need), None,
                                   ctypes.byref(k))
    if rc:
        _raise(rc)
    buf = ctypes.create_string_buffer(need.value)
    ins = (ctypes.c_uint32 * max(1, circuit.info()["num_pis"]))()
    rc = L.fastlec_es_submiter_aag(circuit.handle, cp, pp, cls.size, target, buf, need.value, None, ins, None)
    if rc:
        _raise(rc)
    return buf.value, list(ins[:k.value])


def fastlec_es_memory_get(device: int = 0) -> dict:
    """Device and pinned host bytes held by the library's buffer pool on a device."""
    d, p = ctypes.c_uint64(), ctypes.c_uint64()
    rc = lib().fastlec_es_memory_get(device, ctypes.byref(d), ctypes.byref(p))
    if rc:
        _raise(rc)
    return {"device_bytes": d.value, "pinned_bytes": p.value}


def fastlec_es_valu_probe(variant: int, waves_per_simd: int, iters: int, device: int = 0) -> dict:
    """Issue rate of independent VALU chains (wave64 instructions/s) and kernel time; variant 0:
    v_bitop3_b32 on three VGPRs, 1: on two VGPRs and an SGPR, 2: v_xor_b32."""
    r, ms = ctypes.c_double(), ctypes.c_double()
    rc = lib().fastlec_es_valu_probe(device, variant, waves_per_simd, iters, ctypes.byref(r), ctypes.byref(ms))
    if rc:
        _raise(rc)
    return {"instr_per_s": r.value, "kernel_ms": ms.value}


class Server:
    """Continuous-batching ES server (fastlec_es_server_*)."""

    def __init__(self, budget_bytes: int, **opts):
        self._o = options(**opts)
        h = ctypes.c_void_p()
        rc = lib().fastlec_es_server_create(ctypes.byref(self._o), budget_bytes, ctypes.byref(h))
        if rc:
            _raise(rc)
        self._h = h

    def submit(self, circuit: Circuit) -> int:
        t = ctypes.c_uint64()
        rc = lib().fastlec_es_server_submit(self._h, circuit.handle, ctypes.byref(t))
        if rc:
            _raise(rc)
        return t.value

    def poll(self, ticket: int, wait: bool = False):
        r = fastlec_es_result()
        rc = lib().fastlec_es_server_poll(self._h, ticket, ctypes.byref(r), 1 if wait else 0)
        if rc < 0:
            _raise(rc, r.as_dict())
        return r.as_dict() if rc == 1 else None

    def stats(self) -> dict:
        s = fastlec_es_server_stats()
        rc = lib().fastlec_es_server_stats_get(self._h, ctypes.byref(s))
        if rc:
            _raise(rc)
        return {f: getattr(s, f) for f, _ in s._fields_}

    def close(self):
        if self._h and self._h.value:
            lib().fastlec_es_server_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
