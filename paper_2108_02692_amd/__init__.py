"""paper_2108_02692_amd -- XOR-SLP erasure coding on MI355X (gfx950).

Thin ctypes binding over ``libec.so`` (C ABI in ``include/ec.h``).  Every
step of coding runs in the library's HIP kernels; this module only marshals
arguments.  PyTorch is used for device memory and streams: pass
``torch.Tensor`` buffers (uint8, on a ROCm device) or raw integer pointers.

The names mirror the C entry points (``ec_compile_slp``, ``ec_encode``,
``ec_decode``, ...); ``Program`` is a small owner of an ``ec_program*``.
"""
from __future__ import annotations

import ctypes
import os

from . import _build

__all__ = [
    "EcError", "Program", "ec_matrix_cauchy", "ec_matrix_vandermonde", "ec_compile_slp",
    "ec_encode", "ec_decode", "ec_status_str", "Batch", "ec_batch_build", "ec_batch_run_noalloc", "ec_device_copy",
    "ec_stripe_stream", "lib",
    "Server", "ec_server_create",
    "LEVEL_PLAIN", "LEVEL_CO", "LEVEL_CO_FU", "LEVEL_CO_FU_SCHED", "COMPRESS_XORREPAIR", "COMPRESS_REPAIR",
    "STAGE_PLAIN", "STAGE_CO", "STAGE_FU", "STAGE_SCHED", "STAGE_EXEC", "SPLIT_AUTO", "SPLIT_NEVER", "SPLIT_ALWAYS",
    "SPLIT_ROWS", "SPLIT_PAIRS", "SPLIT_PASSES", "SPLIT_STAGED", "SCHED_PUSH", "SCHED_GREEDY",
    "ec_program_upload_many", "ec_program_pool_stats", "NATIVE_WHOLE", "NATIVE_PAIRS", "NATIVE_BLOCKS",
]

LEVEL_PLAIN, LEVEL_CO, LEVEL_CO_FU, LEVEL_CO_FU_SCHED = 0, 1, 2, 3
COMPRESS_XORREPAIR, COMPRESS_REPAIR = 0, 1
SPLIT_AUTO, SPLIT_NEVER, SPLIT_ALWAYS, SPLIT_ROWS, SPLIT_PAIRS, SPLIT_PASSES, SPLIT_STAGED = 0, 1, 2, 3, 4, 5, 6
SCHED_PUSH, SCHED_GREEDY = 0, 1
NATIVE_WHOLE, NATIVE_PAIRS, NATIVE_BLOCKS = 1, 2, 4
STAGE_PLAIN, STAGE_CO, STAGE_FU, STAGE_SCHED, STAGE_EXEC = 0, 1, 2, 3, 4

STATUS = {
    0: "EC_OK", 1: "EC_ERR_ARG", 2: "EC_ERR_ALIGN", 3: "EC_ERR_TOO_MANY_ERASURES", 4: "EC_ERR_SINGULAR",
    5: "EC_ERR_NOMEM", 6: "EC_ERR_DEVICE", 7: "EC_ERR_UNSUPPORTED", 8: "EC_ERR_CAPACITY",
}


class EcError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__("%s: %s (%s)" % (what, self.name, ec_status_str(status)))


# L2 prefetch distance (strips) used when none is given (the library's own
# default for NULL options is the same).
DEFAULT_PREFETCH = 0


class CompileOpts(ctypes.Structure):
    _fields_ = [("level", ctypes.c_uint32), ("slot_budget", ctypes.c_uint32),
                ("compress", ctypes.c_uint32), ("block_strips", ctypes.c_uint32),
                ("prefetch", ctypes.c_uint32), ("split", ctypes.c_uint32), ("scheduler", ctypes.c_uint32),
                ("native", ctypes.c_uint32)]


class ProgramInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in (
        "n", "p", "n_in", "n_out", "n_stmt", "n_xor2", "n_mem", "nvar", "plain_xor2", "slots",
        "peak_open", "ring", "passes", "n_loads", "n_stores", "n_records", "n_ops", "n_words", "n_parts",
        "n_row_parts", "n_pair_parts", "n_pass_parts", "scheduler", "n_stage_parts", "native")] + [
        ("in_blocks", ctypes.POINTER(ctypes.c_int)), ("out_blocks", ctypes.POINTER(ctypes.c_int))]


class ServeRequest(ctypes.Structure):
    _fields_ = [("arrival_s", ctypes.c_double), ("prog", ctypes.c_void_p), ("in_", ctypes.c_void_p),
                ("block_bytes", ctypes.c_size_t)]


class ServeOpts(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("n_slots", ctypes.c_int), ("max_batch", ctypes.c_int)]


SERVE_DONE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_size_t))


class Stripe(ctypes.Structure):
    # in_ / out are `const uint8_t *const *` in C; held as plain addresses
    # (same layout) so that they can point into one array per batch
    _fields_ = [("prog", ctypes.c_void_p), ("in_", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("block_bytes", ctypes.c_size_t)]


_lib = None


def lib():
    """The loaded libec.so (built in-tree on first use if missing)."""
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = ctypes.CDLL(path)
        vp, u8p, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int)
        st = ctypes.c_int
        L.ec_matrix_cauchy.argtypes = [ctypes.c_int, ctypes.c_int, u8p]
        L.ec_matrix_vandermonde.argtypes = [ctypes.c_int, ctypes.c_int, u8p]
        L.ec_compile_slp.argtypes = [ctypes.c_int, ctypes.c_int, u8p, ip, ctypes.c_int,
                                     ctypes.POINTER(CompileOpts), ctypes.POINTER(vp)]
        L.ec_program_query.argtypes = [vp, ctypes.POINTER(ProgramInfo)]
        L.ec_encode.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_size_t, vp]
        L.ec_decode.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_size_t, vp]
        L.ec_program_free.argtypes = [vp]
        L.ec_program_free.restype = None
        L.ec_status_str.argtypes = [st]
        L.ec_status_str.restype = ctypes.c_char_p
        L.ec_program_export.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int32), ctypes.c_size_t,
                                        ctypes.POINTER(ctypes.c_size_t)]
        L.ec_program_export_greedy.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int32), ctypes.c_size_t,
                                               ctypes.POINTER(ctypes.c_size_t)]
        L.ec_program_bytecode.argtypes = [vp, ctypes.POINTER(ctypes.POINTER(ctypes.c_uint32)),
                                          ctypes.POINTER(ctypes.c_size_t)]
        L.ec_program_part_bytecode.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.POINTER(ctypes.c_uint32)),
                                               ctypes.POINTER(ctypes.c_size_t)]
        L.ec_device_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.ec_stripe_stream.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(vp), ctypes.c_int,
                                       ctypes.c_size_t, vp]
        L.ec_program_upload.argtypes = [vp]
        L.ec_program_upload_many.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
        L.ec_program_native_source.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_char_p),
                                               ctypes.POINTER(ctypes.c_size_t)]
        L.ec_program_pool_stats.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                            ctypes.POINTER(ctypes.c_size_t)]
        L.ec_batch_reserve.argtypes = [vp, ctypes.c_int, ctypes.c_size_t]
        L.ec_batch_build.argtypes = [ctypes.POINTER(Stripe), ctypes.c_int, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
        L.ec_batch_launch.argtypes = [vp, vp]
        L.ec_batch_enqueue.argtypes = [vp, vp]
        L.ec_batch_create.argtypes = [ctypes.POINTER(vp)]
        L.ec_batch_set.argtypes = [vp, ctypes.POINTER(Stripe), ctypes.c_int, ctypes.c_size_t, vp]
        L.ec_batch_query.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                     ctypes.POINTER(ctypes.c_size_t)]
        L.ec_batch_run_noalloc.argtypes = [ctypes.POINTER(Stripe), ctypes.c_int, ctypes.c_size_t, vp]
        L.ec_batch_free.argtypes = [vp]
        L.ec_batch_free.restype = None
        L.ec_server_create.argtypes = [vp, ctypes.c_size_t, ctypes.POINTER(ServeOpts), ctypes.POINTER(vp)]
        dp = ctypes.POINTER(ctypes.c_double)
        L.ec_server_run.argtypes = [vp, ctypes.POINTER(ServeRequest), ctypes.c_int, ctypes.c_int, SERVE_DONE_FN, vp,
                                    dp, ctypes.POINTER(ctypes.c_size_t), dp, ctypes.POINTER(ctypes.c_int)]
        L.ec_server_free.argtypes = [vp]
        L.ec_server_free.restype = None
        for name in ("ec_matrix_cauchy", "ec_matrix_vandermonde", "ec_compile_slp", "ec_program_query",
                     "ec_encode", "ec_decode", "ec_program_export", "ec_program_export_greedy", "ec_program_bytecode", "ec_program_part_bytecode", "ec_batch_build", "ec_device_copy",
                     "ec_stripe_stream", "ec_batch_launch", "ec_batch_enqueue", "ec_batch_query", "ec_batch_create", "ec_batch_set",
                     "ec_batch_run_noalloc", "ec_program_upload", "ec_program_upload_many", "ec_program_pool_stats", "ec_program_native_source",
                     "ec_server_create", "ec_server_run"):
            getattr(L, name).restype = st
        _lib = L
    return _lib


def ec_status_str(s: int) -> str:
    return lib().ec_status_str(int(s)).decode()


def _check(rc: int, what: str):
    if rc != 0:
        raise EcError(rc, what)


def _u8buf(n: int):
    return (ctypes.c_uint8 * n)()


def ec_matrix_cauchy(n: int, p: int):
    """(n+p) x n generator [I; P] with P[i][j] = 1/(i + (p + j)), as a list of rows."""
    buf = _u8buf((n + p) * n)
    _check(lib().ec_matrix_cauchy(n, p, buf), "ec_matrix_cauchy")
    return [list(buf[r * n:(r + 1) * n]) for r in range(n + p)]


def ec_matrix_vandermonde(n: int, p: int):
    buf = _u8buf((n + p) * n)
    _check(lib().ec_matrix_vandermonde(n, p, buf), "ec_matrix_vandermonde")
    return [list(buf[r * n:(r + 1) * n]) for r in range(n + p)]


def _flat_gen(gen, n, p):
    flat = [int(x) for row in gen for x in row]
    if len(flat) != (n + p) * n:
        raise ValueError("generator must be (n+p) x n")
    return (ctypes.c_uint8 * len(flat))(*flat)


def _ptr(x) -> int:
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    raise TypeError("expected a device tensor or an integer pointer")


def _ptr_array(xs):
    return (ctypes.c_void_p * max(1, len(xs)))(*[x if type(x) is int else _ptr(x) for x in xs])


def _stream_handle(stream) -> int | None:
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return int(torch.cuda.current_stream().cuda_stream) or None
        except Exception:  # pragma: no cover - torch without a device
            return None
        return None
    if isinstance(stream, int):
        return stream or None
    return int(stream.cuda_stream) or None


class Program:
    """Owner of a compiled ``ec_program``."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)
        info = ProgramInfo()
        _check(lib().ec_program_query(self._h, ctypes.byref(info)), "ec_program_query")
        self.info = {f: getattr(info, f) for f, _ in ProgramInfo._fields_ if not f.endswith("blocks")}
        self.in_blocks = [info.in_blocks[i] for i in range(info.n_in)]
        self.out_blocks = [info.out_blocks[i] for i in range(info.n_out)]

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h is not None and self._h.value:
            lib().ec_program_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def export(self, stage: int):
        """Program of one pipeline stage: (stmts, outputs) with terms as in
        ec_program_export (>= 0 variable, -1 zero, <= -2 input strip -t-2)."""
        return self._exported(lambda buf, cap, n: lib().ec_program_export(self._h, stage, buf, cap, n),
                              "ec_program_export")

    def export_greedy(self, capacity: int):
        """The fused stage scheduled by the greedy heuristic for an LRU cache
        of `capacity` entries: (stmts, outputs) whose variables are pebbles."""
        return self._exported(lambda buf, cap, n: lib().ec_program_export_greedy(self._h, capacity, buf, cap, n),
                              "ec_program_export_greedy")

    @staticmethod
    def _exported(call, what):
        n = ctypes.c_size_t()
        _check(call(None, 0, ctypes.byref(n)), what)
        buf = (ctypes.c_int32 * n.value)()
        _check(call(buf, n.value, ctypes.byref(n)), what)
        v = list(buf)
        ns, no = v[0], v[1]
        i = 2
        stmts = []
        for _ in range(ns):
            var, ar = v[i], v[i + 1]
            stmts.append((var, v[i + 2:i + 2 + ar]))
            i += 2 + ar
        return stmts, v[i:i + no]

    def upload(self):
        """Copy the records to the current device now (else the first launch
        does it, synchronously)."""
        _check(lib().ec_program_upload(self._h), "ec_program_upload")

    def native_source(self, kernel: int = 1) -> str:
        """Source of the program's native kernel ``kernel`` (NATIVE_WHOLE,
        NATIVE_PAIRS or NATIVE_BLOCKS; EcError if it has none)."""
        src, n = ctypes.c_char_p(), ctypes.c_size_t()
        _check(lib().ec_program_native_source(self._h, kernel, ctypes.byref(src), ctypes.byref(n)),
               "ec_program_native_source")
        return src.value[:n.value].decode()

    def bytecode(self):
        w = ctypes.POINTER(ctypes.c_uint32)()
        n = ctypes.c_size_t()
        _check(lib().ec_program_bytecode(self._h, ctypes.byref(w), ctypes.byref(n)), "ec_program_bytecode")
        return [w[i] for i in range(n.value)]

    def part_bytecode(self, part: int):
        """Words of row-split part ``part``: block parts first
        (``part < info["n_parts"]``), then row parts, then pair parts, then
        pass parts, then stage parts (up to ``n_parts + n_row_parts +
        n_pair_parts + n_pass_parts + n_stage_parts``)."""
        w = ctypes.POINTER(ctypes.c_uint32)()
        n = ctypes.c_size_t()
        _check(lib().ec_program_part_bytecode(self._h, part, ctypes.byref(w), ctypes.byref(n)),
               "ec_program_part_bytecode")
        return [w[i] for i in range(n.value)]


def ec_compile_slp(n: int, p: int, gen, erased=(), level: int = LEVEL_CO_FU_SCHED, slot_budget: int = 0,
                   compress: int = COMPRESS_XORREPAIR, block_strips: int = 0,
                   prefetch: int | None = None, split: int = SPLIT_AUTO, scheduler: int = SCHED_PUSH,
                   native: int = 0) -> Program:
    er = list(erased)
    er_arr = (ctypes.c_int * max(1, len(er)))(*er)
    opts = CompileOpts(level, slot_budget, compress, block_strips,
                       DEFAULT_PREFETCH if prefetch is None else prefetch, split, scheduler, int(native))
    h = ctypes.c_void_p()
    _check(lib().ec_compile_slp(n, p, _flat_gen(gen, n, p), er_arr, len(er), ctypes.byref(opts), ctypes.byref(h)),
           "ec_compile_slp")
    return Program(h.value)


def ec_encode(prog: Program, data, parity, block_bytes: int, stream=None):
    """Enqueue an encode on ``stream`` (default: torch's current stream)."""
    _check(lib().ec_encode(prog.handle, _ptr_array(data), _ptr_array(parity), block_bytes,
                           _stream_handle(stream)), "ec_encode")


def ec_decode(prog: Program, survivors, recovered, block_bytes: int, stream=None):
    """Enqueue a decode; ``survivors`` in ``prog.in_blocks`` order, ``recovered``
    in ``prog.out_blocks`` order."""
    _check(lib().ec_decode(prog.handle, _ptr_array(survivors), _ptr_array(recovered), block_bytes,
                           _stream_handle(stream)), "ec_decode")


def ec_program_upload_many(progs):
    """Copy many programs' records to the current device, setting aside the
    space they need in one piece first (at most one device allocation)."""
    progs = list(progs)
    arr = (ctypes.c_void_p * max(1, len(progs)))(*[p.handle for p in progs])
    _check(lib().ec_program_upload_many(arr, len(progs)), "ec_program_upload_many")


def ec_program_pool_stats():
    """(chunks, distinct records, bytes in use) of the current device's
    program pool."""
    c, i, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
    _check(lib().ec_program_pool_stats(ctypes.byref(c), ctypes.byref(i), ctypes.byref(b)), "ec_program_pool_stats")
    return c.value, i.value, b.value


def ec_device_copy(dst, src, nbytes: int, stream=None):
    """Plain device copy kernel (bandwidth ceiling / counter calibration)."""
    _check(lib().ec_device_copy(_ptr(dst), _ptr(src), nbytes, _stream_handle(stream)), "ec_device_copy")


def ec_stripe_stream(inputs, outputs, block_bytes: int, stream=None):
    """A coding launch's data movement without a program (every output
    strip-tile = XOR of the tile's input strip-tiles): the ceiling for a
    launch of that shape."""
    _check(lib().ec_stripe_stream(_ptr_array(inputs), len(inputs), _ptr_array(outputs), len(outputs), block_bytes,
                                  _stream_handle(stream)), "ec_stripe_stream")


class Batch:
    """Owner of an ``ec_batch`` (many stripes, one persistent launch)."""

    def __init__(self, handle: int, keepalive=None):
        self._h = ctypes.c_void_p(handle)
        self._keep = keepalive
        self._query()

    def _query(self):
        n_items, nin, nout = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().ec_batch_query(self._h, ctypes.byref(n_items), ctypes.byref(nin), ctypes.byref(nout)),
               "ec_batch_query")
        self.n_items, self.in_bytes, self.out_bytes = n_items.value, nin.value, nout.value

    @classmethod
    def create(cls):
        """An empty reusable batch (see ``set``)."""
        h = ctypes.c_void_p()
        _check(lib().ec_batch_create(ctypes.byref(h)), "ec_batch_create")
        return cls(h.value)

    def set(self, stripes, tile_bytes: int = 0, stream=None):
        """Refill with ``stripes`` ((Program, inputs, outputs, block_bytes));
        asynchronous on ``stream``; the previous launch must have finished."""
        arr, keep, n = _stripe_array(stripes)
        _check(lib().ec_batch_set(self._h, arr, n, tile_bytes, _stream_handle(stream)),
               "ec_batch_set")
        self._keep = keep
        self._query()

    def reserve(self, n_stripes: int, n_items: int):
        """Size the tables so that ``set`` up to these sizes allocates nothing."""
        _check(lib().ec_batch_reserve(self._h, n_stripes, n_items), "ec_batch_reserve")

    def launch(self, stream=None):
        """One launch of the batch's HIP graph (reset + persistent kernel)."""
        _check(lib().ec_batch_launch(self._h, _stream_handle(stream)), "ec_batch_launch")

    def enqueue(self, stream=None):
        """The same kernels enqueued directly (for callers capturing graphs)."""
        _check(lib().ec_batch_enqueue(self._h, _stream_handle(stream)), "ec_batch_enqueue")

    def free(self):
        if self._h is not None and self._h.value:
            lib().ec_batch_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _stripe_array(stripes):
    """(ctypes array of Stripe, objects to keep alive, number of stripes):
    every stripe's block pointers in one flat array."""
    stripes = list(stripes)
    arr = (Stripe * max(1, len(stripes)))()
    flat = [p if type(p) is int else _ptr(p) for _, ins, outs, _ in stripes for p in (*ins, *outs)]
    ptrs = (ctypes.c_void_p * max(1, len(flat)))(*flat)
    base, step = ctypes.addressof(ptrs), ctypes.sizeof(ctypes.c_void_p)
    keep = [ptrs]
    k = 0
    for i, (prog, ins, outs, bb) in enumerate(stripes):
        keep.append(prog)
        s = arr[i]
        s.prog = prog.handle.value
        s.in_ = base + step * k
        k += len(ins)
        s.out = base + step * k
        k += len(outs)
        s.block_bytes = bb
    return arr, keep, len(stripes)


def ec_batch_build(stripes, tile_bytes: int = 0, stream=None) -> Batch:
    """``stripes``: iterable of (Program, inputs, outputs, block_bytes).
    Uploads the tables (waiting on ``stream``) and captures a HIP graph."""
    arr, keep, n = _stripe_array(stripes)
    h = ctypes.c_void_p()
    _check(lib().ec_batch_build(arr, n, tile_bytes, _stream_handle(stream), ctypes.byref(h)),
           "ec_batch_build")
    return Batch(h.value, keep)


def ec_batch_run_noalloc(stripes, tile_bytes: int = 0, stream=None):
    """One batched launch over ``stripes`` ((Program, inputs, outputs,
    block_bytes)) whose tables live in the library's fixed per-device array:
    no allocation (every program must be uploaded to the device first).
    Launches overlapping on one device race on that array."""
    arr, keep, n = _stripe_array(stripes)
    _check(lib().ec_batch_run_noalloc(arr, n, tile_bytes, _stream_handle(stream)), "ec_batch_run_noalloc")


class Server:
    """Owner of an ``ec_server``: the native serving loop (``ec_server_run``)
    over a device arena that must outlive it."""

    def __init__(self, handle: int, arena):
        self._h = ctypes.c_void_p(handle)
        self._arena = arena

    @property
    def handle(self):
        return self._h

    def run(self, requests, realtime: bool = True, on_done=None):
        """``requests``: list of (arrival_s, Program, input pointers,
        block_bytes), arrivals nondecreasing.  ``on_done(ids, out_offsets)``
        sees each completed launch (request indices, output offsets in the
        arena) before its space is reused.  Returns (completion times in s,
        output offsets in the arena, wall time in s, launches)."""
        n = len(requests)
        arr = (ServeRequest * max(1, n))()
        flat = [p if type(p) is int else _ptr(p) for _, _, ins, _ in requests for p in ins]
        ptrs = (ctypes.c_void_p * max(1, len(flat)))(*flat)
        base, step, k = ctypes.addressof(ptrs), ctypes.sizeof(ctypes.c_void_p), 0
        for i, (t, prog, ins, bb) in enumerate(requests):
            r = arr[i]
            r.arrival_s = t
            r.prog = prog.handle.value
            r.in_ = base + step * k
            r.block_bytes = bb
            k += len(ins)
        done = (ctypes.c_double * max(1, n))()
        offs = (ctypes.c_size_t * max(1, n))()
        wall, nb = ctypes.c_double(), ctypes.c_int()
        cb = SERVE_DONE_FN(0)
        if on_done is not None:
            def _cb(_user, ids, n_ids, offs):
                on_done([ids[j] for j in range(n_ids)], [offs[j] for j in range(n_ids)])
            cb = SERVE_DONE_FN(_cb)
        _check(lib().ec_server_run(self._h, arr, n, 1 if realtime else 0, cb, None, done, offs, ctypes.byref(wall),
                                   ctypes.byref(nb)), "ec_server_run")
        return list(done)[:n], list(offs)[:n], wall.value, nb.value

    def free(self):
        if self._h is not None and self._h.value:
            lib().ec_server_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def ec_server_create(arena, arena_bytes: int, budget_bytes: int, n_slots: int = 4, max_batch: int = 2048) -> Server:
    """A native serving loop over the device arena ``arena`` (a tensor or a
    pointer; ``arena_bytes`` long): ``n_slots`` streams, launches of up to
    ``max_batch`` requests, admission within ``budget_bytes``."""
    opts = ServeOpts(budget_bytes, n_slots, max_batch)
    h = ctypes.c_void_p()
    _check(lib().ec_server_create(_ptr(arena), arena_bytes, ctypes.byref(opts), ctypes.byref(h)), "ec_server_create")
    return Server(h.value, arena)
