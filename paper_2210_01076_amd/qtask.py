"""ctypes binding of libqtask.so (the C ABI in include/qtask.h).

Functions keep the C names and only marshal arguments; every step of the
simulation runs in the library's HIP kernels.  Loading fails loudly when the
library has not been built: there is no fallback.

``Simulator`` is a small convenience wrapper that builds a circuit from the
nested-list form of ``paper_2210_01076_amd.workloads`` and applies its edits.
"""
from __future__ import annotations

import ctypes
import json
import os
import tempfile
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libqtask.so")

# status codes
QTASK_OK, QTASK_E_ARG, QTASK_E_CONFLICT, QTASK_E_NOTFOUND = 0, 1, 2, 3
QTASK_E_NOMEM, QTASK_E_DEVICE, QTASK_E_STALE, QTASK_E_UNSUPPORTED, QTASK_E_BUSY = 4, 5, 6, 7, 8
QTASK_C128, QTASK_C64 = 0, 1
QTASK_FUSE_AUTO, QTASK_FUSE_NONE, QTASK_FUSE_DENSE = 0, 1, 2
QTASK_DEVICE_NONE = -1
QTASK_FRONT = 0

KIND = {name: i for i, name in enumerate(
    ["h", "x", "y", "z", "s", "sdg", "t", "tdg", "rx", "ry", "rz", "cx", "cz", "swap", "cp", "ccx"])}

u64 = ctypes.c_uint64
i32 = ctypes.c_int32


class qtask_opts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("device", i32), ("tile_bits", i32), ("low_bits", i32),
                ("block_bits", i32), ("fusion", i32), ("fuse_width", i32), ("ckpt_interval", i32),
                ("max_ckpts", i32), ("renorm", i32), ("autotune", i32), ("closed_mode", i32),
                ("stream", ctypes.c_void_p), ("alloc", ctypes.c_void_p), ("free", ctypes.c_void_p),
                ("alloc_ctx", ctypes.c_void_p), ("relabel", i32), ("ckpt_delta", i32)]


class qtask_stats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("mode", i32), ("levels_total", u64),
                ("levels_replayed", u64), ("segments_replayed", u64), ("first_level", u64), ("passes", u64),
                ("tiles", u64), ("stages", u64), ("dirty_blocks", u64), ("total_blocks", u64),
                ("gate_amp_updates", u64), ("bytes", ctypes.c_double), ("flops", ctypes.c_double),
                ("mfma_flops", ctypes.c_double),
                ("kernel_ms", ctypes.c_double), ("pass_kernel_ms", ctypes.c_double),
                ("plan_ms", ctypes.c_double), ("wall_ms", ctypes.c_double), ("ckpt_bytes", u64),
                ("ckpt_full_bytes", u64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "struct_size"}


class qtask_server_opts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("device", i32), ("budget_bytes", u64),
                ("max_inflight", i32), ("small_qubits", i32), ("use_graph", i32), ("order", i32)]


class qtask_edit(ctypes.Structure):
    _fields_ = [("op", i32), ("kind", i32), ("level", u64), ("gate_index", u64), ("qubits", i32 * 3),
                ("nq", i32), ("params", ctypes.c_double * 3), ("np", i32)]


class qtask_result(ctypes.Structure):
    _fields_ = [("ticket", u64), ("status", i32), ("session", i32), ("submit_ms", ctypes.c_double),
                ("start_ms", ctypes.c_double), ("done_ms", ctypes.c_double), ("latency_ms", ctypes.c_double),
                ("state_hash", u64), ("stats", qtask_stats)]


P = ctypes.POINTER
vp = ctypes.c_void_p
_SIGS = {
    "qtask_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "qtask_version": ([P(ctypes.c_int), P(ctypes.c_int)], ctypes.c_int),
    "qtask_last_error": ([vp], ctypes.c_char_p),
    "qtask_opts_default": ([P(qtask_opts)], ctypes.c_int),
    "qtask_device_count": ([P(ctypes.c_int)], ctypes.c_int),
    "qtask_create": ([ctypes.c_int, ctypes.c_int, P(qtask_opts), P(vp)], ctypes.c_int),
    "qtask_destroy": ([vp], ctypes.c_int),
    "qtask_insert_level": ([vp, u64, P(u64)], ctypes.c_int),
    "qtask_remove_level": ([vp, u64], ctypes.c_int),
    "qtask_insert_gate": ([vp, u64, ctypes.c_int, P(i32), ctypes.c_int, P(ctypes.c_double), ctypes.c_int,
                           P(u64)], ctypes.c_int),
    "qtask_remove_gate": ([vp, u64], ctypes.c_int),
    "qtask_num_levels": ([vp, P(u64)], ctypes.c_int),
    "qtask_level_at": ([vp, u64, P(u64)], ctypes.c_int),
    "qtask_num_gates": ([vp, P(u64)], ctypes.c_int),
    "qtask_update_state": ([vp], ctypes.c_int),
    "qtask_update_state_full": ([vp], ctypes.c_int),
    "qtask_last_update_stats": ([vp, P(qtask_stats)], ctypes.c_int),
    "qtask_read_amplitudes": ([vp, u64, u64, vp], ctypes.c_int),
    "qtask_norm": ([vp, P(ctypes.c_double)], ctypes.c_int),
    "qtask_inner": ([vp, vp, P(ctypes.c_double)], ctypes.c_int),
    "qtask_inner_noalloc": ([vp, vp, P(ctypes.c_double)], ctypes.c_int),
    "qtask_compare_states": ([vp, vp, P(u64)], ctypes.c_int),
    "qtask_state_hash": ([vp, P(u64)], ctypes.c_int),
    "qtask_state_device_ptr": ([vp, P(vp), P(u64)], ctypes.c_int),
    "qtask_device_bytes": ([vp, P(u64)], ctypes.c_int),
    "qtask_get_opts": ([vp, P(qtask_opts)], ctypes.c_int),
    "qtask_dump_plan": ([vp, ctypes.c_char_p], ctypes.c_int),
    "qtask_copy_bandwidth": ([ctypes.c_int, u64, ctypes.c_int, P(ctypes.c_double)], ctypes.c_int),
    "qtask_server_opts_default": ([P(qtask_server_opts)], ctypes.c_int),
    "qtask_server_create": ([P(qtask_server_opts), P(vp)], ctypes.c_int),
    "qtask_server_destroy": ([vp], ctypes.c_int),
    "qtask_server_open": ([vp, ctypes.c_int, ctypes.c_int, P(qtask_opts), u64, u64, P(i32), P(i32), P(i32),
                           P(ctypes.c_double), P(u64), P(i32)], ctypes.c_int),
    "qtask_server_submit": ([vp, i32, P(qtask_edit), ctypes.c_int, P(u64)], ctypes.c_int),
    "qtask_server_wait": ([vp, u64, ctypes.c_double, P(qtask_result)], ctypes.c_int),
    "qtask_server_poll": ([vp, u64, P(ctypes.c_int), P(qtask_result)], ctypes.c_int),
    "qtask_server_drain": ([vp], ctypes.c_int),
    "qtask_server_session": ([vp, i32, P(vp)], ctypes.c_int),
    "qtask_server_usage": ([vp, P(u64), P(i32)], ctypes.c_int),
    "qtask_server_peak_bytes": ([vp, P(u64)], ctypes.c_int),
    "qtask_server_paths": ([vp, P(u64), P(u64), P(u64)], ctypes.c_int),
}

_lib = None


class QtaskError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = _lib.qtask_status_string(code).decode() if _lib is not None else str(code)
        super().__init__("%s (status %d)%s" % (msg, code, (": " + what) if what else ""))


def load() -> ctypes.CDLL:
    """Load the built library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libqtask.so is not built (run __graft_entry__.build()): %s" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def check(rc: int, what: str = "") -> None:
    if rc != QTASK_OK:
        raise QtaskError(rc, what)


# ---------------------------------------------------------------- same names

def qtask_opts_default(**overrides) -> qtask_opts:
    o = qtask_opts()
    check(load().qtask_opts_default(ctypes.byref(o)))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def qtask_device_count() -> int:
    c = ctypes.c_int(0)
    load().qtask_device_count(ctypes.byref(c))
    return c.value


def qtask_create(n: int, dtype: int = QTASK_C128, opts: Optional[qtask_opts] = None) -> int:
    h = vp()
    check(load().qtask_create(n, dtype, ctypes.byref(opts) if opts is not None else None, ctypes.byref(h)),
          "qtask_create")
    return h.value


def qtask_destroy(h) -> None:
    check(load().qtask_destroy(h))


def qtask_insert_level(h, after: int = QTASK_FRONT) -> int:
    out = u64()
    check(load().qtask_insert_level(h, after, ctypes.byref(out)), "qtask_insert_level")
    return out.value


def qtask_remove_level(h, level: int) -> None:
    check(load().qtask_remove_level(h, level), "qtask_remove_level")


def qtask_insert_gate(h, level: int, kind, qubits: Sequence[int], params: Sequence[float] = ()) -> int:
    k = KIND[kind] if isinstance(kind, str) else int(kind)
    qs = (i32 * max(1, len(qubits)))(*qubits)
    ps = (ctypes.c_double * max(1, len(params)))(*params)
    out = u64()
    check(load().qtask_insert_gate(h, level, k, qs, len(qubits), ps, len(params), ctypes.byref(out)),
          "qtask_insert_gate")
    return out.value


def qtask_remove_gate(h, gate: int) -> None:
    check(load().qtask_remove_gate(h, gate), "qtask_remove_gate")


def qtask_num_levels(h) -> int:
    out = u64()
    check(load().qtask_num_levels(h, ctypes.byref(out)))
    return out.value


def qtask_level_at(h, index: int) -> int:
    out = u64()
    check(load().qtask_level_at(h, index, ctypes.byref(out)), "qtask_level_at")
    return out.value


def qtask_last_error(h) -> str:
    return load().qtask_last_error(h).decode()


def qtask_update_state(h) -> None:
    rc = load().qtask_update_state(h)
    check(rc, "qtask_update_state: " + qtask_last_error(h) if rc else "")


def qtask_update_state_full(h) -> None:
    rc = load().qtask_update_state_full(h)
    check(rc, "qtask_update_state_full: " + qtask_last_error(h) if rc else "")


def qtask_last_update_stats(h) -> dict:
    st = qtask_stats()
    check(load().qtask_last_update_stats(h, ctypes.byref(st)))
    return st.as_dict()


def qtask_read_amplitudes(h, first: int, count: int, dtype: int) -> np.ndarray:
    out = np.empty(count, dtype=np.complex128 if dtype == QTASK_C128 else np.complex64)
    check(load().qtask_read_amplitudes(h, first, count, out.ctypes.data if count else None),
          "qtask_read_amplitudes")
    return out


def qtask_norm(h) -> float:
    v = ctypes.c_double()
    check(load().qtask_norm(h, ctypes.byref(v)), "qtask_norm")
    return v.value


def qtask_inner(a, b) -> complex:
    v = (ctypes.c_double * 2)()
    check(load().qtask_inner(a, b, v), "qtask_inner")
    return complex(v[0], v[1])


def qtask_inner_noalloc(a, b) -> complex:
    v = (ctypes.c_double * 2)()
    check(load().qtask_inner_noalloc(a, b, v), "qtask_inner_noalloc")
    return complex(v[0], v[1])


def qtask_compare_states(a, b) -> int:
    v = u64()
    check(load().qtask_compare_states(a, b, ctypes.byref(v)), "qtask_compare_states")
    return v.value


def qtask_state_hash(h) -> int:
    v = u64()
    check(load().qtask_state_hash(h, ctypes.byref(v)), "qtask_state_hash")
    return v.value


def qtask_device_bytes(h) -> int:
    v = u64()
    check(load().qtask_device_bytes(h, ctypes.byref(v)))
    return v.value


def qtask_get_opts(h) -> qtask_opts:
    o = qtask_opts()
    check(load().qtask_get_opts(h, ctypes.byref(o)))
    return o


def qtask_dump_plan(h, path: str) -> None:
    check(load().qtask_dump_plan(h, path.encode()), "qtask_dump_plan")


def qtask_copy_bandwidth(device: int = 0, nbytes: int = 1 << 30, iters: int = 20) -> float:
    v = ctypes.c_double()
    check(load().qtask_copy_bandwidth(device, nbytes, iters, ctypes.byref(v)), "qtask_copy_bandwidth")
    return v.value


# ----------------------------------------------------------------- serving

def qtask_server_opts_default(**overrides) -> qtask_server_opts:
    o = qtask_server_opts()
    check(load().qtask_server_opts_default(ctypes.byref(o)))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def qtask_server_create(opts: Optional[qtask_server_opts] = None) -> int:
    s = vp()
    check(load().qtask_server_create(ctypes.byref(opts) if opts is not None else None, ctypes.byref(s)),
          "qtask_server_create")
    return s.value


def qtask_server_destroy(s) -> None:
    check(load().qtask_server_destroy(s), "qtask_server_destroy")


def qtask_server_open(s, n: int, dtype: int, opts: Optional[qtask_opts], nets) -> int:
    """Open a session whose circuit is ``nets`` (lists of (kind, qubits, params))."""
    kinds, qubits, nq, params, level_of = [], [], [], [], []
    for li, net in enumerate(nets):
        for kind, qs, ps in net:
            kinds.append(KIND[kind] if isinstance(kind, str) else int(kind))
            qubits.extend(list(qs) + [-1] * (3 - len(qs)))
            nq.append(len(qs))
            params.extend(list(ps) + [0.0] * (3 - len(ps)))
            level_of.append(li)
    g = len(kinds)
    out = i32()
    check(load().qtask_server_open(
        s, n, dtype, ctypes.byref(opts) if opts is not None else None, len(nets), g,
        (i32 * max(1, g))(*kinds), (i32 * max(3, 3 * g))(*qubits), (i32 * max(1, g))(*nq),
        (ctypes.c_double * max(3, 3 * g))(*params), (u64 * max(1, g))(*level_of), ctypes.byref(out)),
        "qtask_server_open")
    return out.value


def make_edits(e) -> List[qtask_edit]:
    """C edit records of a ``workloads.Edit`` (positions refer to the current circuit)."""
    out = []
    if e.op == "insert":
        li = e.net
        if e.new_net:
            out.append(qtask_edit(op=2, level=e.net))
            li = e.net + 1
        kind, qs, ps = e.gate
        c = qtask_edit(op=0, kind=KIND[kind] if isinstance(kind, str) else int(kind), level=li, nq=len(qs),
                       np=len(ps))
        for j, q in enumerate(qs):
            c.qubits[j] = q
        for j, v in enumerate(ps):
            c.params[j] = v
        out.append(c)
    elif e.op == "remove":
        out.append(qtask_edit(op=1, level=e.net, gate_index=e.pos))
    else:
        raise ValueError(e.op)
    return out


def qtask_server_submit(s, session: int, edits: Sequence[qtask_edit]) -> int:
    arr = (qtask_edit * max(1, len(edits)))(*edits)
    t = u64()
    check(load().qtask_server_submit(s, session, arr, len(edits), ctypes.byref(t)), "qtask_server_submit")
    return t.value


def _result(r: qtask_result) -> dict:
    return {"ticket": r.ticket, "status": r.status, "session": r.session, "submit_ms": r.submit_ms,
            "start_ms": r.start_ms, "done_ms": r.done_ms, "latency_ms": r.latency_ms,
            "state_hash": r.state_hash, "stats": r.stats.as_dict()}


def qtask_server_wait(s, ticket: int, timeout_ms: float = -1.0) -> dict:
    r = qtask_result()
    check(load().qtask_server_wait(s, ticket, timeout_ms, ctypes.byref(r)), "qtask_server_wait")
    return _result(r)


def qtask_server_poll(s, ticket: int) -> Optional[dict]:
    r = qtask_result()
    done = ctypes.c_int(0)
    check(load().qtask_server_poll(s, ticket, ctypes.byref(done), ctypes.byref(r)), "qtask_server_poll")
    return _result(r) if done.value else None


def qtask_server_drain(s) -> None:
    check(load().qtask_server_drain(s), "qtask_server_drain")


def qtask_server_session(s, session: int) -> int:
    h = vp()
    check(load().qtask_server_session(s, session, ctypes.byref(h)), "qtask_server_session")
    return h.value


def qtask_server_usage(s):
    b = u64()
    r = i32()
    check(load().qtask_server_usage(s, ctypes.byref(b), ctypes.byref(r)), "qtask_server_usage")
    return b.value, r.value


def qtask_server_peak_bytes(s) -> int:
    b = u64()
    check(load().qtask_server_peak_bytes(s, ctypes.byref(b)), "qtask_server_peak_bytes")
    return b.value


def qtask_server_paths(s) -> dict:
    """Requests started in batched ticks, requests launched on their
    session's own stream, and batched ticks, since the server was created."""
    a, b, t = u64(), u64(), u64()
    check(load().qtask_server_paths(s, ctypes.byref(a), ctypes.byref(b), ctypes.byref(t)), "qtask_server_paths")
    return {"batched": a.value, "streamed": b.value, "ticks": t.value}


# ------------------------------------------------------------- convenience

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class DeviceAllocator:
    """The ``alloc``/``free`` hooks of ``qtask_opts`` backed by Python
    callables: ``alloc(nbytes) -> int`` (a device pointer, 0 on failure)
    and ``free(ptr)``.  Keep the object alive as long as the session."""

    def __init__(self, alloc, free):
        self._alloc, self._free = alloc, free
        self.c_alloc = ALLOC_FN(lambda nbytes, ctx: self._alloc(int(nbytes)) or None)
        self.c_free = FREE_FN(lambda ptr, ctx: self._free(int(ptr)) if ptr else None)

    def install(self, o: qtask_opts) -> None:
        o.alloc = ctypes.cast(self.c_alloc, ctypes.c_void_p)
        o.free = ctypes.cast(self.c_free, ctypes.c_void_p)
        o.alloc_ctx = None


def _runtime_lib() -> ctypes.CDLL:
    """The HIP runtime libqtask.so is linked against (found through the
    process's mappings, so it is the same copy, not another one)."""
    load()
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64" in line:
                return ctypes.CDLL(line.split()[-1])
    raise RuntimeError("the HIP runtime of libqtask.so is not mapped")


def hip_allocator(on_alloc=None, on_free=None) -> DeviceAllocator:
    """Hooks that allocate with hipMalloc/hipFree of the library's own HIP
    runtime.  ``on_alloc(nbytes)`` may return False to refuse an allocation
    (the hook then returns NULL, as an exhausted allocator would);
    ``on_free(ptr)`` observes frees.  Memory from another runtime in the
    process (torch's wheel bundles its own HIP runtime) is not usable here:
    the library's runtime does not know its pointers."""
    rt = _runtime_lib()
    rt.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    rt.hipMalloc.restype = ctypes.c_int
    rt.hipFree.argtypes = [ctypes.c_void_p]
    rt.hipFree.restype = ctypes.c_int

    def alloc(nbytes):
        if on_alloc is not None and on_alloc(nbytes) is False:
            return 0
        p = ctypes.c_void_p()
        if rt.hipMalloc(ctypes.byref(p), nbytes) != 0:
            return 0
        return p.value or 0

    def free(ptr):
        if on_free is not None:
            on_free(ptr)
        rt.hipFree(ptr)

    return DeviceAllocator(alloc, free)


class Simulator:
    """A session built from nets of ``(kind, qubits, params)`` tuples.
    ``allocator`` is None (the library calls hipMalloc itself) or a
    ``DeviceAllocator`` whose hooks the library calls instead."""

    def __init__(self, n: int, dtype: str = "c128", allocator=None, **opts):
        self.n = n
        self.dtype = QTASK_C128 if dtype in ("c128", QTASK_C128) else QTASK_C64
        self.h = None
        o = qtask_opts_default(**opts)
        self.allocator = allocator
        if allocator is not None:
            allocator.install(o)
        self.h = qtask_create(n, self.dtype, o)
        self.levels: List[int] = []          # level ids in circuit order
        self.gates: List[List[int]] = []     # gate ids per level, insertion order

    def close(self):
        if self.h:
            qtask_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_level(self, index: Optional[int] = None) -> int:
        """Insert an empty level at position ``index`` (default: the end)."""
        if index is None:
            index = len(self.levels)
        after = QTASK_FRONT if index == 0 else self.levels[index - 1]
        lid = qtask_insert_level(self.h, after)
        self.levels.insert(index, lid)
        self.gates.insert(index, [])
        return lid

    def remove_level(self, index: int) -> None:
        """Remove the level at position ``index`` with its gates."""
        qtask_remove_level(self.h, self.levels[index])
        del self.levels[index]
        del self.gates[index]

    def add_gate(self, level_index: int, gate) -> int:
        kind, qs, ps = gate
        gid = qtask_insert_gate(self.h, self.levels[level_index], kind, qs, ps)
        self.gates[level_index].append(gid)
        return gid

    def build(self, nets) -> "Simulator":
        for net in nets:
            li = len(self.levels)
            self.add_level(li)
            for g in net:
                self.add_gate(li, g)
        return self

    def apply_edit(self, e) -> None:
        """Apply a ``workloads.Edit`` (positions refer to the current circuit)."""
        if e.op == "insert":
            li = e.net
            if e.new_net:
                li = e.net + 1
                self.add_level(li)
            self.add_gate(li, e.gate)
        elif e.op == "remove":
            gid = self.gates[e.net].pop(e.pos)
            qtask_remove_gate(self.h, gid)
        else:
            raise ValueError(e.op)

    def update(self, full: bool = False) -> dict:
        (qtask_update_state_full if full else qtask_update_state)(self.h)
        return qtask_last_update_stats(self.h)

    def stats(self) -> dict:
        return qtask_last_update_stats(self.h)

    def state(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        if count is None:
            count = (1 << self.n) - first
        return qtask_read_amplitudes(self.h, first, count, self.dtype)

    def norm(self) -> float:
        return qtask_norm(self.h)

    def hash(self) -> int:
        return qtask_state_hash(self.h)

    def dump(self) -> dict:
        fd, path = tempfile.mkstemp(suffix=".json")
        os.close(fd)
        try:
            qtask_dump_plan(self.h, path)
            with open(path) as f:
                return json.load(f)
        finally:
            os.unlink(path)
