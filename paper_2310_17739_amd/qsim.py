"""ctypes binding of the C ABI in ``include/qsim.h``.

This module only marshals arguments: every step of the simulation runs in
``libqsim.so`` (host compile in C++, sweeps and reductions in HIP kernels on
the GPU).  PyTorch provides the device memory and the stream.  If the
library has not been built, importing this module raises an error: there is
no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from workloads import GATE_DTYPE, PAULI_DTYPE

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("QSIM_LIB") or os.path.join(_HERE, "libqsim.so")

C64, C128 = 1, 2
OK, E_ARG, E_QUBIT, E_NOMEM, E_ZERO_PROB, E_NOT_DEFINITE, E_HIP, E_CAPACITY, E_UNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
F_ONE_OP_PER_PASS, F_NO_SPARSE, F_FULL_SUPPORT, F_REG_ENGINE = 1, 2, 4, 8


class QsimError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        msg = _lib.qsim_strerror(code).decode() if _lib is not None else str(code)
        if code in (E_HIP, E_NOMEM) and _lib is not None:
            last = _lib.qsim_last_error().decode()
            if last:
                msg += " [" + last + "]"
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")
        self.code = code


class qsim_fuse_opts(C.Structure):
    _fields_ = [("level", C.c_int32), ("max_width", C.c_int32), ("tile_qubits", C.c_int32),
                ("flags", C.c_int32), ("op_cost", C.c_float), ("low_qubits", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class qsim_apply_stats(C.Structure):
    _fields_ = [("input_gates", C.c_int64), ("ops_after", C.c_int64 * 6), ("fused_ops", C.c_int64),
                ("passes", C.c_int64), ("terms", C.c_int64), ("bytes_moved", C.c_int64),
                ("compile_seconds", C.c_double), ("tile_qubits", C.c_int32), ("max_width", C.c_int32),
                ("reg_passes", C.c_int64), ("reg_swaps", C.c_int64), ("reg_relayouts", C.c_int64)]

    def as_dict(self):
        return {"input_gates": self.input_gates, "ops_after": list(self.ops_after),
                "fused_ops": self.fused_ops, "passes": self.passes, "terms": self.terms,
                "bytes_moved": self.bytes_moved, "compile_seconds": self.compile_seconds,
                "tile_qubits": self.tile_qubits, "max_width": self.max_width,
                "reg_passes": self.reg_passes, "reg_swaps": self.reg_swaps,
                "reg_relayouts": self.reg_relayouts}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'`")
    # torch ships its own HIP runtime under the soname libamdhip64.so.7 but
    # asks for it as libamdhip64.so, so the loader cannot match the two:
    # loading this library first would map ROCm's runtime as well, and the
    # second runtime then finds no device.  Loading torch first makes this
    # library bind to torch's runtime, which also lets torch streams and
    # device pointers be passed straight through.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P, I, SZ, D = C.c_void_p, C.c_int, C.c_size_t, C.c_double
    sig = {
        "qsim_version": ([], I),
        "qsim_debug_fail_alloc": ([I], I),
        "qsim_strerror": ([I], C.c_char_p),
        "qsim_last_error": ([], C.c_char_p),
        "qsim_create": ([I, I, P, SZ, P, P], I),
        "qsim_destroy": ([P], I),
        "qsim_set_stream": ([P, P], I),
        "qsim_init_zero": ([P], I),
        "qsim_apply": ([P, P, SZ, P, SZ, P, SZ, P], I),
        "qsim_last_stats": ([P, P], I),
        "qsim_measure": ([P, I, D, P, P], I),
        "qsim_measure_assert": ([P, I, I, P], I),
        "qsim_reset": ([P, I], I),
        "qsim_expval": ([P, P, SZ, P], I),
        "qsim_probs": ([P, P, I, P], I),
        "qsim_norm": ([P, P], I),
        "qsim_probs_noalloc": ([P, P, I, P], I),
        "qsim_get_state": ([P, P], I),
        "qsim_set_state": ([P, P], I),
        "qsim_debug_fuse": ([I, P, SZ, P, SZ, P, SZ, P, P, P, P, SZ, SZ, P, P], I),
        "qsim_parse_qasm": ([C.c_char_p, SZ, P, SZ, P, P, P], I),
        "qsim_compile": ([I, I, P, SZ, P, SZ, P, SZ, P, P], I),
        "qsim_run": ([P, P], I),
        "qsim_program_graph": ([P, P, I], I),
        "qsim_run_timed": ([P, P], I),
        "qsim_program_kernel_ms": ([P, P, P], I),
        "qsim_program_stats": ([P, P], I),
        "qsim_program_destroy": ([P], I),
        "qsim_debug_plan": ([I, I, P, SZ, P, SZ, P, SZ, P, P], I),
        "qsim_debug_emulate": ([I, I, P, SZ, P, SZ, P, SZ, P, P], I),
        "qsim_autotune": ([P, P, SZ, P, SZ, P, SZ, SZ, P, P], I),
        "qsim_sample": ([P, P, SZ, P], I),
        "qsim_stream_copy": ([P, P, SZ, I, C.c_uint32, P], I),
        "qsim_batch_create": ([P, I, P, P], I),
        "qsim_batch_run": ([P, P], I),
        "qsim_batch_results": ([P, I, P, P, P, P, P], I),
        "qsim_batch_get_state": ([P, I, I, P], I),
        "qsim_batch_info_get": ([P, P], I),
        "qsim_batch_group_stats": ([P, I, P, P], I),
        "qsim_batch_destroy": ([P], I),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _bind_optional(lib)
    return lib


def _bind_optional(lib):
    """Entry points of the served form."""
    P, I, SZ, D = C.c_void_p, C.c_int, C.c_size_t, C.c_double
    opt = {
        "qsim_server_create": ([P, P], I),
        "qsim_server_submit": ([P, P, P], I),
        "qsim_server_poll": ([P, P, I, P, I], I),
        "qsim_server_get_stats": ([P, P], I),
        "qsim_server_clock": ([], D),
        "qsim_server_destroy": ([P], I),
    }
    for name, (args, res) in opt.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res


class qsim_batch_group(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_states", C.c_int32), ("g", C.c_void_p), ("ng", C.c_size_t),
                ("mats", C.c_void_p), ("n_mats", C.c_size_t), ("params", C.c_void_p), ("n_params", C.c_int32),
                ("uniforms", C.c_void_p), ("forced", C.c_void_p), ("n_slots", C.c_int32),
                ("terms", C.c_void_p), ("n_terms", C.c_size_t), ("dev_states", C.c_void_p)]


class qsim_batch_opts(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("use_graph", C.c_int32), ("max_params", C.c_int32),
                ("autotune", C.c_int32), ("fuse", qsim_fuse_opts)]


class qsim_batch_info(C.Structure):
    _fields_ = [("states", C.c_int64), ("input_gates", C.c_int64), ("fused_ops", C.c_int64),
                ("passes", C.c_int64), ("state_bytes", C.c_int64), ("coef_bytes", C.c_int64),
                ("compile_seconds", C.c_double), ("tune_seconds", C.c_double), ("records", C.c_int64)]


_lib = _load()


def lib():
    return _lib


def check(rc: int, what: str = ""):
    if rc != OK:
        raise QsimError(rc, what)


def _p(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _n(a):
    return 0 if a is None else int(a.size)


def _opts(level=None, max_width=None, tile_qubits=None, flags=0, op_cost=None, low_qubits=None):
    if isinstance(level, qsim_fuse_opts):
        return level
    if (level is None and max_width is None and tile_qubits is None and not flags and op_cost is None
            and low_qubits is None):
        return None
    o = qsim_fuse_opts()
    o.level = 5 if level is None else int(level)
    o.max_width = int(max_width or 0)
    o.tile_qubits = int(tile_qubits or 0)
    o.flags = int(flags)
    o.op_cost = float(op_cost or 0.0)
    o.low_qubits = int(low_qubits or 0)
    return o


def _torch():
    import torch
    return torch


class StateVector:
    """A 2^n complex state in device memory owned by a torch tensor."""

    def __init__(self, n: int, dtype: str = "complex128", device="cuda", stream=None, tensor=None):
        torch = _torch()
        self.n = int(n)
        self.dtype = QSIM_DTYPES[dtype]
        tdt = torch.complex64 if self.dtype == C64 else torch.complex128
        if tensor is None:
            tensor = torch.empty(1 << self.n, dtype=tdt, device=device)
        assert tensor.dtype == tdt and tensor.is_contiguous() and tensor.numel() >= (1 << self.n)
        self.tensor = tensor
        self.stream = stream if stream is not None else torch.cuda.current_stream(tensor.device)
        h = C.c_void_p()
        check(_lib.qsim_create(self.n, self.dtype, C.c_void_p(tensor.data_ptr()),
                               tensor.numel() * tensor.element_size(),
                               C.c_void_p(self.stream.cuda_stream), C.byref(h)), "qsim_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            _lib.qsim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------------- calls
    def qsim_init_zero(self):
        check(_lib.qsim_init_zero(self.h), "qsim_init_zero")

    def qsim_apply(self, gates, mats=None, params=None, level=None, max_width=None,
                   tile_qubits=None, flags=0, op_cost=None):
        g = np.ascontiguousarray(gates, dtype=GATE_DTYPE)
        m = None if mats is None else np.ascontiguousarray(mats, dtype=np.complex128)
        pr = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
        o = _opts(level, max_width, tile_qubits, flags, op_cost)
        check(_lib.qsim_apply(self.h, _p(g), len(g), _p(m), _n(m), _p(pr), _n(pr), C.byref(o) if o else None),
              "qsim_apply")

    def qsim_last_stats(self) -> dict:
        s = qsim_apply_stats()
        check(_lib.qsim_last_stats(self.h, C.byref(s)))
        return s.as_dict()

    def qsim_measure(self, q: int, u: float):
        o, p = C.c_int(), C.c_double()
        check(_lib.qsim_measure(self.h, int(q), float(u), C.byref(o), C.byref(p)), "qsim_measure")
        return o.value, p.value

    def qsim_measure_assert(self, q: int, want: int = 0) -> float:
        p = C.c_double()
        check(_lib.qsim_measure_assert(self.h, int(q), int(want), C.byref(p)), "qsim_measure_assert")
        return p.value

    def qsim_reset(self, q: int):
        check(_lib.qsim_reset(self.h, int(q)), "qsim_reset")

    def qsim_expval(self, terms) -> float:
        t = np.ascontiguousarray(terms, dtype=PAULI_DTYPE)
        out = C.c_double()
        check(_lib.qsim_expval(self.h, _p(t), len(t), C.byref(out)), "qsim_expval")
        return out.value

    def qsim_probs(self, qs) -> np.ndarray:
        q = np.ascontiguousarray(qs, dtype=np.int32)
        out = np.zeros(1 << len(q), dtype=np.float64)
        check(_lib.qsim_probs(self.h, _p(q), len(q), _p(out)), "qsim_probs")
        return out

    def qsim_probs_noalloc(self, qs, dev_out):
        """qsim_probs into a caller-owned float64 device tensor `dev_out`
        (2^len(qs) entries), asynchronously on the state's stream."""
        q = np.ascontiguousarray(qs, dtype=np.int32)
        assert dev_out.is_cuda and dev_out.numel() >= (1 << len(q)) and dev_out.element_size() == 8
        check(_lib.qsim_probs_noalloc(self.h, _p(q), len(q), C.c_void_p(dev_out.data_ptr())),
              "qsim_probs_noalloc")

    def qsim_norm(self) -> float:
        out = C.c_double()
        check(_lib.qsim_norm(self.h, C.byref(out)), "qsim_norm")
        return out.value

    def qsim_autotune(self, gates, mats=None, params=None, prefix_gates=0):
        """Returns (qsim_fuse_opts, ns per input gate) of the fastest candidate;
        pass the options back as `level=` to qsim_apply / Program."""
        g = np.ascontiguousarray(gates, dtype=GATE_DTYPE)
        m = None if mats is None else np.ascontiguousarray(mats, dtype=np.complex128)
        pr = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
        best = qsim_fuse_opts()
        ns = C.c_double()
        check(_lib.qsim_autotune(self.h, _p(g), len(g), _p(m), _n(m), _p(pr), _n(pr), int(prefix_gates), C.byref(best),
                                 C.byref(ns)), "qsim_autotune")
        return best, ns.value

    def qsim_sample(self, uniforms) -> np.ndarray:
        u = np.ascontiguousarray(uniforms, dtype=np.float64)
        out = np.zeros(len(u), dtype=np.uint64)
        check(_lib.qsim_sample(self.h, _p(u), len(u), _p(out)), "qsim_sample")
        return out

    def qsim_get_state(self) -> np.ndarray:
        out = np.empty(1 << self.n, dtype=np.complex64 if self.dtype == C64 else np.complex128)
        check(_lib.qsim_get_state(self.h, _p(out)), "qsim_get_state")
        return out

    def qsim_set_state(self, psi):
        src = np.ascontiguousarray(psi, dtype=np.complex64 if self.dtype == C64 else np.complex128)
        assert src.shape == (1 << self.n,)
        check(_lib.qsim_set_state(self.h, _p(src)), "qsim_set_state")


class Program:
    """A circuit compiled once (qsim_compile) and replayed with qsim_run."""

    def __init__(self, n, gates, dtype="complex128", mats=None, params=None, level=None,
                 max_width=None, tile_qubits=None, flags=0):
        g = np.ascontiguousarray(gates, dtype=GATE_DTYPE)
        m = None if mats is None else np.ascontiguousarray(mats, dtype=np.complex128)
        pr = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
        o = _opts(level, max_width, tile_qubits, flags)
        self.n = int(n)
        self.dtype = QSIM_DTYPES[dtype]
        p = C.c_void_p()
        check(_lib.qsim_compile(self.n, self.dtype, _p(g), len(g), _p(m), _n(m), _p(pr), _n(pr),
                                C.byref(o) if o else None, C.byref(p)), "qsim_compile")
        self.p = p

    def qsim_run(self, sv: "StateVector"):
        check(_lib.qsim_run(sv.h, self.p), "qsim_run")

    def qsim_run_timed(self, sv: "StateVector"):
        check(_lib.qsim_run_timed(sv.h, self.p), "qsim_run_timed")

    def qsim_program_kernel_ms(self):
        ms, n = C.c_double(), C.c_int64()
        check(_lib.qsim_program_kernel_ms(self.p, C.byref(ms), C.byref(n)), "qsim_program_kernel_ms")
        return ms.value, n.value

    def qsim_program_graph(self, sv: "StateVector", enable=True):
        check(_lib.qsim_program_graph(self.p, sv.h, int(bool(enable))), "qsim_program_graph")

    def qsim_program_stats(self) -> dict:
        s = qsim_apply_stats()
        check(_lib.qsim_program_stats(self.p, C.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "p", None):
            _lib.qsim_program_destroy(self.p)
            self.p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Batched programs (qsim_batch_*): each group is a dict with keys
    n, n_states, gates, and optionally mats, params (n_states x n_params),
    uniforms / forced (n_states x n_slots), n_slots, terms, states (a torch
    tensor of n_states * 2^n elements to run in place)."""

    def __init__(self, groups, dtype="complex64", use_graph=False, max_params=0,
                 level=None, max_width=None, tile_qubits=None, flags=0, autotune=False):
        self.dtype = QSIM_DTYPES[dtype]
        self._keep = []
        arr = (qsim_batch_group * len(groups))()
        self.groups = []
        for i, gd in enumerate(groups):
            g = np.ascontiguousarray(gd["gates"], dtype=GATE_DTYPE)
            n_states = int(gd["n_states"])
            mats = gd.get("mats")
            mats = None if mats is None else np.ascontiguousarray(mats, dtype=np.complex128)
            params = gd.get("params")
            params = None if params is None else np.ascontiguousarray(params, dtype=np.float64).reshape(n_states, -1)
            n_slots = int(gd.get("n_slots", 0))
            uni = gd.get("uniforms")
            uni = None if uni is None else np.ascontiguousarray(uni, dtype=np.float64).reshape(n_states, n_slots)
            forced = gd.get("forced")
            forced = None if forced is None else np.ascontiguousarray(forced, dtype=np.int32).reshape(n_states, n_slots)
            terms = gd.get("terms")
            terms = None if terms is None else np.ascontiguousarray(terms, dtype=PAULI_DTYPE)
            states = gd.get("states")
            self._keep += [g, mats, params, uni, forced, terms, states]
            a = arr[i]
            a.n = int(gd["n"])
            a.n_states = n_states
            a.g = g.ctypes.data
            a.ng = len(g)
            a.mats = None if mats is None else mats.ctypes.data
            a.n_mats = 0 if mats is None else mats.size
            a.params = None if params is None else params.ctypes.data
            a.n_params = 0 if params is None else params.shape[1]
            a.uniforms = None if uni is None else uni.ctypes.data
            a.forced = None if forced is None else forced.ctypes.data
            a.n_slots = n_slots
            a.terms = None if terms is None else terms.ctypes.data
            a.n_terms = 0 if terms is None else len(terms)
            a.dev_states = None if states is None else states.data_ptr()
            self.groups.append({"n": a.n, "n_states": n_states, "n_slots": n_slots})
        o = qsim_batch_opts()
        o.dtype = self.dtype
        o.use_graph = int(bool(use_graph))
        o.max_params = int(max_params)
        o.autotune = int(bool(autotune))
        fo = _opts(level, max_width, tile_qubits, flags)
        if fo is not None:
            o.fuse = fo
        h = C.c_void_p()
        check(_lib.qsim_batch_create(arr, len(groups), C.byref(o), C.byref(h)), "qsim_batch_create")
        self.h = h

    def qsim_batch_run(self, stream=None):
        if stream is None:
            stream = _torch().cuda.current_stream()
        check(_lib.qsim_batch_run(self.h, C.c_void_p(stream.cuda_stream)), "qsim_batch_run")

    def qsim_batch_results(self, group: int) -> dict:
        gd = self.groups[group]
        ns, nsl = gd["n_states"], gd["n_slots"]
        outc = np.zeros((ns, max(nsl, 1)), dtype=np.int32)
        probs = np.zeros((ns, max(nsl, 1)), dtype=np.float64)
        ev = np.zeros(ns, dtype=np.float64)
        nrm = np.zeros(ns, dtype=np.float64)
        status = np.zeros(ns, dtype=np.int32)
        check(_lib.qsim_batch_results(self.h, int(group), _p(outc), _p(probs), _p(ev), _p(nrm), _p(status)),
              "qsim_batch_results")
        return {"outcomes": outc[:, :nsl], "probs": probs[:, :nsl], "expvals": ev, "norms": nrm,
                "status": status}

    def qsim_batch_get_state(self, group: int, index: int) -> np.ndarray:
        n = self.groups[group]["n"]
        out = np.empty(1 << n, dtype=np.complex64 if self.dtype == C64 else np.complex128)
        check(_lib.qsim_batch_get_state(self.h, int(group), int(index), _p(out)), "qsim_batch_get_state")
        return out

    def qsim_batch_info(self) -> dict:
        i = qsim_batch_info()
        check(_lib.qsim_batch_info_get(self.h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in qsim_batch_info._fields_}

    def qsim_batch_group_stats(self, group: int) -> dict:
        s = qsim_apply_stats()
        w = C.c_int32()
        check(_lib.qsim_batch_group_stats(self.h, int(group), C.byref(s), C.byref(w)), "qsim_batch_group_stats")
        d = s.as_dict()
        d["tuned_width"] = w.value
        return d

    def close(self):
        if getattr(self, "h", None):
            _lib.qsim_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class qsim_server_opts(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("slots", C.c_int32), ("compile_threads", C.c_int32),
                ("pad", C.c_int32), ("pool_bytes", C.c_size_t), ("fuse", qsim_fuse_opts)]


class qsim_request(C.Structure):
    _fields_ = [("n", C.c_int32), ("pad", C.c_int32), ("g", C.c_void_p), ("ng", C.c_size_t),
                ("mats", C.c_void_p), ("n_mats", C.c_size_t), ("terms", C.c_void_p),
                ("n_terms", C.c_size_t), ("host_state_out", C.c_void_p)]


class qsim_result(C.Structure):
    _fields_ = [("id", C.c_int64), ("status", C.c_int32), ("n", C.c_int32), ("expval", C.c_double),
                ("norm", C.c_double), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("passes", C.c_int64)]


class qsim_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64),
                ("in_flight", C.c_int64), ("waiting", C.c_int64), ("pool_bytes", C.c_size_t),
                ("pool_in_use", C.c_size_t), ("pool_peak", C.c_size_t), ("peak_in_flight", C.c_int64)]


class Server:
    """The serving form (qsim_server_*): submit circuits, poll results."""

    def __init__(self, dtype="complex64", slots=8, compile_threads=4, pool_bytes=8 << 30,
                 level=None, max_width=None, tile_qubits=None, flags=0):
        o = qsim_server_opts()
        o.dtype = QSIM_DTYPES[dtype]
        o.slots = int(slots)
        o.compile_threads = int(compile_threads)
        o.pool_bytes = int(pool_bytes)
        fo = _opts(level, max_width, tile_qubits, flags)
        if fo is not None:
            o.fuse = fo
        self.dtype = o.dtype
        h = C.c_void_p()
        check(_lib.qsim_server_create(C.byref(o), C.byref(h)), "qsim_server_create")
        self.h = h
        self._keep = {}

    def qsim_server_submit(self, n, gates, terms=None, mats=None, want_state=False) -> int:
        g = np.ascontiguousarray(gates, dtype=GATE_DTYPE)
        t = None if terms is None else np.ascontiguousarray(terms, dtype=PAULI_DTYPE)
        m = None if mats is None else np.ascontiguousarray(mats, dtype=np.complex128)
        out = None
        if want_state:
            out = np.empty(1 << n, dtype=np.complex64 if self.dtype == C64 else np.complex128)
        r = qsim_request()
        r.n = int(n)
        r.g = g.ctypes.data
        r.ng = len(g)
        r.mats = None if m is None else m.ctypes.data
        r.n_mats = 0 if m is None else len(m)
        r.terms = None if t is None else t.ctypes.data
        r.n_terms = 0 if t is None else len(t)
        r.host_state_out = None if out is None else out.ctypes.data
        rid = C.c_int64()
        check(_lib.qsim_server_submit(self.h, C.byref(r), C.byref(rid)), "qsim_server_submit")
        if out is not None:
            self._keep[rid.value] = out
        return rid.value

    def qsim_server_poll(self, max_results=256, wait_ms=0):
        arr = (qsim_result * max_results)()
        k = C.c_int()
        check(_lib.qsim_server_poll(self.h, arr, max_results, C.byref(k), int(wait_ms)), "qsim_server_poll")
        res = []
        for i in range(k.value):
            a = arr[i]
            d = {f: getattr(a, f) for f, _ in qsim_result._fields_}
            if a.id in self._keep:
                d["state"] = self._keep.pop(a.id)
            res.append(d)
        return res

    def qsim_server_stats(self) -> dict:
        st = qsim_server_stats()
        check(_lib.qsim_server_get_stats(self.h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in qsim_server_stats._fields_}

    @staticmethod
    def qsim_server_clock() -> float:
        return _lib.qsim_server_clock()

    def close(self):
        if getattr(self, "h", None):
            _lib.qsim_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


QSIM_DTYPES = {"complex64": C64, "c64": C64, "complex128": C128, "c128": C128}


def qsim_debug_fuse(n, gates, mats=None, params=None, level=5, max_width=4, flags=0):
    """Host-only: the fused operators as a list of (qubits, matrix), and the
    operator count after each fusion level."""
    g = np.ascontiguousarray(gates, dtype=GATE_DTYPE)
    m = None if mats is None else np.ascontiguousarray(mats, dtype=np.complex128)
    pr = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
    o = _opts(level, max_width, None, flags)
    cap = max(len(g), 1)
    out_k = np.zeros(cap, dtype=np.int32)
    out_q = np.zeros(5 * cap, dtype=np.int32)
    cap_d = 2 * 1024 * cap
    out_m = np.zeros(min(cap_d, 2 * 1024 * 4096 + 2 * 16 * cap), dtype=np.float64)
    nops = C.c_size_t()
    counts = np.zeros(6, dtype=np.int64)
    rc = _lib.qsim_debug_fuse(int(n), _p(g), len(g), _p(m), _n(m), _p(pr), _n(pr), C.byref(o) if o else None,
                              _p(out_k), _p(out_q), _p(out_m), cap, len(out_m), C.byref(nops), _p(counts))
    if rc == E_CAPACITY:
        out_m = np.zeros(2 * 1024 * cap, dtype=np.float64)
        rc = _lib.qsim_debug_fuse(int(n), _p(g), len(g), _p(m), _n(m), _p(pr), _n(pr), C.byref(o) if o else None,
                                  _p(out_k), _p(out_q), _p(out_m), cap, len(out_m), C.byref(nops), _p(counts))
    check(rc, "qsim_debug_fuse")
    ops = []
    pos = 0
    for i in range(nops.value):
        k = int(out_k[i])
        d = 1 << k
        mat = (out_m[pos:pos + 2 * d * d:2] + 1j * out_m[pos + 1:pos + 2 * d * d:2]).reshape(d, d)
        pos += 2 * d * d
        ops.append((list(out_q[5 * i:5 * i + k]), mat))
    return ops, counts


def qsim_parse_qasm(text):
    """OpenQASM 2.0 text -> (gate records, n_qubits, n_clbits)."""
    b = text.encode() if isinstance(text, str) else bytes(text)
    n_out, nq, nc = C.c_size_t(), C.c_int32(), C.c_int32()
    # one record per statement unless broadcasts or gate definitions expand:
    # then the first call reports the size and a second one fills it
    out = np.zeros(max(b.count(b";"), 1), dtype=GATE_DTYPE)
    for _ in range(2):
        rc = _lib.qsim_parse_qasm(b, len(b), _p(out), len(out), C.byref(n_out), C.byref(nq), C.byref(nc))
        if rc == E_CAPACITY:
            out = np.zeros(n_out.value, dtype=GATE_DTYPE)
            continue
        if rc != OK:
            raise QsimError(rc, "qsim_parse_qasm: " + _lib.qsim_last_error().decode())
        return out[:n_out.value], nq.value, nc.value
    check(rc, "qsim_parse_qasm")


def qsim_debug_emulate(n, gates, dtype="complex128", mats=None, params=None, level=None,
                       max_width=None, tile_qubits=None, flags=0, psi=None) -> np.ndarray:
    """Host-only: the state after the circuit, applied in FP64 from the packed
    device tables of the plan compiled for n and dtype (|0...0> if psi is None)."""
    g = np.ascontiguousarray(gates, dtype=GATE_DTYPE)
    m = None if mats is None else np.ascontiguousarray(mats, dtype=np.complex128)
    pr = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
    o = _opts(level, max_width, tile_qubits, flags)
    if psi is None:
        out = np.zeros(1 << int(n), dtype=np.complex128)
        out[0] = 1.0
    else:
        out = np.array(psi, dtype=np.complex128, copy=True)
    check(_lib.qsim_debug_emulate(int(n), QSIM_DTYPES[dtype], _p(g), len(g), _p(m), _n(m), _p(pr), _n(pr),
                                  C.byref(o) if o else None, _p(out)), "qsim_debug_emulate")
    return out


def qsim_debug_plan(n, gates, dtype="complex128", mats=None, params=None, level=None,
                    max_width=None, tile_qubits=None, flags=0) -> dict:
    """Host-only: compile statistics (fused operators, passes) without a GPU."""
    g = np.ascontiguousarray(gates, dtype=GATE_DTYPE)
    m = None if mats is None else np.ascontiguousarray(mats, dtype=np.complex128)
    pr = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
    o = _opts(level, max_width, tile_qubits, flags)
    s = qsim_apply_stats()
    check(_lib.qsim_debug_plan(int(n), QSIM_DTYPES[dtype], _p(g), len(g), _p(m), _n(m), _p(pr), _n(pr),
                               C.byref(o) if o else None, C.byref(s)), "qsim_debug_plan")
    return s.as_dict()


def exported_symbols():
    """Names of every function declared in include/qsim.h."""
    import re
    hdr = os.path.join(os.path.dirname(_HERE), "include", "qsim.h")
    txt = open(hdr).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qsim_[a-z0-9_]+)\s*\(", txt)))


def qsim_stream_copy(dst, src, flags=0, rotate=0, stream=None):
    """Device copy src -> dst (torch tensors of the same byte size; dst may be
    src) with the tile kernel's grid shape; asynchronous on `stream` (default:
    torch's current stream)."""
    torch = _torch()
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes and src.is_cuda and dst.is_cuda
    st = stream if stream is not None else torch.cuda.current_stream(src.device)
    check(_lib.qsim_stream_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nbytes, int(flags),
                                int(rotate) & 0xffffffff, C.c_void_p(st.cuda_stream)), "qsim_stream_copy")


def qsim_debug_fail_alloc(after: int):
    """Make the library's allocation attempt `after` attempts from now fail
    once (QSIM_E_NOMEM); -1 disarms."""
    check(_lib.qsim_debug_fail_alloc(int(after)), "qsim_debug_fail_alloc")
