"""CPU oracle (complex double precision, one gate at a time, no fusion).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark load this package; the library under test never does.  The
arithmetic lives in ``oracle.c`` (plain C); this module builds it with gcc,
loads it with ctypes and wraps it for numpy arrays.

Functions and the passages they follow:

* :func:`run`      -- Eq. (1q-op) and Eq. (2q-op) of Section 3.2, gate by gate;
                      MEASURE / RESET / ASSERT0 records as in Section 4.3 and
                      Listing 1 (measure, reset, measurement assertion).
* :func:`measure`  -- Born rule, projection, renormalisation (Section 4.3).
* :func:`assert0`  -- measurement assertion: assert outcome 0 when
                      P(q = 0) > 0, fail otherwise (Section 4.3).
* :func:`reset`    -- reset of a definite qubit (Listing 1).
* :func:`expval`   -- <psi|H|psi>/<psi|psi> for a Pauli sum (the energies of
                      Table 7 are such expectation values).
* :func:`probs`, :func:`norm` -- marginal probabilities and the squared norm.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from workloads import GATE_DTYPE, PAULI_DTYPE

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# a prebuilt variant of the same source (the sanitizer build) may be named
# instead; it is then loaded as is
_LIB_OVERRIDE = os.environ.get("ORACLE_LIB")

E_OK, E_ARG, E_QUBIT, E_ZERO_PROB, E_NOT_DEFINITE = 0, -1, -2, -4, -5


class OracleError(RuntimeError):
    def __init__(self, code, where=None):
        super().__init__(f"oracle error {code}" + (f" at record {where}" if where is not None else ""))
        self.code = code
        self.where = where


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP on the sweeps)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def build_sanitized(out: str) -> str:
    """Compile oracle.c with clang's AddressSanitizer and UBSan (shared
    sanitizer runtime) into `out`, for host-side checks of the oracle."""
    clang = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    subprocess.check_call([clang, "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-shared-libsan", "-fno-omit-frame-pointer", "-o", out, _SRC, "-lm"])
    return out


def _load():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            lib = C.CDLL(_LIB_OVERRIDE)
        else:
            build()
            lib = C.CDLL(_LIB)
        P = C.c_void_p
        lib.orc_run.argtypes = [C.c_int, P, P, C.c_int64, P, P, P, P, P, P, P]
        lib.orc_run.restype = C.c_int
        lib.orc_measure.argtypes = [C.c_int, P, C.c_int, C.c_double, P, P]
        lib.orc_assert0.argtypes = [C.c_int, P, C.c_int, P]
        lib.orc_reset.argtypes = [C.c_int, P, C.c_int]
        lib.orc_norm.argtypes = [C.c_int, P]
        lib.orc_norm.restype = C.c_double
        lib.orc_probs.argtypes = [C.c_int, P, P, C.c_int, P]
        lib.orc_expval.argtypes = [C.c_int, P, P, C.c_int64]
        lib.orc_expval.restype = C.c_double
        lib.orc_gate_matrix.argtypes = [P, P, P]
        lib.orc_set_threads.argtypes = [C.c_int]
        lib.orc_set_threads.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def set_threads(k: int = 0) -> int:
    """OpenMP threads of the amplitude loops (0: leave as is); returns the
    number in effect.  For timing only: results do not depend on it."""
    return _load().orc_set_threads(int(k))


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def run(n, gates, psi=None, mats=None, params=None, uniforms=None,
        forced=None, n_slots=None, raise_on_error=True):
    """Apply ``gates`` to ``psi`` (|0...0> if None) one at a time.

    Returns (psi, outcomes, probs) where outcomes/probs are indexed by the
    MEASURE/ASSERT0 slot (length ``n_slots``, inferred from the records)."""
    lib = _load()
    g = np.ascontiguousarray(gates, dtype=GATE_DTYPE)
    psi = zero_state(n) if psi is None else np.ascontiguousarray(psi, dtype=np.complex128).copy()
    assert psi.shape == (1 << n,)
    if n_slots is None:
        meas = g[(g["kind"] == 61) | (g["kind"] == 63)]
        n_slots = int(meas["slot"].max()) + 1 if len(meas) else 0
    outcomes = np.full(max(n_slots, 1), -1, dtype=np.int32)
    probs = np.full(max(n_slots, 1), np.nan, dtype=np.float64)
    mats = None if mats is None else np.ascontiguousarray(mats, dtype=np.complex128)
    params = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
    uniforms = None if uniforms is None else np.ascontiguousarray(uniforms, dtype=np.float64)
    forced = None if forced is None else np.ascontiguousarray(forced, dtype=np.int32)
    fail = C.c_int64(-1)
    rc = lib.orc_run(n, _ptr(psi), _ptr(g), len(g), _ptr(mats), _ptr(params), _ptr(uniforms),
                     _ptr(forced), _ptr(outcomes), _ptr(probs), C.byref(fail))
    if rc and raise_on_error:
        raise OracleError(rc, fail.value)
    return psi, outcomes[:n_slots], probs[:n_slots]


def gate_matrix(gate_record, theta=None) -> np.ndarray:
    """The oracle's dense matrix of one record (in the record's qubit order)."""
    lib = _load()
    g = np.ascontiguousarray(np.array([gate_record], dtype=GATE_DTYPE))
    out = np.zeros(32 * 32, dtype=np.complex128)
    th = None if theta is None else np.ascontiguousarray(theta, dtype=np.float64)
    k = lib.orc_gate_matrix(_ptr(g), _ptr(th), _ptr(out))
    if k <= 0:
        raise OracleError(k)
    d = 1 << k
    return out[: d * d].reshape(d, d).copy()


def measure(n, psi, q, u):
    lib = _load()
    o, p = C.c_int(), C.c_double()
    rc = lib.orc_measure(n, _ptr(psi), q, float(u), C.byref(o), C.byref(p))
    if rc:
        raise OracleError(rc)
    return o.value, p.value


def assert0(n, psi, q):
    lib = _load()
    p = C.c_double()
    rc = lib.orc_assert0(n, _ptr(psi), q, C.byref(p))
    if rc:
        raise OracleError(rc)
    return p.value


def reset(n, psi, q):
    rc = _load().orc_reset(n, _ptr(psi), q)
    if rc:
        raise OracleError(rc)


def norm(n, psi) -> float:
    return _load().orc_norm(n, _ptr(np.ascontiguousarray(psi, dtype=np.complex128)))


def probs(n, psi, qs) -> np.ndarray:
    qs = np.ascontiguousarray(qs, dtype=np.int32)
    out = np.zeros(1 << len(qs), dtype=np.float64)
    _load().orc_probs(n, _ptr(np.ascontiguousarray(psi, dtype=np.complex128)), _ptr(qs), len(qs), _ptr(out))
    return out


def expval(n, psi, terms) -> float:
    t = np.ascontiguousarray(terms, dtype=PAULI_DTYPE)
    return _load().orc_expval(n, _ptr(np.ascontiguousarray(psi, dtype=np.complex128)), _ptr(t), len(t))


def sample(n, psi, uniforms) -> np.ndarray:
    """m shots of all qubits at once from psi (Section 4.3, sampling after
    measurement assertion): shot s is the smallest x with C(x) > u_s C(2^n-1),
    C the inclusive cumulative sum of |psi_x|^2 in index order."""
    w = np.abs(np.asarray(psi, dtype=np.complex128)) ** 2
    c = np.cumsum(w)
    return np.searchsorted(c, np.asarray(uniforms) * c[-1], side="right").astype(np.uint64)


def infidelity(a, b) -> float:
    """1 - |<a|b>|^2 / (<a|a><b|b>) in float64 (the reading of infidelity
    for states that need not have unit norm).  Rounding limits its
    resolution to about 1e-16 times the dimension's square root."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    ov = np.vdot(a, b)
    na = np.vdot(a, a).real
    nb = np.vdot(b, b).real
    return float(max(0.0, 1.0 - (abs(ov) ** 2) / (na * nb)))
