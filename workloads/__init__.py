"""Seeded synthetic inputs for the state-vector simulator and its oracle.

This module is the only code shared by the HIP path and the CPU oracle.  It
draws random numbers and builds gate *records* (kind, qubits, angles); it holds
none of the simulation arithmetic (no gate matrices, no state updates, no
probabilities).  Every generator is deterministic in its seed.

Gate-record layout (56 bytes, little-endian, natural C alignment)::

    uint16 kind      one of the KIND_* codes below
    uint16 nq        number of qubits the record names (1..5)
    int32  q[5]      qubits; for controlled gates the controls come first and
                     the target last
    int32  slot      -1: angles come from theta[]; >= 0 for a rotation in a
                     parameterised template: theta[0] is read from the
                     circuit's parameter vector at this index.  For MEASURE and
                     ASSERT0 records it is the measurement slot (index of the
                     uniform draw and of the recorded outcome)
    uint32 mat_off   MAT records: offset, in complex entries, of a row-major
                     2^nq x 2^nq complex128 matrix in the caller's matrix pool
    float64 theta[3] angles (radians)

The workloads follow the circuit families of the paper's evaluation
(Section 5.1, Table 5: deep Trotterised circuits of Pauli-string exponentials
with one ancilla measured and reset per filtering step, Listing 1), at the
widths the paper uses (7, 13 and 21 qubits) and beyond.  The paper's own QASM
files and nuclear interactions are not available, so these synthetic circuits
stand in for them.
"""
from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------- gate codes
# Gate names follow the OpenQASM 2.0 table of the paper (Section 4.1, Table 3).
KIND_ID, KIND_H, KIND_X, KIND_Y, KIND_Z = 0, 1, 2, 3, 4
KIND_S, KIND_SDG, KIND_T, KIND_TDG, KIND_SX = 5, 6, 7, 8, 9
KIND_RX, KIND_RY, KIND_RZ, KIND_U1, KIND_U2, KIND_U3 = 10, 11, 12, 13, 14, 15
KIND_CX, KIND_CY, KIND_CZ, KIND_CH, KIND_SWAP = 20, 21, 22, 23, 24
KIND_CRX, KIND_CRY, KIND_CRZ, KIND_CU1, KIND_CU3 = 25, 26, 27, 28, 29
KIND_RXX, KIND_RZZ = 30, 31
KIND_CCX, KIND_CSWAP, KIND_C3X, KIND_C3XSQRTX, KIND_C4X = 40, 41, 44, 45, 46
KIND_RCCX, KIND_RC3X = 42, 43
KIND_MAT = 50
KIND_BARRIER, KIND_MEASURE, KIND_RESET, KIND_ASSERT0 = 60, 61, 62, 63

KIND_NAMES = {
    KIND_ID: "id", KIND_H: "h", KIND_X: "x", KIND_Y: "y", KIND_Z: "z",
    KIND_S: "s", KIND_SDG: "sdg", KIND_T: "t", KIND_TDG: "tdg", KIND_SX: "sx",
    KIND_RX: "rx", KIND_RY: "ry", KIND_RZ: "rz", KIND_U1: "u1", KIND_U2: "u2",
    KIND_U3: "u3", KIND_CX: "cx", KIND_CY: "cy", KIND_CZ: "cz", KIND_CH: "ch",
    KIND_SWAP: "swap", KIND_CRX: "crx", KIND_CRY: "cry", KIND_CRZ: "crz",
    KIND_CU1: "cu1", KIND_CU3: "cu3", KIND_RXX: "rxx", KIND_RZZ: "rzz",
    KIND_CCX: "ccx", KIND_CSWAP: "cswap", KIND_C3X: "c3x",
    KIND_C3XSQRTX: "c3sqrtx", KIND_C4X: "c4x", KIND_RCCX: "rccx", KIND_RC3X: "rc3x", KIND_MAT: "mat",
    KIND_BARRIER: "barrier", KIND_MEASURE: "measure", KIND_RESET: "reset",
    KIND_ASSERT0: "assert0",
}
KIND_QUBITS = {
    KIND_ID: 1, KIND_H: 1, KIND_X: 1, KIND_Y: 1, KIND_Z: 1, KIND_S: 1,
    KIND_SDG: 1, KIND_T: 1, KIND_TDG: 1, KIND_SX: 1, KIND_RX: 1, KIND_RY: 1,
    KIND_RZ: 1, KIND_U1: 1, KIND_U2: 1, KIND_U3: 1, KIND_CX: 2, KIND_CY: 2,
    KIND_CZ: 2, KIND_CH: 2, KIND_SWAP: 2, KIND_CRX: 2, KIND_CRY: 2,
    KIND_CRZ: 2, KIND_CU1: 2, KIND_CU3: 2, KIND_RXX: 2, KIND_RZZ: 2,
    KIND_CCX: 3, KIND_CSWAP: 3, KIND_C3X: 4, KIND_C3XSQRTX: 4, KIND_C4X: 5,
    KIND_RCCX: 3, KIND_RC3X: 4, KIND_MEASURE: 1, KIND_RESET: 1, KIND_ASSERT0: 1,
}
KIND_NPARAMS = {KIND_RX: 1, KIND_RY: 1, KIND_RZ: 1, KIND_U1: 1, KIND_U2: 2,
                KIND_U3: 3, KIND_CRX: 1, KIND_CRY: 1, KIND_CRZ: 1,
                KIND_CU1: 1, KIND_CU3: 3, KIND_RXX: 1, KIND_RZZ: 1}

GATE_DTYPE = np.dtype([
    ("kind", "<u2"), ("nq", "<u2"), ("q", "<i4", (5,)), ("slot", "<i4"),
    ("mat_off", "<u4"), ("theta", "<f8", (3,)),
], align=True)
assert GATE_DTYPE.itemsize == 56

# Pauli-sum term layout (24 bytes): coefficient, x-mask, z-mask.
# Letter on qubit j: I (x=0,z=0), X (x=1,z=0), Z (x=0,z=1), Y (x=1,z=1).
PAULI_DTYPE = np.dtype([("coeff", "<f8"), ("xmask", "<u8"), ("zmask", "<u8")],
                       align=True)
assert PAULI_DTYPE.itemsize == 24


def gates(records) -> np.ndarray:
    """Build a gate array from tuples ``(kind, qubits, thetas[, slot])``."""
    n = len(records)
    out = np.zeros(n, dtype=GATE_DTYPE)
    if n == 0:
        return out
    kinds = np.empty(n, dtype=np.uint16)
    nq = np.empty(n, dtype=np.uint16)
    q = np.zeros((n, 5), dtype=np.int32)
    th = np.zeros((n, 3), dtype=np.float64)
    slot = np.full(n, -1, dtype=np.int32)
    for i, rec in enumerate(records):
        kinds[i] = rec[0]
        qs = rec[1]
        if np.iterable(qs):
            k = len(qs)
            q[i, :k] = qs
        else:
            k = 1
            q[i, 0] = qs
        nq[i] = k
        if len(rec) > 2:
            t = rec[2]
            if np.iterable(t):
                if len(t):
                    th[i, :len(t)] = t
            else:
                th[i, 0] = t
        if len(rec) > 3:
            slot[i] = rec[3]
    out["kind"] = kinds
    out["nq"] = nq
    out["q"] = q
    out["theta"] = th
    out["slot"] = slot
    return out


def _rng(*key) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(list(key)))


# ------------------------------------------------------------------ config 1
def random_circuit(n: int = 6, n_gates: int = 200, seed: int = 1) -> np.ndarray:
    """Random circuit over {H, X, Ry, Rz, CNOT}: kind uniform, 1q qubit uniform,
    CNOT ordered pair uniform over the n(n-1) ordered pairs, angle U[0, 2pi)."""
    rng = _rng(seed)
    kinds = [KIND_H, KIND_X, KIND_RY, KIND_RZ, KIND_CX]
    out = np.zeros(n_gates, dtype=GATE_DTYPE)
    out["slot"] = -1
    for i in range(n_gates):
        k = kinds[rng.integers(len(kinds))]
        out[i]["kind"] = k
        if k == KIND_CX:
            a, b = rng.choice(n, size=2, replace=False)
            out[i]["nq"] = 2
            out[i]["q"][:2] = (a, b)
        else:
            out[i]["nq"] = 1
            out[i]["q"][0] = rng.integers(n)
            if k in (KIND_RY, KIND_RZ):
                out[i]["theta"][0] = rng.uniform(0.0, 2.0 * math.pi)
    return out


def random_all_kinds(n: int, n_gates: int, seed: int,
                     max_arity: int = 5) -> np.ndarray:
    """Random circuit drawing every fixed gate kind of the table (and dense
    MAT records are left to callers): used for coverage tests."""
    rng = _rng(seed, 77)
    kinds = [k for k, a in KIND_QUBITS.items()
             if a <= min(n, max_arity) and k not in (KIND_MEASURE, KIND_RESET,
                                                     KIND_ASSERT0)]
    out = np.zeros(n_gates, dtype=GATE_DTYPE)
    out["slot"] = -1
    for i in range(n_gates):
        k = kinds[rng.integers(len(kinds))]
        a = KIND_QUBITS[k]
        out[i]["kind"] = k
        out[i]["nq"] = a
        out[i]["q"][:a] = rng.choice(n, size=a, replace=False)
        out[i]["theta"][:] = rng.uniform(-math.pi, 2 * math.pi, size=3)
    return out


def diagonal_rich_circuit(n: int, n_gates: int, seed: int, p_diag: float = 0.8) -> np.ndarray:
    """Random circuit in which a fraction ``p_diag`` of the gates is diagonal
    (Z, S, T, Rz, U1, CZ, CU1, CRZ, RZZ) and the rest mixes (H, Rx, Ry, CX,
    CRY); p_diag = 1 gives a circuit diagonal on every qubit.  Qubits uniform
    without replacement, angles U[0, 2pi)."""
    rng = _rng(seed, 91)
    diag = [KIND_Z, KIND_S, KIND_T, KIND_RZ, KIND_U1, KIND_CZ, KIND_CU1, KIND_CRZ, KIND_RZZ]
    mix = [KIND_H, KIND_RX, KIND_RY, KIND_CX, KIND_CRY]
    out = np.zeros(n_gates, dtype=GATE_DTYPE)
    out["slot"] = -1
    for i in range(n_gates):
        pool = diag if rng.random() < p_diag else mix
        k = pool[rng.integers(len(pool))]
        a = KIND_QUBITS[k]
        out[i]["kind"] = k
        out[i]["nq"] = a
        out[i]["q"][:a] = rng.choice(n, size=a, replace=False)
        out[i]["theta"][0] = rng.uniform(0.0, 2.0 * math.pi)
    return out


# ------------------------------------------------------------------ config 2
def pauli_strings(n: int, count: int, rng: np.random.Generator,
                  wmin: int = 2, wmax: int = 4):
    """``count`` random Pauli strings: weight U{wmin..wmax}, qubits drawn
    without replacement (the first w of a random permutation), letters
    U{X, Y, Z}.  Returns a list of (sorted qubit array, letter array) with
    letters 1=X, 2=Y, 3=Z."""
    wmax = min(wmax, n)
    ws = rng.integers(wmin, wmax + 1, size=count)
    perm = np.argsort(rng.random((count, n)), axis=1)[:, :wmax]
    lets = rng.integers(1, 4, size=(count, wmax))
    out = []
    for i in range(count):
        w = int(ws[i])
        out.append((np.sort(perm[i, :w]), lets[i, :w].copy()))
    return out


def compile_pauli_exponential(qs, letters, theta, slot=-1, into=None):
    """Gate records for exp(-i theta P / 2): basis change (X: H, Y: Rx(pi/2)),
    CNOT ladder in ascending qubit order, Rz(theta) on the last qubit, then the
    ladder and the basis change undone (X: H, Y: Rx(-pi/2)).

    With ``slot >= 0`` the Rz angle is a template parameter read at run time
    from the circuit's parameter vector (theta is then ignored by the device).
    """
    recs = [] if into is None else into
    for q, l in zip(qs, letters):
        if l == 1:
            recs.append((KIND_H, (q,), ()))
        elif l == 2:
            recs.append((KIND_RX, (q,), (math.pi / 2,)))
    for a, b in zip(qs[:-1], qs[1:]):
        recs.append((KIND_CX, (a, b), ()))
    recs.append((KIND_RZ, (qs[-1],), (theta,), slot))
    for a, b in reversed(list(zip(qs[:-1], qs[1:]))):
        recs.append((KIND_CX, (a, b), ()))
    for q, l in zip(qs, letters):
        if l == 1:
            recs.append((KIND_H, (q,), ()))
        elif l == 2:
            recs.append((KIND_RX, (q,), (-math.pi / 2,)))
    return recs


def pauli_exponential_circuit(n: int = 21, n_exp: int = 50_000, seed: int = 2,
                              sigma: float = 0.1, parameterised: bool = False):
    """UCC-style circuit: ``n_exp`` Pauli exponentials exp(-i theta P/2),
    theta ~ N(0, sigma^2) (sigma read as the standard deviation).

    Returns (gates, thetas, strings).  With ``parameterised`` the Rz records
    carry slot = exponential index so a batch can bind its own angles."""
    rng = _rng(seed)
    strings = pauli_strings(n, n_exp, rng)
    thetas = rng.normal(0.0, sigma, size=n_exp)
    recs = []
    for e, (qs, letters) in enumerate(strings):
        compile_pauli_exponential(qs, letters, float(thetas[e]),
                                  e if parameterised else -1, recs)
    return gates(recs), thetas, strings


def pauli_sum(n: int = 21, n_terms: int = 100, seed: int = 3) -> np.ndarray:
    """Random Pauli sum: weight U{2,3,4} on distinct qubits, letters
    U{X,Y,Z}, coefficient N(0,1)."""
    rng = _rng(seed)
    out = np.zeros(n_terms, dtype=PAULI_DTYPE)
    for i, (qs, letters) in enumerate(pauli_strings(n, n_terms, rng,
                                                    2, min(4, n))):
        xm = zm = 0
        for q, l in zip(qs, letters):
            if l in (1, 2):
                xm |= 1 << int(q)
            if l in (2, 3):
                zm |= 1 << int(q)
        out[i] = (rng.normal(), xm, zm)
    return out


def z_terms(n: int) -> np.ndarray:
    """The n single-qubit terms Z_i with unit coefficient."""
    out = np.zeros(n, dtype=PAULI_DTYPE)
    for i in range(n):
        out[i] = (1.0, 0, 1 << i)
    return out


# ------------------------------------------------------------------ config 3
def trajectory_round_program(n_sys: int = 12, rounds: int = 500, seed: int = 4):
    """Mid-circuit measurement workload (one ancilla pair measured and reset
    per round, after Listing 1).  Qubits 0 and 1 are the ancillas, 2..n-1 the
    system.  Each round: Ry(U[0,2pi)) and Rz(U[0,2pi)) on every qubit, a CNOT
    chain q_i -> q_{i+1}, CRy(U[0,pi]) from ancilla (j mod 2) onto system
    qubit j, measure q0 then q1, reset both.  Angles are shared by every
    trajectory.  MEASURE records carry slot = 2*round + ancilla."""
    n = n_sys + 2
    rng = _rng(seed)
    recs = []
    for r in range(rounds):
        for q in range(n):
            recs.append((KIND_RY, (q,), (rng.uniform(0, 2 * math.pi),)))
        for q in range(n):
            recs.append((KIND_RZ, (q,), (rng.uniform(0, 2 * math.pi),)))
        for q in range(n - 1):
            recs.append((KIND_CX, (q, q + 1), ()))
        for j in range(2, n):
            recs.append((KIND_CRY, (j % 2, j), (rng.uniform(0, math.pi),)))
        for a in (0, 1):
            recs.append((KIND_MEASURE, (a,), (), 2 * r + a))
        for a in (0, 1):
            recs.append((KIND_RESET, (a,), ()))
    return gates(recs)


def projection_filter(n_sys: int = 20, n_steps: int = 8, seed: int = 12, record: str = "assert",
                      t1: float = None, delta: float = 0.0):
    """Projection-filter workload on one ancilla (qubit 0) and n_sys system
    qubits (1..n_sys), with a synthetic diagonal Hamiltonian
    H = h0 + sum_j h_j Z_j (h0 = 0.1, h_j ~ N(0, 0.6^2)) standing in for the
    paper's nuclear Hamiltonians.  The trial state is a product of Ry(U[0, pi))
    rotations.  Step i applies exp[-i (H t_i + delta) Y_a], compiled as
    Ry_a(2 (t_i h0 + delta)) and, for every system qubit j, the exponential of
    t_i h_j Z_j Y_a (the two commute term by term because H is diagonal), with
    t_1 = pi / (2 Delta) (Delta = 2 sum |h_j|, the spectral width) unless given
    and t_i = t_(i-1) / 2.  After each step the ancilla is measured
    (record="measure", slot i) or asserted to 0 (record="assert", slot i),
    then reset.

    Returns (gates, info) with info = {"h0", "h", "t", "n"}."""
    rng = _rng(seed)
    h0 = 0.1
    h = rng.normal(0.0, 0.6, size=n_sys)
    if t1 is None:
        t1 = math.pi / (2.0 * 2.0 * float(np.abs(h).sum()))
    ts = [t1 / 2 ** i for i in range(n_steps)]
    recs = [(KIND_RY, (j + 1,), (float(rng.uniform(0, math.pi)),)) for j in range(n_sys)]
    kind = {"assert": KIND_ASSERT0, "measure": KIND_MEASURE}[record]
    for i, t in enumerate(ts):
        recs.append((KIND_RY, (0,), (2.0 * (t * h0 + delta),)))
        for j in range(n_sys):
            compile_pauli_exponential(np.array([0, j + 1]), np.array([2, 3]), 2.0 * t * float(h[j]), -1, recs)
        recs.append((kind, (0,), (), i))
        recs.append((KIND_RESET, (0,), ()))
    return gates(recs), {"h0": h0, "h": h, "t": ts, "n": n_sys + 1}


def uniforms(shape, seed: int = 5) -> np.ndarray:
    """float64 uniforms in [0, 1) used as measurement draws."""
    return _rng(seed).random(size=shape)


# ------------------------------------------------------------------ config 4
def batch_templates(wmin: int = 10, wmax: int = 20, n_exp: int = 500,
                    n_terms: int = 100):
    """One parameterised Pauli-exponential template and one Pauli sum per
    width; template seed (6, w), Hamiltonian seed (7, w)."""
    out = {}
    for w in range(wmin, wmax + 1):
        rng = _rng(6, w)
        strings = pauli_strings(w, n_exp, rng)
        recs = []
        for e, (qs, letters) in enumerate(strings):
            compile_pauli_exponential(qs, letters, 0.0, e, recs)
        out[w] = (gates(recs), pauli_sum(w, n_terms, seed=7000 + w))
    return out


def batch_instances(n_circuits: int = 4096, wmin: int = 10, wmax: int = 20,
                    n_exp: int = 500, sigma: float = 0.1, seed: int = 6):
    """Per-circuit width U{wmin..wmax} and angle vector N(0, sigma^2)^n_exp."""
    rng = _rng(seed, 1)
    widths = rng.integers(wmin, wmax + 1, size=n_circuits)
    thetas = rng.normal(0.0, sigma, size=(n_circuits, n_exp))
    return widths, thetas


# ------------------------------------------------------------------ config 5
def serving_requests(n_requests: int = 2000, wmin: int = 12, wmax: int = 30,
                     dmin_exp: float = 3.0, dmax_exp: float = 5.0,
                     rate: float = 100.0, seed: int = 8):
    """Poisson arrivals (exponential gaps, ``rate`` per second); width
    floor(exp(U[ln wmin, ln(wmax+1)))); depth floor(10^U[dmin, dmax]) gates
    of the Pauli-exponential style (about depth/9 exponentials).

    Returns a list of dicts with arrival time, width, circuit seed and the
    number of exponentials; the circuit itself is built lazily with
    :func:`request_circuit`."""
    rng = _rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        w = int(math.floor(math.exp(rng.uniform(math.log(wmin),
                                                math.log(wmax + 1)))))
        w = min(max(w, wmin), wmax)
        depth = int(math.floor(10 ** rng.uniform(dmin_exp, dmax_exp)))
        out.append({"id": i, "arrival": t, "width": w, "depth": depth,
                    "n_exp": max(1, depth // 9), "seed": 100000 + i})
    return out


def request_circuit(req) -> np.ndarray:
    g, _, _ = pauli_exponential_circuit(req["width"], req["n_exp"],
                                        req["seed"])
    return g


# --------------------------------------------------- random test matrices
def random_complex_matrix(dim: int, seed: int) -> np.ndarray:
    """A dense complex matrix with N(0,1) parts (not unitary): used to check
    that the update needs no unitarity and to catch transposed operands."""
    rng = _rng(seed, 99)
    return rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))


def random_unitary(dim: int, rng: np.random.Generator) -> np.ndarray:
    """A Haar-random unitary: QR of a complex Gaussian matrix, with the phases
    of R's diagonal moved into Q."""
    z = (rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))) / math.sqrt(2)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))


def dense_brickwork_circuit(n: int, layers: int, seed: int = 41):
    """Dense workload: `layers` brick-wall layers of Haar-random two-qubit
    unitaries (MAT records on (q, q+1), offset alternating between layers).
    Fusion merges them into dense 4-qubit operators (all 16 XOR shifts
    present).  Returns (gates, mats)."""
    rng = _rng(seed, 5)
    recs, mats = [], []
    for layer in range(layers):
        for q in range(layer % 2, n - 1, 2):
            recs.append((KIND_MAT, (q, q + 1), ()))
            mats.append(random_unitary(4, rng).ravel())
    g = gates(recs)
    off = 0
    for i in range(len(g)):
        g[i]["mat_off"] = off
        off += 16
    return g, np.concatenate(mats) if mats else np.zeros(0, complex)


def dense_operator_circuit(n: int, count: int, k: int = 5, seed: int = 43):
    """`count` Haar-random k-qubit unitaries (MAT records) on random qubits:
    every one a dense operator with all 2^k XOR shifts.  Returns
    (gates, mats)."""
    rng = _rng(seed, 6)
    recs, mats = [], []
    for _ in range(count):
        qs = [int(q) for q in rng.choice(n, size=k, replace=False)]
        recs.append((KIND_MAT, qs, ()))
        mats.append(random_unitary(1 << k, rng).ravel())
    g = gates(recs)
    for i in range(len(g)):
        g[i]["mat_off"] = i * (1 << (2 * k))
    return g, np.concatenate(mats) if mats else np.zeros(0, complex)


def random_state(n: int, seed: int) -> np.ndarray:
    """A normalised complex128 state with N(0,1) parts."""
    rng = _rng(seed, 98)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


QASM_NAMES = {
    KIND_ID: "id", KIND_H: "h", KIND_X: "x", KIND_Y: "y", KIND_Z: "z", KIND_S: "s", KIND_SDG: "sdg",
    KIND_T: "t", KIND_TDG: "tdg", KIND_SX: "sx", KIND_RX: "rx", KIND_RY: "ry", KIND_RZ: "rz",
    KIND_U1: "u1", KIND_U2: "u2", KIND_U3: "u3", KIND_CX: "cx", KIND_CY: "cy", KIND_CZ: "cz",
    KIND_CH: "ch", KIND_SWAP: "swap", KIND_CRX: "crx", KIND_CRY: "cry", KIND_CRZ: "crz",
    KIND_CU1: "cu1", KIND_CU3: "cu3", KIND_RXX: "rxx", KIND_RZZ: "rzz", KIND_CCX: "ccx",
    KIND_CSWAP: "cswap", KIND_C3X: "c3x", KIND_C3XSQRTX: "c3sqrtx", KIND_C4X: "c4x",
    KIND_RCCX: "rccx", KIND_RC3X: "rc3x",
}


def to_qasm(g: np.ndarray, n: int, n_clbits: int = 0) -> str:
    """OpenQASM 2.0 text of gate records (one qreg q[n], one creg c[n_clbits]
    when measurements occur; angles printed with 17 significant digits)."""
    lines = ["OPENQASM 2.0;", 'include "qelib1.inc";', f"qreg q[{n}];"]
    if n_clbits:
        lines.append(f"creg c[{n_clbits}];")
    for r in g:
        k = int(r["kind"])
        qs = ", ".join(f"q[{int(x)}]" for x in r["q"][:int(r["nq"])])
        if k == KIND_BARRIER:
            lines.append(f"barrier q;")
        elif k == KIND_MEASURE:
            lines.append(f"measure q[{int(r['q'][0])}] -> c[{int(r['slot'])}];")
        elif k == KIND_RESET:
            lines.append(f"reset q[{int(r['q'][0])}];")
        else:
            npar = KIND_NPARAMS.get(k, 0)
            par = "(" + ", ".join(repr(float(x)) for x in r["theta"][:npar]) + ")" if npar else ""
            lines.append(f"{QASM_NAMES[k]}{par} {qs};")
    return "\n".join(lines) + "\n"


def inverse_circuit(g: np.ndarray) -> np.ndarray:
    """The gate list of the inverse of a circuit made of self-inverse gates
    (H, X, Y, Z, CX, CY, CZ, SWAP) and rotations (angle negated): records in
    reverse order."""
    self_inverse = {KIND_ID, KIND_H, KIND_X, KIND_Y, KIND_Z, KIND_CX, KIND_CY,
                    KIND_CZ, KIND_SWAP, KIND_CCX, KIND_CSWAP, KIND_C3X, KIND_C4X}
    rot = {KIND_RX, KIND_RY, KIND_RZ, KIND_U1, KIND_CRX, KIND_CRY, KIND_CRZ,
           KIND_CU1, KIND_RXX, KIND_RZZ}
    out = g[::-1].copy()
    for i in range(len(out)):
        k = int(out[i]["kind"])
        if k in rot:
            out[i]["theta"][0] = -out[i]["theta"][0]
        elif k not in self_inverse:
            raise ValueError(f"no inverse record for kind {k}")
    return out


def probe_vectors(n: int, count: int, seed: int = 4049):
    """Yield ``count`` complex vectors of length 2^n with independent N(0,1)
    real and imaginary parts (E|r_x|^2 = 2).  For any fixed d, |<r|d>|^2
    averaged over such vectors estimates 2 ||d||^2: the tests compare a
    state with a stored one through these overlaps when the stored state is
    too large to keep."""
    for k in range(count):
        rng = _rng(seed, 97, k)
        yield rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
