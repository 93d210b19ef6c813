"""Host-only checks of the library's lowering and fusion (no GPU needed).

The fused operators exported by qsim_debug_fuse are applied by the CPU
oracle as dense matrix records; the result must equal the unfused circuit
run by the oracle (fusion is exact matrix algebra, Section 3.2: the update
need not be unitary, which is what makes fusion possible).
"""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from paper_2310_17739_amd import qsim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def fused_as_records(ops):
    recs, mats, off = [], [], 0
    for qs, m in ops:
        recs.append((W.KIND_MAT, qs, ()))
        mats.append(m.ravel())
        off += m.size
    g = W.gates(recs)
    o = 0
    for i, (qs, m) in enumerate(ops):
        g[i]["mat_off"] = o
        o += m.size
    return g, (np.concatenate(mats) if mats else np.zeros(0, complex))


def check_fused_equals_unfused(n, g, level, width, tol=1e-12, params=None, mats=None):
    ops, counts = qsim.qsim_debug_fuse(n, g, mats=mats, params=params, level=level, max_width=width)
    fg, fm = fused_as_records(ops)
    psi0 = W.random_state(n, seed=level * 10 + width)
    want, _, _ = oracle.run(n, g, psi=psi0, mats=mats, params=params)
    got, _, _ = oracle.run(n, fg, psi=psi0, mats=fm)
    assert oracle.infidelity(want, got) < tol
    np.testing.assert_allclose(got, want, atol=1e-11)
    return ops, counts


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4, 5])
def test_random_circuit_fusion_levels(level):
    n = 6
    g = W.random_circuit(n, 200, seed=1)
    ops, counts = check_fused_equals_unfused(n, g, level, 4)
    c = [x for x in counts if x >= 0]
    assert all(a >= b for a, b in zip(c, c[1:]))
    assert len(ops) == c[-1]


@pytest.mark.parametrize("width", [2, 3, 4, 5])
def test_all_gate_kinds_fusion(width):
    n = 7
    g = W.random_all_kinds(n, 150, seed=width)
    check_fused_equals_unfused(n, g, 5, width)


def test_pauli_exponentials_fusion():
    n = 8
    g, _, _ = W.pauli_exponential_circuit(n, 120, seed=5)
    ops, counts = check_fused_equals_unfused(n, g, 5, 4)
    # the F1..F2 steps merge each exponential's ladder into about 3 C2 operators
    assert counts[4] < counts[0] / 2.0
    # width-4 fusion leaves at most about one operator per exponential
    assert counts[5] <= 120


def test_matrix_records_and_both_orders():
    n = 6
    rng = np.random.default_rng(3)
    recs, mats, off = [], [], 0
    for i in range(30):
        k = int(rng.integers(1, 4))
        qs = list(rng.choice(n, size=k, replace=False))
        m = W.random_complex_matrix(1 << k, seed=i)
        recs.append((W.KIND_MAT, qs, ()))
        mats.append(m.ravel())
    g = W.gates(recs)
    o = 0
    for i in range(len(g)):
        g[i]["mat_off"] = o
        o += len(mats[i])
    allm = np.concatenate(mats)
    for level in (2, 4, 5):
        ops, _ = qsim.qsim_debug_fuse(n, g, mats=allm, level=level, max_width=4)
        fg, fm = fused_as_records(ops)
        psi0 = W.random_state(n, 1)
        want, _, _ = oracle.run(n, g, psi=psi0, mats=allm)
        got, _, _ = oracle.run(n, fg, psi=psi0, mats=fm)
        # non-unitary random factors: compare relative to the result's size
        assert np.max(np.abs(got - want)) < 1e-10 * np.max(np.abs(want))


def test_parameter_slots_bind_angles():
    n = 5
    recs = []
    for e in range(6):
        W.compile_pauli_exponential(np.array([e % n, (e + 2) % n]), np.array([1, 2]), 0.0, e, recs)
    g = W.gates(recs)
    params = np.linspace(-0.7, 0.9, 6)
    check_fused_equals_unfused(n, g, 5, 4, params=params)


def test_barrier_fences_fusion():
    g = W.gates([(W.KIND_H, (0,), ()), (W.KIND_BARRIER, (0,), ()), (W.KIND_H, (0,), ())])
    ops, counts = qsim.qsim_debug_fuse(2, g, level=5, max_width=4)
    assert len(ops) == 2
    g2 = W.gates([(W.KIND_H, (0,), ()), (W.KIND_H, (0,), ())])
    ops2, _ = qsim.qsim_debug_fuse(2, g2, level=5, max_width=4)
    assert len(ops2) == 1
    np.testing.assert_allclose(ops2[0][1], np.eye(2), atol=1e-15)


def test_f2_needs_swap_normalisation_for_reversed_pairs():
    """Level 3 (F2 without SWAP normalisation) cannot merge CX(a,b) with
    CX(b,a); level 4 (the paper's normalisation, Section 4.2) can."""
    g = W.gates([(W.KIND_CX, (0, 1), ()), (W.KIND_CX, (1, 0), ()), (W.KIND_CX, (0, 1), ())])
    _, c3 = qsim.qsim_debug_fuse(2, g, level=3, max_width=4)
    _, c4 = qsim.qsim_debug_fuse(2, g, level=4, max_width=4)
    assert c3[3] == 3 and c4[4] == 1
    check_fused_equals_unfused(2, g, 3, 4)
    check_fused_equals_unfused(2, g, 4, 4)


def test_lowering_errors():
    bad_q = W.gates([(W.KIND_H, (7,), ())])
    with pytest.raises(qsim.QsimError) as e:
        qsim.qsim_debug_fuse(3, bad_q)
    assert e.value.code == qsim.E_QUBIT
    dup = W.gates([(W.KIND_CX, (1, 1), ())])
    with pytest.raises(qsim.QsimError) as e:
        qsim.qsim_debug_fuse(3, dup)
    assert e.value.code == qsim.E_QUBIT
    nan = W.gates([(W.KIND_RX, (0,), (float("nan"),))])
    with pytest.raises(qsim.QsimError) as e:
        qsim.qsim_debug_fuse(3, nan)
    assert e.value.code == qsim.E_ARG
    meas = W.gates([(W.KIND_MEASURE, (0,), (), 0)])
    with pytest.raises(qsim.QsimError) as e:
        qsim.qsim_debug_fuse(3, meas)
    assert e.value.code == qsim.E_UNSUPPORTED


def test_parameter_and_matrix_bounds():
    """A parameter slot past the caller's vector, or a MAT record whose
    matrix runs past the caller's pool, is rejected (QSIM_E_ARG) instead of
    reading beyond the arrays."""
    g = W.gates([(W.KIND_RY, (0,), (0.0,), 3)])
    ops, _ = qsim.qsim_debug_fuse(2, g, params=np.zeros(4))
    assert len(ops) == 1
    for params in (None, np.zeros(3)):
        with pytest.raises(qsim.QsimError) as e:
            qsim.qsim_debug_fuse(2, g, params=params)
        assert e.value.code == qsim.E_ARG
    m = W.gates([(W.KIND_MAT, (0, 1), ())])
    m["mat_off"] = 4
    ok = np.zeros(20, complex)
    qsim.qsim_debug_fuse(2, m, mats=ok)
    with pytest.raises(qsim.QsimError) as e:
        qsim.qsim_debug_fuse(2, m, mats=np.zeros(19, complex))
    assert e.value.code == qsim.E_ARG


def test_plan_statistics():
    """The pass planner packs several fused operators per full-state pass."""
    g, _, _ = W.pauli_exponential_circuit(21, 1000, seed=2)
    s = qsim.qsim_debug_plan(21, g, "complex128")
    assert s["input_gates"] == len(g)
    assert s["passes"] < s["fused_ops"]
    one = qsim.qsim_debug_plan(21, g, "complex128", flags=qsim.F_ONE_OP_PER_PASS)
    assert one["passes"] == one["fused_ops"]
    # a state that fits one workgroup's LDS runs as resident passes over the
    # whole state, split only where the operator tables outgrow the LDS
    g14, _, _ = W.pauli_exponential_circuit(14, 300, seed=2)
    s14 = qsim.qsim_debug_plan(14, g14, "complex64")
    assert s14["tile_qubits"] == 14 and 1 <= s14["passes"] <= s14["fused_ops"] / 10
    g14s, _, _ = W.pauli_exponential_circuit(14, 20, seed=2)
    assert qsim.qsim_debug_plan(14, g14s, "complex64")["passes"] == 1


def test_plan_keeps_diagonal_qubits_outside_tiles():
    """Only the qubits an operator's XOR shifts move must lie in its tile:
    the Pauli-exponential benchmark circuit needs about a third fewer passes
    than with every operator qubit in the tile, with the same operators and
    terms; a circuit diagonal on every qubit fits a handful of passes."""
    g, _, _ = W.pauli_exponential_circuit(21, 3000, seed=2)
    for dt in ("complex128", "complex64"):
        a = qsim.qsim_debug_plan(21, g, dt)
        b = qsim.qsim_debug_plan(21, g, dt, flags=qsim.F_FULL_SUPPORT)
        assert (a["fused_ops"], a["terms"]) == (b["fused_ops"], b["terms"])
        assert a["passes"] < 0.75 * b["passes"], (dt, a["passes"], b["passes"])
    d = W.diagonal_rich_circuit(16, 400, seed=3, p_diag=1.0)
    a = qsim.qsim_debug_plan(16, d, "complex128", tile_qubits=9)
    b = qsim.qsim_debug_plan(16, d, "complex128", tile_qubits=9, flags=qsim.F_FULL_SUPPORT)
    assert a["passes"] <= 4 < b["passes"]


def test_abi_exports_every_declared_symbol():
    import ctypes
    lib = ctypes.CDLL(qsim.LIB_PATH)
    missing = [s for s in qsim.exported_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_profiler_ranges_library_mapped():
    """The library marks its calls and compile stages with roctx ranges
    (shown by rocprofv3 --marker-trace); the roctx library is mapped once the
    binding is loaded, and compiles run with the ranges in place."""
    g = W.random_circuit(8, 60, seed=5)
    assert qsim.qsim_debug_plan(8, g)["passes"] >= 1
    maps = open("/proc/self/maps").read()
    assert "librocprofiler-sdk-roctx" in maps


def test_one_hip_runtime_after_import():
    """Importing the binding in a fresh process (before anything else loads
    torch) maps a single HIP runtime: the library shares torch's."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2310_17739_amd import qsim\n"
            "import torch\n"
            "paths = set()\n"
            "for line in open('/proc/self/maps'):\n"
            "    p = line.split()[-1]\n"
            "    if 'libamdhip64' in p: paths.add(p)\n"
            "print(len(paths), sorted(paths))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.split()[0] == "1", out.stdout


def test_allocation_failure_reports_nomem_once():
    """The allocation-failure hook makes the next compile report
    QSIM_E_NOMEM; the call after it succeeds and gives the same plan."""
    g = W.random_circuit(8, 120, seed=4)
    ok = qsim.qsim_debug_plan(8, g)
    for call in (lambda: qsim.qsim_debug_plan(8, g), lambda: qsim.qsim_debug_emulate(8, g),
                 lambda: qsim.qsim_debug_fuse(8, g)):
        qsim.qsim_debug_fail_alloc(0)
        with pytest.raises(qsim.QsimError) as e:
            call()
        assert e.value.code == qsim.E_NOMEM
    again = qsim.qsim_debug_plan(8, g)
    assert again["passes"] == ok["passes"] and again["fused_ops"] == ok["fused_ops"]
    qsim.qsim_debug_fail_alloc(-1)


def test_level5_fusion_is_deterministic():
    """Level 5 computes its two candidates on concurrent threads (the run
    partition on its own worker pool, F1-F4 and the greedy merge beside it)
    and keeps the cheaper: the operators chosen, and every matrix entry,
    must not depend on thread timing."""
    g, _, _ = W.pauli_exponential_circuit(12, 1500, seed=5)
    runs = [qsim.qsim_debug_fuse(12, g, level=5, max_width=4) for _ in range(3)]
    ops0, counts0 = runs[0]
    for ops, counts in runs[1:]:
        assert list(counts) == list(counts0)
        assert len(ops) == len(ops0)
        for (qa, ma), (qb, mb) in zip(ops, ops0):
            assert tuple(qa) == tuple(qb)
            assert np.array_equal(ma, mb)


@pytest.mark.parametrize("first", ["qubit", "arg", "record"])
def test_first_bad_record_decides_the_error(first):
    """Lowering builds the operators of a long circuit on several threads;
    the error reported is still that of the first bad record in program
    order (a qubit out of range, a non-finite angle, a measurement record
    where none is allowed)."""
    n = 8
    g = W.random_circuit(n, 60000, seed=3)
    bad_q = W.gates([(W.KIND_H, (n,), ())])[0]
    bad_a = W.gates([(W.KIND_RX, (1,), (float("nan"),))])[0]
    rec = W.gates([(W.KIND_MEASURE, (0,), (), 0)])[0]
    order = {"qubit": (bad_q, bad_a, rec), "arg": (bad_a, rec, bad_q), "record": (rec, bad_q, bad_a)}[first]
    for pos, r in zip((7000, 31000, 52000), order):
        g[pos] = r
    with pytest.raises(qsim.QsimError) as e:
        qsim.qsim_debug_plan(n, g, "complex128")
    assert e.value.code == {"qubit": qsim.E_QUBIT, "arg": qsim.E_ARG, "record": qsim.E_UNSUPPORTED}[first]
