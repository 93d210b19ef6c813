"""Host-only checks of the pass planner and the packer (no GPU needed).

qsim_debug_emulate applies a circuit in FP64 from the packed device tables
of its compiled plan, reading the fields the tile kernel reads:
- the tile position table;
- the operator records (tile positions, present shifts, block qubits);
- the coefficient blocks.

The result must equal the oracle's plain gate-by-gate run (fusion is exact
matrix algebra, Section 3.2). This covers tile passes of every width, the
qubits an operator leaves outside its tile, resident whole-state passes,
strided sweeps of wide operators, and one-operator-per-pass plans.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from paper_2310_17739_amd import qsim


def check(got, want, rel=1e-12):
    assert oracle.infidelity(want, got) < 1e-12
    assert np.max(np.abs(got - want)) < rel * max(1.0, np.max(np.abs(want)))


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("n,tile", [(8, 5), (12, 8), (14, None), (15, 9), (16, 12)])
@pytest.mark.parametrize("gen", ["all_kinds", "pauli", "diagonal"])
def test_packed_plan_equals_oracle(dtype, n, tile, gen):
    if gen == "all_kinds":
        g = W.random_all_kinds(n, 300, seed=n)
    elif gen == "pauli":
        g, _, _ = W.pauli_exponential_circuit(n, 80, seed=n)
    else:
        g = W.diagonal_rich_circuit(n, 300, seed=n, p_diag=0.8)
    want, _, _ = oracle.run(n, g)
    for flags in (0, qsim.F_FULL_SUPPORT):
        check(qsim.qsim_debug_emulate(n, g, dtype, tile_qubits=tile, flags=flags), want)


def test_fully_diagonal_operators_outside_every_tile():
    """Operators diagonal on all their qubits address no tile position."""
    n = 14
    g = W.diagonal_rich_circuit(n, 400, seed=5, p_diag=1.0)
    psi0 = W.random_state(n, 2)
    want, _, _ = oracle.run(n, g, psi=psi0)
    check(qsim.qsim_debug_emulate(n, g, "complex128", tile_qubits=8, psi=psi0), want)


def test_dense_matrices_wide_operators_and_single_operator_passes():
    """Dense matrix records in both qubit orders, 5-qubit fused operators
    (strided sweeps) and plans with one operator per pass."""
    n = 11
    rng = np.random.default_rng(7)
    recs, mats = [], []
    for i in range(60):
        k = int(rng.integers(1, 4))
        qs = list(rng.choice(n, size=k, replace=False))
        recs.append((W.KIND_MAT, qs, ()))
        mats.append(W.random_complex_matrix(1 << k, seed=100 + i).ravel())
    g = W.gates(recs)
    o = 0
    for i in range(len(g)):
        g[i]["mat_off"] = o
        o += len(mats[i])
    allm = np.concatenate(mats)
    psi0 = W.random_state(n, 3)
    want, _, _ = oracle.run(n, g, psi=psi0, mats=allm)
    for kw in ({"tile_qubits": 7}, {"tile_qubits": 7, "max_width": 5},
               {"flags": qsim.F_ONE_OP_PER_PASS}, {"tile_qubits": 11}):
        got = qsim.qsim_debug_emulate(n, g, "complex64", mats=allm, psi=psi0, **kw)
        # random non-unitary factors: compare relative to the result's size
        check(got, want, rel=1e-10)


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("n,tile", [(15, 10), (15, 11), (16, 12), (16, 13)])
@pytest.mark.parametrize("gen", ["all_kinds", "pauli", "diagonal"])
def test_register_resident_passes_equal_oracle(dtype, n, tile, gen):
    """Tiles of 10..13 qubits run register-resident: every operator on the
    four register bits, qubits swapped in from lane bits 4 and 5, LDS
    re-layouts otherwise.  The emulation moves the elements exactly as the
    kernel does (position bits, lane/register exchanges, re-layouts checked
    against the layout the records before them leave)."""
    if gen == "all_kinds":
        g = W.random_all_kinds(n, 250, seed=n + tile, max_arity=4)
    elif gen == "pauli":
        g, _, _ = W.pauli_exponential_circuit(n, 120, seed=n + tile)
    else:
        g = W.diagonal_rich_circuit(n, 250, seed=n + tile, p_diag=0.7)
    psi0 = W.random_state(n, tile)
    want, _, _ = oracle.run(n, g, psi=psi0)
    st = qsim.qsim_debug_plan(n, g, dtype, tile_qubits=tile, flags=qsim.F_REG_ENGINE)
    assert st["reg_passes"] == st["passes"] > 0
    check(qsim.qsim_debug_emulate(n, g, dtype, tile_qubits=tile, psi=psi0, flags=qsim.F_REG_ENGINE), want)


def test_register_programs_use_swaps_and_relayouts():
    """On the benchmark-style circuit both ways of bringing a qubit onto the
    register bits occur, and low qubits are restored before the store."""
    g, _, _ = W.pauli_exponential_circuit(18, 400, seed=9)
    st = qsim.qsim_debug_plan(18, g, "complex128", flags=qsim.F_REG_ENGINE)
    assert st["reg_passes"] == st["passes"]
    assert qsim.qsim_debug_plan(18, g, "complex128")["reg_passes"] == 0
    assert st["reg_swaps"] > 0 and st["reg_relayouts"] > 0


def _pauli_strings_circuit(n, strings, seed):
    rng = np.random.default_rng(seed)
    recs = []
    for qs, letters in strings:
        W.compile_pauli_exponential(qs, letters, float(rng.normal(0, 0.4)), -1, recs)
    return W.gates(recs)


@pytest.mark.parametrize("n,tile,fewer", [(12, 7, False), (16, 10, True), (17, 10, True), (18, 9, False)])
def test_commuting_operators_pass_skipped_ones(n, tile, fewer, monkeypatch):
    """The planner moves an operator ahead of skipped ones it commutes with
    (functions of commuting Pauli strings, diagonals): on these circuits
    fewer passes than with qubit-disjoint reordering only, and always the
    same state as the oracle's gate-by-gate run.  Strings that share qubits mostly anticommute or
    commute at random, so a wrong reordering would show in the state."""
    g, _, _ = W.pauli_exponential_circuit(n, 240, seed=n + 7)
    # plus runs of mutually commuting strings on shared qubits (ZZ, XX, YY on
    # one pair commute pairwise)
    rng = np.random.default_rng(n)
    extra = []
    for _ in range(40):
        a, b = (int(x) for x in rng.choice(n, 2, replace=False))
        for l in (1, 2, 3):
            extra.append((np.array(sorted((a, b))), np.array([l, l])))
    g = np.concatenate([g, _pauli_strings_circuit(n, extra, seed=n)])
    want, _, _ = oracle.run(n, g)
    monkeypatch.setenv("QSIM_PLAN_COMMUTE", "0")
    off = qsim.qsim_debug_plan(n, g, "complex128", tile_qubits=tile)["passes"]
    monkeypatch.setenv("QSIM_PLAN_COMMUTE", "1")
    on = qsim.qsim_debug_plan(n, g, "complex128", tile_qubits=tile)["passes"]
    # (the greedy choice can also end a pass differently and cost one more)
    if fewer:
        assert on < off, (on, off)
    for dtype in ("complex128", "complex64"):
        check(qsim.qsim_debug_emulate(n, g, dtype, tile_qubits=tile), want)
