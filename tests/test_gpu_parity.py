"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances: complex128 states within infidelity 1e-12 and 1e-12 elementwise
(times a small factor for very deep circuits), complex64 states within
infidelity 1e-5; <H> within 1e-6 * sum|c|; measurement outcomes bit-exact
for the same uniform draws.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_17739_amd import qsim
    return qsim


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run_gpu(Q, n, g, dtype="complex128", **kw):
    sv = Q.StateVector(n, dtype)
    sv.qsim_apply(g, **kw)
    return sv


def check_state(got, want, dtype, tol128=1e-12):
    inf = oracle.infidelity(want, got)
    if dtype == "complex128":
        assert inf < tol128, inf
        np.testing.assert_allclose(got, want, atol=tol128 * 10)
    else:
        assert inf < 1e-5, inf
        np.testing.assert_allclose(got, want, atol=3e-4)
    return inf


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("level", [0, 2, 4, 5])
def test_cfg1_random_circuit(Q, dtype, level):
    n = 6
    g = W.random_circuit(n, 200, seed=1)
    say("cfg1", dtype, "level", level)
    sv = run_gpu(Q, n, g, dtype, level=level)
    want, _, _ = oracle.run(n, g)
    check_state(sv.qsim_get_state(), want, dtype)
    zt = W.z_terms(n)
    for q in range(n):
        assert abs(sv.qsim_expval(zt[q:q + 1]) - oracle.expval(n, want, zt[q:q + 1])) < (
            1e-12 if dtype == "complex128" else 1e-5)


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_one_op_per_pass(Q, dtype):
    n = 12
    g, _, _ = W.pauli_exponential_circuit(n, 60, seed=3)
    for level in (0, 5):
        say("one-op-per-pass", dtype, level)
        sv = run_gpu(Q, n, g, dtype, level=level, flags=Q.F_ONE_OP_PER_PASS)
        want, _, _ = oracle.run(n, g)
        check_state(sv.qsim_get_state(), want, dtype)


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("n,tile", [(10, None), (13, None), (14, None), (16, 8), (16, 10),
                                    (17, None), (18, 12)])
def test_pauli_circuits_tiled(Q, dtype, n, tile):
    g, _, _ = W.pauli_exponential_circuit(n, 250, seed=n)
    H = W.pauli_sum(n, 40, seed=n + 1)
    say("pauli", dtype, n, tile)
    sv = run_gpu(Q, n, g, dtype, tile_qubits=tile)
    st = sv.qsim_last_stats()
    want, _, _ = oracle.run(n, g)
    check_state(sv.qsim_get_state(), want, dtype)
    e = sv.qsim_expval(H)
    assert abs(e - oracle.expval(n, want, H)) <= 1e-6 * np.abs(H["coeff"]).sum()
    assert st["passes"] >= 1


@pytest.mark.parametrize("width", [2, 3, 4, 5])
def test_all_gate_kinds(Q, width):
    for n, tile in ((9, None), (15, 10)):
        g = W.random_all_kinds(n, 300, seed=width + n)
        for dtype in ("complex128", "complex64"):
            if dtype == "complex128" and width > 4:
                continue
            say("all kinds", n, tile, dtype, width)
            sv = run_gpu(Q, n, g, dtype, max_width=width, tile_qubits=tile)
            want, _, _ = oracle.run(n, g)
            check_state(sv.qsim_get_state(), want, dtype)


def test_dense_nonunitary_matrices(Q):
    n = 14
    rng = np.random.default_rng(1)
    recs, mats = [], []
    for i in range(40):
        k = int(rng.integers(1, 6))
        qs = list(rng.choice(n, size=k, replace=False))
        m = W.random_complex_matrix(1 << k, seed=500 + i)
        m /= np.linalg.norm(m, 2)   # keep the state bounded
        recs.append((W.KIND_MAT, qs, ()))
        mats.append(m.ravel())
    g = W.gates(recs)
    o = 0
    for i in range(len(g)):
        g[i]["mat_off"] = o
        o += len(mats[i])
    allm = np.concatenate(mats)
    psi0 = W.random_state(n, 4)
    want, _, _ = oracle.run(n, g, psi=psi0, mats=allm)
    for dtype, tile in (("complex128", 10), ("complex64", None)):
        say("dense matrices", dtype)
        sv = Q.StateVector(n, dtype)
        sv.qsim_set_state(psi0)
        sv.qsim_apply(g, mats=allm, max_width=5 if dtype == "complex64" else 4, tile_qubits=tile)
        got = sv.qsim_get_state()
        scale = np.max(np.abs(want))
        assert np.max(np.abs(got - want)) < (1e-12 if dtype == "complex128" else 2e-5) * scale


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("n", [11, 19])
def test_measure_assert_reset(Q, dtype, n):
    g = W.random_circuit(n, 400, seed=n)
    us = W.uniforms(12, seed=n)
    say("measure", dtype, n)
    sv = run_gpu(Q, n, g, dtype)
    psi, _, _ = oracle.run(n, g)
    tol = 1e-12 if dtype == "complex128" else 1e-5
    for i, q in enumerate([0, 3, n - 1, 5]):
        o_gpu, p_gpu = sv.qsim_measure(q, us[i])
        o_orc, p_orc = oracle.measure(n, psi, q, us[i])
        if abs(us[i] - p_orc if o_orc == 0 else us[i] - (1 - p_orc)) > 1e-5 or dtype == "complex128":
            assert o_gpu == o_orc
        assert abs(p_gpu - p_orc) < tol
        sv.qsim_reset(q)
        oracle.reset(n, psi, q)
    check_state(sv.qsim_get_state(), psi, dtype)
    p = sv.qsim_measure_assert(2)
    assert abs(p - oracle.assert0(n, psi, 2)) < tol
    check_state(sv.qsim_get_state(), psi, dtype)


def test_measurement_errors_leave_state(Q):
    n = 15
    sv = run_gpu(Q, n, W.gates([(W.KIND_X, (4,), ()), (W.KIND_H, (7,), ())]))
    before = sv.qsim_get_state()
    with pytest.raises(Q.QsimError) as e:
        sv.qsim_measure_assert(4)
    assert e.value.code == Q.E_ZERO_PROB
    with pytest.raises(Q.QsimError) as e:
        sv.qsim_reset(7)
    assert e.value.code == Q.E_NOT_DEFINITE
    with pytest.raises(Q.QsimError) as e:
        sv.qsim_measure(3, 1.0)
    assert e.value.code == Q.E_ARG
    with pytest.raises(Q.QsimError) as e:
        sv.qsim_apply(W.gates([(W.KIND_H, (n,), ())]))
    assert e.value.code == Q.E_QUBIT
    assert np.array_equal(sv.qsim_get_state(), before)
    sv.qsim_reset(4)   # definite |1> -> |0>
    psi = before.copy()
    oracle.reset(n, psi, 4)
    np.testing.assert_allclose(sv.qsim_get_state(), psi, atol=0)


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_probs_norm_expval(Q, dtype):
    n = 17
    g, _, _ = W.pauli_exponential_circuit(n, 200, seed=9)
    sv = run_gpu(Q, n, g, dtype)
    psi, _, _ = oracle.run(n, g)
    tol = 1e-12 if dtype == "complex128" else 2e-6
    for qs in ([0], [16], [3, 0, 9], list(range(8))):
        np.testing.assert_allclose(sv.qsim_probs(qs), oracle.probs(n, psi, qs), atol=tol)
    assert abs(sv.qsim_norm() - 1) < (1e-12 if dtype == "complex128" else 1e-4)
    H = W.pauli_sum(n, 100, seed=4)
    assert abs(sv.qsim_expval(H) - oracle.expval(n, psi, H)) <= 1e-6 * np.abs(H["coeff"]).sum()


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_expval_terms_sharing_x_masks(Q, dtype):
    """Terms with a common X mask share one read of the state (rows of up to
    8 terms, served by kernels for rows of 8, 4, 2 and 1 terms): all-Z
    terms, 11 terms on one X mask (two rows), X masks with 2, 4 and 6
    terms, and singles, in scrambled order; each term and the sum against
    the oracle."""
    n = 16
    g, _, _ = W.pauli_exponential_circuit(n, 150, seed=31)
    sv = run_gpu(Q, n, g, dtype)
    psi, _, _ = oracle.run(n, g)
    rng = np.random.default_rng(8)
    terms = []
    for i in range(n):
        terms.append((rng.normal(), 0, 1 << i))
    xm = (1 << 3) | (1 << 9) | (1 << 14)
    for j in range(11):
        terms.append((rng.normal(), xm, int(rng.integers(0, 1 << n))))
    for cnt, xo in ((2, (1 << 0) | (1 << 5)), (4, 1 << 12), (6, (1 << 2) | (1 << 7) | (1 << 15))):
        for j in range(cnt):
            terms.append((rng.normal(), xo, int(rng.integers(0, 1 << n))))
    H0 = W.pauli_sum(n, 12, seed=5)
    for t in H0:
        terms.append((float(t["coeff"]), int(t["xmask"]), int(t["zmask"])))
    order = rng.permutation(len(terms))
    H = np.array([terms[i] for i in order], dtype=W.PAULI_DTYPE)
    tol = 1e-6 * np.abs(H["coeff"]).sum()
    assert abs(sv.qsim_expval(H) - oracle.expval(n, psi, H)) <= tol
    for k in range(0, len(H), 7):
        assert abs(sv.qsim_expval(H[k:k + 1]) - oracle.expval(n, psi, H[k:k + 1])) <= 1e-6 * abs(H["coeff"][k])


def test_deterministic_repeat(Q):
    n = 20
    g, _, _ = W.pauli_exponential_circuit(n, 300, seed=12)
    H = W.pauli_sum(n, 50, seed=13)
    a = run_gpu(Q, n, g, "complex64")
    b = run_gpu(Q, n, g, "complex64")
    assert np.array_equal(a.qsim_get_state(), b.qsim_get_state())
    assert a.qsim_expval(H) == b.qsim_expval(H)
    assert a.qsim_norm() == b.qsim_norm()


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_cfg2_full_width_prefix(Q, dtype):
    """21 qubits in the benchmark's launch configuration, on the first 400
    exponentials of the benchmark circuit (the oracle finishes in seconds)."""
    n = 21
    g, _, _ = W.pauli_exponential_circuit(n, 400, seed=2)
    H = W.pauli_sum(n, 100, seed=3)
    say("cfg2 prefix", dtype)
    sv = run_gpu(Q, n, g, dtype)
    want, _, _ = oracle.run(n, g)
    check_state(sv.qsim_get_state(), want, dtype)
    assert abs(sv.qsim_expval(H) - oracle.expval(n, want, H)) <= 1e-6 * np.abs(H["coeff"]).sum()


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_wide_state_default_tiles(Q, dtype):
    """23 qubits with the default options: complex64 takes 13-qubit tiles
    from 23 qubits up (several tiles per CU), complex128 12-qubit tiles."""
    n = 23
    g, _, _ = W.pauli_exponential_circuit(n, 60, seed=23)
    H = W.pauli_sum(n, 30, seed=24)
    say("wide default tiles", dtype)
    sv = run_gpu(Q, n, g, dtype)
    st = sv.qsim_last_stats()
    assert st["tile_qubits"] == (13 if dtype == "complex64" else 12)
    want, _, _ = oracle.run(n, g)
    check_state(sv.qsim_get_state(), want, dtype)
    assert abs(sv.qsim_expval(H) - oracle.expval(n, want, H)) <= 1e-6 * np.abs(H["coeff"]).sum()


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_cfg2_full_circuit_inverse_property(Q, dtype):
    """The full benchmark circuit (50,000 exponentials, 21 qubits) followed
    by its inverse returns |0...0>: a property that holds at any size."""
    n = 21
    g, _, _ = W.pauli_exponential_circuit(n, 50_000, seed=2)
    say("cfg2 full + inverse", dtype)
    sv = run_gpu(Q, n, g, dtype)
    nrm = sv.qsim_norm()
    sv.qsim_apply(W.inverse_circuit(g))
    st = sv.qsim_get_state()
    p0 = abs(complex(st[0])) ** 2 / nrm
    if dtype == "complex128":
        assert abs(nrm - 1) < 1e-9 and 1 - p0 < 1e-9
    else:
        assert abs(nrm - 1) < 1e-3 and 1 - p0 < 1e-4


def test_autotune_picks_valid_options(Q):
    n = 18
    g, _, _ = W.pauli_exponential_circuit(n, 400, seed=21)
    sv = Q.StateVector(n, "complex64")
    best, ns = sv.qsim_autotune(g, prefix_gates=2000)
    assert best.level == 5 and 3 <= best.max_width <= 5 and ns > 0
    # state left at |0...0>, and the tuned options give the oracle's result
    st = sv.qsim_get_state()
    assert st[0] == 1 and np.count_nonzero(st) == 1
    sv.qsim_apply(g, level=best)
    want, _, _ = oracle.run(n, g)
    check_state(sv.qsim_get_state(), want, "complex64")


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_program_graph_replays_match_eager(Q, dtype):
    """A compiled program captured as a HIP graph: every replay (with eager
    work and synchronisations between them) equals the eager run."""
    import torch
    n = 19
    g, _, _ = W.pauli_exponential_circuit(n, 300, seed=33)
    prog = Q.Program(n, g, dtype)
    eager = Q.StateVector(n, dtype)
    prog.qsim_run(eager)
    want = eager.qsim_get_state()
    sv = Q.StateVector(n, dtype)
    prog.qsim_program_graph(sv, True)
    for rep in range(3):
        sv.qsim_init_zero()
        prog.qsim_run(sv)
        x = torch.randn(1 << 18, device="cuda")
        assert torch.isfinite((x * x).sum()).item()
        torch.cuda.synchronize()
        assert np.array_equal(sv.qsim_get_state(), want), rep
    ref, _, _ = oracle.run(n, g)
    check_state(want, ref, dtype)


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("p_diag", [0.8, 1.0])
@pytest.mark.parametrize("n,tile", [(16, 9), (17, None)])
def test_block_qubits_outside_tile(Q, dtype, p_diag, n, tile):
    """Qubits an operator is diagonal on may stay outside the tile, where the
    tile's base index picks the operator's coefficient block.  With p_diag = 1
    every operator is diagonal on all its qubits (no qubit addressed in the
    tile).  Both plans match the oracle, and the default one takes fewer
    passes than keeping every operator qubit in the tile."""
    g = W.diagonal_rich_circuit(n, 500, seed=n + int(10 * p_diag), p_diag=p_diag)
    want, _, _ = oracle.run(n, g)
    passes = {}
    for flags in (0, Q.F_FULL_SUPPORT):
        say("block qubits", dtype, p_diag, n, tile, flags)
        sv = run_gpu(Q, n, g, dtype, tile_qubits=tile, flags=flags)
        check_state(sv.qsim_get_state(), want, dtype)
        passes[flags] = sv.qsim_last_stats()["passes"]
    assert passes[0] < passes[Q.F_FULL_SUPPORT], passes


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_register_operators_on_and_off(Q, dtype, monkeypatch):
    """The first and last operators of a tiled pass may run on a thread's
    registers (the tile as loaded, the tile as stored); with the planner's
    placement switched off every operator runs in LDS.  Both plans match the
    oracle, on a circuit of mixed kinds, at several tile sizes."""
    n = 17
    g = W.random_all_kinds(n, 400, seed=23)
    psi0 = W.random_state(n, 4)
    want, _, _ = oracle.run(n, g, psi=psi0)
    for flag in ("1", "0"):
        monkeypatch.setenv("QSIM_FIRST_IN_REGS", flag)
        for tile in (10, 12, 13):
            say("register operators", dtype, flag, tile)
            sv = Q.StateVector(n, dtype)
            sv.qsim_set_state(psi0)
            sv.qsim_apply(g, tile_qubits=tile)
            check_state(sv.qsim_get_state(), want, dtype)
