"""GPU parity of the batched form (qsim_batch_*) against the CPU oracle.

Trajectories with mid-circuit measurement (device-side decisions from
shared uniform draws), measurement assertion, parameterised templates with
per-state angles, and the invariance of a state's result to the batch it
runs in.
"""
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


def check_trajectories(Q, n, g, uniforms, dtype, res, batch, tol_state):
    """Outcomes equal the oracle's for the same draws; for complex64 a draw
    within 1e-5 of the oracle's p0 may go either way (the oracle is then
    forced to the GPU's outcome and the states compared conditionally)."""
    ntraj, nslots = uniforms.shape
    ties = 0
    for t in range(ntraj):
        go = res["outcomes"][t]
        psi, oo, op = oracle.run(n, g, uniforms=uniforms[t], forced=go, n_slots=nslots)
        # what the oracle decides with the draw, given the same history
        p_out = op
        p0 = np.where(go == 0, p_out, 1 - p_out)
        decided = np.where(uniforms[t] < p0, 0, 1)
        mism = decided != go
        if dtype == "complex128":
            assert not mism.any(), (t, np.nonzero(mism))
        else:
            assert np.all(np.abs(uniforms[t][mism] - p0[mism]) < 1e-5)
            ties += int(mism.sum())
        tol_p = 1e-12 if dtype == "complex128" else 2e-5
        np.testing.assert_allclose(res["probs"][t], op, atol=tol_p)
        got = batch.qsim_batch_get_state(0, t)
        assert oracle.infidelity(psi, got) < tol_state
        assert abs(res["norms"][t] - 1) < (1e-12 if dtype == "complex128" else 1e-5)
    return ties


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_trajectories_resident(Q, dtype):
    n_sys, rounds, ntraj = 6, 20, 64
    n = n_sys + 2
    g = W.trajectory_round_program(n_sys, rounds, seed=4)
    u = W.uniforms((ntraj, 2 * rounds), seed=5)
    say("trajectories resident", dtype)
    b = Q.Batch([{"n": n, "n_states": ntraj, "gates": g, "uniforms": u, "n_slots": 2 * rounds}], dtype=dtype)
    b.qsim_batch_run()
    res = b.qsim_batch_results(0)
    assert (res["status"] == 0).all()
    check_trajectories(Q, n, g, u, dtype, res, b, 1e-12 if dtype == "complex128" else 1e-5)


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_trajectories_tiled(Q, dtype):
    """States wider than one workgroup's LDS: measurements become a marginal
    reduction plus a device-side decision kernel between tiled passes."""
    n_sys, rounds, ntraj = 13, 3, 3
    n = n_sys + 2
    g = W.trajectory_round_program(n_sys, rounds, seed=7)
    u = W.uniforms((ntraj, 2 * rounds), seed=8)
    say("trajectories tiled", dtype)
    b = Q.Batch([{"n": n, "n_states": ntraj, "gates": g, "uniforms": u, "n_slots": 2 * rounds}],
                dtype=dtype, tile_qubits=10)
    b.qsim_batch_run()
    res = b.qsim_batch_results(0)
    assert (res["status"] == 0).all()
    check_trajectories(Q, n, g, u, dtype, res, b, 1e-12 if dtype == "complex128" else 1e-5)


def _record_runs_program(n, rounds, seed):
    """Rounds of Ry rotations and a CNOT chain, each followed by record runs
    that meet every reset-folding case: measure 0, measure 1, reset 0,
    reset 1 (two measure-then-reset records); assert 2, reset 2 (the reset
    is dropped); measure 3, reset 3, reset 3 (one record); measure 4, a gate,
    reset 4 and measure 5, a barrier, reset 5 (nothing joins).  Returns
    (gates, n_slots, measured slot mask, records per state with folding,
    records as written)."""
    rng = np.random.default_rng(seed)
    recs, measured, slot = [], [], 0
    for _ in range(rounds):
        for q in range(n):
            recs.append((W.KIND_RY, (q,), (rng.uniform(0, 2 * np.pi),)))
        for q in range(n - 1):
            recs.append((W.KIND_CX, (q, q + 1), ()))
        recs += [(W.KIND_MEASURE, (0,), (), slot), (W.KIND_MEASURE, (1,), (), slot + 1),
                 (W.KIND_RESET, (0,), ()), (W.KIND_RESET, (1,), ()),
                 (W.KIND_ASSERT0, (2,), (), slot + 2), (W.KIND_RESET, (2,), ()),
                 (W.KIND_MEASURE, (3,), (), slot + 3), (W.KIND_RESET, (3,), ()), (W.KIND_RESET, (3,), ()),
                 (W.KIND_MEASURE, (4,), (), slot + 4), (W.KIND_H, (5,), ()), (W.KIND_RESET, (4,), ()),
                 (W.KIND_MEASURE, (5,), (), slot + 5), (W.KIND_BARRIER, (5,), ()), (W.KIND_RESET, (5,), ())]
        measured += [True, True, False, True, True, True]
        slot += 6
    return W.gates(recs), slot, np.array(measured), 8 * rounds, 13 * rounds


@pytest.mark.parametrize("dtype,n,tile", [("complex128", 8, None), ("complex64", 8, None),
                                          ("complex128", 15, 10), ("complex64", 15, 10)])
def test_reset_folding(Q, dtype, n, tile, monkeypatch):
    """A reset that follows a record of its qubit with no gate or barrier
    between joins a measurement or is dropped (resident programs: one LDS
    rewrite; wider states: one decision sweep).  Outcomes, probabilities
    and states equal the oracle's for the same draws, and equal those of
    the program run with every record as written."""
    rounds, ntraj = (4, 32) if n <= 8 else (2, 3)
    g, nslots, measured, n_fold, n_all = _record_runs_program(n, rounds, seed=21)
    u = W.uniforms((ntraj, nslots), seed=22)
    tol = 1e-12 if dtype == "complex128" else 1e-5
    kw = {} if tile is None else {"tile_qubits": tile}
    say("reset folding", dtype, n, tile)

    def run(fold, forced=None):
        monkeypatch.setenv("QSIM_FOLD_RESETS", "1" if fold else "0")
        grp = {"n": n, "n_states": ntraj, "gates": g, "uniforms": u, "n_slots": nslots}
        if forced is not None:
            grp["forced"] = forced
        b = Q.Batch([grp], dtype=dtype, **kw)
        b.qsim_batch_run()
        res = b.qsim_batch_results(0)
        states = [b.qsim_batch_get_state(0, t) for t in range(ntraj)]
        info = b.qsim_batch_info()
        b.close()
        return res, states, info

    res, states, info = run(True)
    assert info["records"] == n_fold and (res["status"] == 0).all()
    for t in range(ntraj):
        go = res["outcomes"][t]
        psi, _, op = oracle.run(n, g, uniforms=u[t], forced=go, n_slots=nslots)
        p0 = np.where(go == 0, op, 1 - op)
        mism = measured & (np.where(u[t] < p0, 0, 1) != go)
        if dtype == "complex128":
            assert not mism.any(), (t, np.nonzero(mism))
        else:
            assert np.all(np.abs(u[t][mism] - p0[mism]) < 1e-5)
        assert np.all(go[~measured] == 0)
        np.testing.assert_allclose(res["probs"][t], op, atol=1e-12 if dtype == "complex128" else 2e-5)
        assert oracle.infidelity(psi, states[t]) < tol
    # the same program with every record as written, forced to the same outcomes
    res2, states2, info2 = run(False, forced=res["outcomes"])
    assert info2["records"] == n_all and (res2["status"] == 0).all()
    assert np.array_equal(res2["outcomes"], res["outcomes"])
    np.testing.assert_allclose(res2["probs"], res["probs"], atol=1e-12 if dtype == "complex128" else 2e-5)
    for t in range(ntraj):
        assert oracle.infidelity(states[t], states2[t]) < tol


@pytest.mark.parametrize("dtype,n,tile", [("complex128", 6, None), ("complex64", 6, None),
                                          ("complex128", 15, 10), ("complex64", 15, 10)])
def test_joined_measure_reset_zero_probability(Q, dtype, n, tile):
    """X then Ry(theta_b) on qubit 0, a measurement forced to 0, a reset of
    qubit 0 (joined to the measurement), a CNOT.  theta = 0 leaves
    P(0) = 0: that state fails with QSIM_E_ZERO_PROB and keeps its value
    from before the record; the others collapse to |0> on qubit 0 and go
    on, as the oracle does with the records as written."""
    recs = [(W.KIND_H, (1,), ()), (W.KIND_X, (0,), ()), (W.KIND_RY, (0,), (0.0,), 0),
            (W.KIND_MEASURE, (0,), (), 0), (W.KIND_RESET, (0,), ()), (W.KIND_CX, (1, n - 1), ())]
    g = W.gates(recs)
    thetas = np.array([[0.7], [0.0], [2.0], [1.3]])
    forced = np.zeros((4, 1), dtype=np.int32)
    kw = {} if tile is None else {"tile_qubits": tile}
    say("joined measure-reset, zero probability", dtype, n, tile)
    u = W.uniforms((4, 1), seed=3)   # measurements take draws even where every outcome is forced
    b = Q.Batch([{"n": n, "n_states": 4, "gates": g, "params": thetas, "uniforms": u, "forced": forced,
                  "n_slots": 1}], dtype=dtype, **kw)
    b.qsim_batch_run()
    res = b.qsim_batch_results(0)
    assert b.qsim_batch_info()["records"] == 1
    assert list(res["status"]) == [0, Q.E_ZERO_PROB, 0, 0]
    tol = 1e-12 if dtype == "complex128" else 1e-5
    for s_ in (0, 2, 3):
        psi, oo, pr = oracle.run(n, g, params=thetas[s_], uniforms=u[s_], forced=forced[s_], n_slots=1)
        assert res["outcomes"][s_][0] == oo[0] == 0
        assert abs(res["probs"][s_][0] - pr[0]) < (1e-12 if dtype == "complex128" else 2e-5)
        assert oracle.infidelity(psi, b.qsim_batch_get_state(0, s_)) < tol
    before, _, _ = oracle.run(n, g[:3], params=thetas[1])
    assert oracle.infidelity(before, b.qsim_batch_get_state(0, 1)) < tol
    b.close()


@pytest.mark.parametrize("n", [6, 15])
def test_assertion_failure_marks_only_that_state(Q, n):
    """X then Ry(theta_b) on the ancilla, then ASSERT0: theta = 0 leaves the
    ancilla exactly in |1>, P(0) = 0, which fails that state (Section 4.3)
    and no other.  (Ry(pi) would not do: cos(pi/2) is not 0 in FP64.)"""
    recs = [(W.KIND_H, (1,), ()), (W.KIND_X, (0,), ()), (W.KIND_RY, (0,), (0.0,), 0),
            (W.KIND_ASSERT0, (0,), (), 0), (W.KIND_RESET, (0,), ()), (W.KIND_CX, (1, n - 1), ())]
    g = W.gates(recs)
    thetas = np.array([[0.3], [0.0], [2.0], [1.0]])
    b = Q.Batch([{"n": n, "n_states": 4, "gates": g, "params": thetas, "n_slots": 1}], dtype="complex128",
                tile_qubits=10)
    b.qsim_batch_run()
    res = b.qsim_batch_results(0)
    assert list(res["status"]) == [0, Q.E_ZERO_PROB, 0, 0]
    for s in (0, 2, 3):
        psi, _, pr = oracle.run(n, g, params=thetas[s], n_slots=1)
        assert abs(res["probs"][s][0] - pr[0]) < 1e-12
        assert oracle.infidelity(psi, b.qsim_batch_get_state(0, s)) < 1e-12


@pytest.mark.parametrize("dtype", ["complex64", "complex128"])
def test_parameterised_templates_mixed_widths(Q, dtype):
    groups, want = [], []
    for w in (9, 12, 15):
        rng = np.random.default_rng(w)
        strings = W.pauli_strings(w, 40, rng)
        recs = []
        for e, (qs, letters) in enumerate(strings):
            W.compile_pauli_exponential(qs, letters, 0.0, e, recs)
        g = W.gates(recs)
        H = W.pauli_sum(w, 30, seed=w)
        th = rng.normal(0, 0.7, size=(6, 40))
        groups.append({"n": w, "n_states": 6, "gates": g, "params": th, "terms": H})
        want.append((w, g, H, th))
    say("templates", dtype)
    b = Q.Batch(groups, dtype=dtype, tile_qubits=10)
    b.qsim_batch_run()
    tol = 1e-12 if dtype == "complex128" else 1e-5
    for gi, (w, g, H, th) in enumerate(want):
        res = b.qsim_batch_results(gi)
        for s in range(6):
            psi, _, _ = oracle.run(w, g, params=th[s])
            assert oracle.infidelity(psi, b.qsim_batch_get_state(gi, s)) < tol
            assert abs(res["expvals"][s] - oracle.expval(w, psi, H)) <= 1e-6 * np.abs(H["coeff"]).sum()


def test_alone_equals_in_batch_and_graph_replays(Q):
    import torch
    w = 13
    rng = np.random.default_rng(3)
    strings = W.pauli_strings(w, 60, rng)
    recs = []
    for e, (qs, letters) in enumerate(strings):
        W.compile_pauli_exponential(qs, letters, 0.0, e, recs)
    g = W.gates(recs)
    th = rng.normal(0, 0.5, size=(8, 60))
    alone = Q.Batch([{"n": w, "n_states": 1, "gates": g, "params": th[5:6]}], dtype="complex64")
    alone.qsim_batch_run()
    a = alone.qsim_batch_get_state(0, 0)
    many = Q.Batch([{"n": w, "n_states": 8, "gates": g, "params": th}], dtype="complex64", use_graph=True)
    first = None
    for rep in range(3):
        many.qsim_batch_run()
        # eager work between replays
        x = torch.randn(1 << 16, device="cuda")
        (x * 2).sum().item()
        st = many.qsim_batch_get_state(0, 5)
        assert np.array_equal(st, a)
        if first is None:
            first = many.qsim_batch_results(0)["norms"]
        else:
            assert np.array_equal(many.qsim_batch_results(0)["norms"], first)


def test_autotuned_batch_uses_tuned_width(Q):
    """With autotune, each group's fusion width is timed (2..5 for complex64)
    on its template with the first state's angles, then the tile width of a
    group whose states need several tiles (12 or 13 qubits, timed over its
    states run together); the group is compiled with the fastest; results
    still match the oracle."""
    groups, want = [], []
    for w in (11, 16):
        rng = np.random.default_rng(100 + w)
        strings = W.pauli_strings(w, 60, rng)
        recs = []
        for e, (qs, letters) in enumerate(strings):
            W.compile_pauli_exponential(qs, letters, 0.0, e, recs)
        g = W.gates(recs)
        H = W.pauli_sum(w, 20, seed=w)
        th = rng.normal(0, 0.4, size=(3, 60))
        groups.append({"n": w, "n_states": 3, "gates": g, "params": th, "terms": H})
        want.append((w, g, H, th))
    say("autotuned batch")
    b = Q.Batch(groups, dtype="complex64", autotune=True)
    info = b.qsim_batch_info()
    assert info["tune_seconds"] > 0
    b.qsim_batch_run()
    for gi, (w, g, H, th) in enumerate(want):
        st = b.qsim_batch_group_stats(gi)
        assert 2 <= st["tuned_width"] <= 5 and st["max_width"] == st["tuned_width"]
        # a 14-qubit complex64 state is one tile; wider ones are tuned
        assert st["tile_qubits"] == w if w <= 14 else st["tile_qubits"] in (12, 13)
        res = b.qsim_batch_results(gi)
        for s in range(3):
            psi, _, _ = oracle.run(w, g, params=th[s])
            assert oracle.infidelity(psi, b.qsim_batch_get_state(gi, s)) < 1e-5
            assert abs(res["expvals"][s] - oracle.expval(w, psi, H)) <= 1e-6 * np.abs(H["coeff"]).sum()
    b.close()
