"""The paper's measurement-assertion workflow end to end on the GPU (Section
4.3): projection-filter steps (Section 3.1, Eq. proj) with the ancilla
asserted to 0 and reset after each step, the tracked success probability,
then all shots sampled at once from the final state."""
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


def filter_steps(n_sys, steps, seed):
    """Trial state of Ry rotations; each step exp[-i (H t + delta) Y_a] with a
    diagonal H = h0 + sum_j h_j Z_j on the system qubits 1..n_sys."""
    rng = np.random.default_rng(seed)
    h0, h = 0.1, rng.normal(0, 0.6, size=n_sys)
    prep = W.gates([(W.KIND_RY, (j + 1,), (float(rng.uniform(0, math.pi)),)) for j in range(n_sys)])
    blocks = []
    for (t, d) in steps:
        recs = [(W.KIND_RY, (0,), (2 * (t * h0 + d),))]
        for j in range(n_sys):
            W.compile_pauli_exponential(np.array([0, j + 1]), np.array([2, 3]), 2 * t * h[j], -1, recs)
        blocks.append(W.gates(recs))
    return prep, blocks


@pytest.mark.parametrize("dtype,n_sys", [("complex128", 11), ("complex64", 17)])
def test_assertion_chain_and_sampling(Q, dtype, n_sys):
    n = n_sys + 1
    steps = [(1.3 / 2 ** i, 0.01 * i) for i in range(6)]
    prep, blocks = filter_steps(n_sys, steps, seed=n)
    sv = Q.StateVector(n, dtype)
    sv.qsim_apply(prep)
    psi, _, _ = oracle.run(n, prep)
    tracked_gpu, tracked_orc = 1.0, 1.0
    for blk in blocks:
        sv.qsim_apply(blk)
        psi, _, _ = oracle.run(n, blk, psi=psi)
        tracked_gpu *= sv.qsim_measure_assert(0)
        tracked_orc *= oracle.assert0(n, psi, 0)
        sv.qsim_reset(0)
        oracle.reset(n, psi, 0)
    tol = 1e-12 if dtype == "complex128" else 1e-5
    assert abs(tracked_gpu - tracked_orc) < tol * max(1.0, tracked_orc)
    got = sv.qsim_get_state()
    assert oracle.infidelity(psi, got) < tol
    u = W.uniforms(4096, seed=n)
    shots = sv.qsim_sample(u)
    want = oracle.sample(n, psi, u)
    mism = np.nonzero(shots != want)[0]
    if len(mism):
        # only draws on a cumulative boundary (within the precision) may differ
        c = np.cumsum(np.abs(psi) ** 2)
        for s in mism:
            edge = np.min(np.abs(c - u[s] * c[-1]))
            assert edge < (1e-12 if dtype == "complex128" else 1e-5), (s, edge)
    assert len(mism) <= (0 if dtype == "complex128" else 40)
    # the ancilla is |0> in every shot
    assert (shots & 1 == 0).all()


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_shots_reproduce_asserted_probability(Q, dtype):
    """The projection filter run shot by shot (the ancilla measured with a
    draw after every step, then reset) succeeds -- every outcome 0 -- at the
    rate the assertion chain tracks: P(all 0) = prod_i p_i (Section 4.3).
    4096 trajectories in one batch, against one asserted state."""
    n_sys, steps, ntraj = 10, 5, 4096
    # delta = 0.3 keeps the success rate near 0.44, where the count is most
    # sensitive to a wrong probability
    ga, info = W.projection_filter(n_sys, steps, seed=31, record="assert", delta=0.3)
    gm, _ = W.projection_filter(n_sys, steps, seed=31, record="measure", delta=0.3)
    n = info["n"]
    sv = Q.StateVector(n, dtype)
    ptrack = 1.0
    g_prev = 0
    # the asserted chain, one step at a time through the ABI
    rec_kinds = ga["kind"]
    cuts = [i for i in range(len(ga)) if rec_kinds[i] == W.KIND_ASSERT0]
    p_steps = []
    for c in cuts:
        sv.qsim_apply(ga[g_prev:c])
        p = sv.qsim_measure_assert(0)
        p_steps.append(p)
        ptrack *= p
        sv.qsim_reset(0)
        g_prev = c + 2          # skip the ASSERT0 and RESET records
    _, _, want_p = oracle.run(n, ga)
    tol = 1e-12 if dtype == "complex128" else 1e-5
    np.testing.assert_allclose(p_steps, want_p, atol=tol)
    u = W.uniforms((ntraj, steps), seed=32)
    say("shots vs assertion", dtype)
    b = Q.Batch([{"n": n, "n_states": ntraj, "gates": gm, "uniforms": u, "n_slots": steps}], dtype=dtype)
    b.qsim_batch_run()
    res = b.qsim_batch_results(0)
    assert (res["status"] == 0).all()
    ok = (res["outcomes"] == 0).all(axis=1)
    k = int(ok.sum())
    mean = ntraj * ptrack
    sd = math.sqrt(ntraj * ptrack * (1 - ptrack))
    assert abs(k - mean) <= 4.5 * sd, (k, mean, sd)
    # along every successful trajectory each step saw the asserted p_i
    np.testing.assert_allclose(res["probs"][ok], np.broadcast_to(want_p, (k, steps)), atol=max(tol, 1e-12) * 10)
