"""GPU parity at the configurations' full sizes.

* The 21-qubit benchmark circuit (50,000 Pauli exponentials, 450,728 gates,
  seed 2) in complex128 and complex64, in the launch configuration the
  benchmark times (default plan, one state), against the oracle's results
  stored by ``tests/golden/make_cfg2_fixture.py`` (a script that runs only
  the oracle): <H> and every term of the 100-term sum, <Z_i>, two 10-qubit
  marginals, 4,096 seeded amplitudes, and overlaps with 48 seeded Gaussian
  probe vectors.  For a difference d of the unit states, |<r|d>|^2 averages
  to 2||d||^2 over the probes, and 1 - |<a|b>|^2 <= ||a - b||^2 for unit
  states, so the probe estimate bounds the infidelity (a 48-probe estimate
  falls below half its mean with probability < 1e-4, hence the factor 2 in
  the bound).
* The mid-circuit measurement workload at its stated shape: 14 qubits (12
  system + 2 ancillas), 500 rounds, complex64 with FP64 reductions, 32
  trajectories with their own draws, against the oracle run with the same
  draws (outcomes, per-round probabilities, final states and norms).
* The batched workload at its stated shape (4,096 circuits of widths 10-20,
  500 exponentials each, own angles, one graph launch) with 64 seeded
  circuits checked against the oracle one by one.
"""
import hashlib
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
FIXTURE = os.path.join(HERE, "golden", "cfg2_21q_50k_oracle.npz")


@pytest.fixture(scope="module")
def Q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_17739_amd import qsim
    return qsim


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def probe_distance2(psi, fx):
    """Estimate of ||psi/|psi| - phi/|phi|||^2 for the oracle state phi
    described by the fixture (its probe overlaps and norm)."""
    n = int(fx["n"])
    a = np.asarray(psi, dtype=np.complex128)
    na = np.sqrt(np.vdot(a, a).real)
    nb = np.sqrt(float(fx["norm"]))
    acc = 0.0
    for k, r in enumerate(W.probe_vectors(n, len(fx["probe"]))):
        acc += abs(np.vdot(r, a) / na - fx["probe"][k] / nb) ** 2
    return acc / (2.0 * len(fx["probe"]))


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_headline_circuit_full(Q, dtype):
    fx = np.load(FIXTURE)
    n = int(fx["n"])
    g, _, _ = W.pauli_exponential_circuit(n, int(fx["n_exp"]), seed=2)
    assert len(g) == int(fx["n_gates"])
    assert hashlib.sha256(g.tobytes()).digest() == fx["gates_sha256"].tobytes()
    H = W.pauli_sum(n, 100, seed=3)
    csum = np.abs(H["coeff"]).sum()
    say("headline circuit, full,", dtype)
    sv = Q.StateVector(n, dtype)
    prog = Q.Program(n, g, dtype=dtype)
    sv.qsim_init_zero()
    prog.qsim_run(sv)
    e = sv.qsim_expval(H)
    terms = np.array([sv.qsim_expval(H[k:k + 1]) for k in range(len(H))])
    z = np.array([sv.qsim_expval(W.z_terms(n)[i:i + 1]) for i in range(n)])
    plo = sv.qsim_probs(list(range(10)))
    phi = sv.qsim_probs(list(range(11, 21)))
    psi = sv.qsim_get_state().astype(np.complex128)
    prog.close()
    sv.close()
    tol = 1e-12 if dtype == "complex128" else 1e-5
    d2 = probe_distance2(psi, fx)
    say(f"  {dtype}: probe ||d||^2 estimate {d2:.3e}, dE {abs(e - fx['energy']):.3e}")
    assert d2 <= tol / 2, d2
    assert abs(e - fx["energy"]) <= 1e-6 * csum
    np.testing.assert_allclose(terms, fx["term"], atol=1e-6 * csum / len(H))
    np.testing.assert_allclose(z, fx["z"], atol=(1e-12 if dtype == "complex128" else 1e-6))
    np.testing.assert_allclose(plo, fx["probs_lo"], atol=(1e-14 if dtype == "complex128" else 1e-8))
    np.testing.assert_allclose(phi, fx["probs_hi"], atol=(1e-14 if dtype == "complex128" else 1e-8))
    # sampled amplitudes, both normalised: the rms amplitude is 2^(-n/2)
    a = psi / np.sqrt(np.vdot(psi, psi).real)
    b = fx["sample_amp"] / np.sqrt(float(fx["norm"]))
    atol = 1e-13 if dtype == "complex128" else 1e-6
    np.testing.assert_allclose(a[fx["sample_idx"]], b, atol=atol)


def test_trajectories_full_shape(Q):
    """14 qubits (12 system + 2 ancillas), 500 rounds, complex64 sweeps with
    FP64 reductions, 32 trajectories."""
    n_sys, rounds, ntraj = 12, 500, 32
    n = n_sys + 2
    g = W.trajectory_round_program(n_sys, rounds, seed=4)
    u = W.uniforms((ntraj, 2 * rounds), seed=5)
    say("trajectories, 14 qubits x 500 rounds x", ntraj)
    b = Q.Batch([{"n": n, "n_states": ntraj, "gates": g, "uniforms": u, "n_slots": 2 * rounds}],
                dtype="complex64")
    b.qsim_batch_run()
    res = b.qsim_batch_results(0)
    assert (res["status"] == 0).all()
    ties = 0
    for t in range(ntraj):
        go = res["outcomes"][t]
        psi, oo, op = oracle.run(n, g, uniforms=u[t], forced=go, n_slots=2 * rounds)
        p0 = np.where(go == 0, op, 1 - op)
        decided = np.where(u[t] < p0, 0, 1)
        mism = decided != go
        # a draw within 1e-5 of the oracle's p0 may go either way in complex64
        assert np.all(np.abs(u[t][mism] - p0[mism]) < 1e-5), t
        ties += int(mism.sum())
        np.testing.assert_allclose(res["probs"][t], op, atol=2e-5)
        assert oracle.infidelity(psi, b.qsim_batch_get_state(0, t)) < 1e-5
        assert abs(res["norms"][t] - 1) < 1e-5
    say("  ties inside the 1e-5 window:", ties, "of", ntraj * 2 * rounds)
    b.close()


def test_batched_full_shape_sampled(Q):
    """4,096 circuits of widths U{10..20}, 500 exponentials each with their own
    angles, complex64 with FP64 <H>, one graph launch; 64 seeded circuits
    checked against the oracle."""
    tmpl = W.batch_templates(10, 20, 500, 100)
    widths, thetas = W.batch_instances(4096, 10, 20, 500)
    groups, index = [], []
    for w in range(10, 21):
        sel = np.nonzero(widths == w)[0]
        g, H = tmpl[w]
        groups.append({"n": w, "n_states": len(sel), "gates": g, "params": thetas[sel], "terms": H})
        index.append(sel)
    say("batched, 4096 circuits")
    b = Q.Batch(groups, dtype="complex64", use_graph=True)
    b.qsim_batch_run()
    rng = np.random.default_rng(np.random.SeedSequence([64, 4096]))
    pick = rng.choice(4096, size=64, replace=False)
    where = {}
    for gi, sel in enumerate(index):
        for j, c in enumerate(sel):
            where[int(c)] = (gi, j)
    worst = 0.0
    for c in pick:
        gi, j = where[int(c)]
        w = int(widths[c])
        g, H = tmpl[w]
        psi, _, _ = oracle.run(w, g, params=thetas[c])
        got = b.qsim_batch_get_state(gi, j)
        inf = oracle.infidelity(psi, got)
        worst = max(worst, inf)
        assert inf <= 1e-5, (c, w, inf)
        ev = b.qsim_batch_results(gi)["expvals"][j]
        assert abs(ev - oracle.expval(w, psi, H)) <= 1e-6 * np.abs(H["coeff"]).sum()
    say(f"  worst infidelity of 64 sampled circuits: {worst:.3e}")
    b.close()
