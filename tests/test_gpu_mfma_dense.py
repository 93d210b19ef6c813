"""GPU parity of the dense matrix-core path: fused 4- and 5-qubit operators
with most XOR diagonals present, on complex64 states, applied as a
real-embedded contraction with FP32 MFMA, against the CPU oracle."""
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


def dense_records(n, k, count, seed):
    rng = np.random.default_rng(seed)
    recs, mats = [], []
    for i in range(count):
        qs = [int(q) for q in rng.choice(n, size=k, replace=False)]
        recs.append((W.KIND_MAT, qs, ()))
        mats.append(W.random_unitary(1 << k, rng).ravel())
    g = W.gates(recs)
    off = 0
    for i in range(len(g)):
        g[i]["mat_off"] = off
        off += len(mats[i])
    return g, np.concatenate(mats)


@pytest.mark.parametrize("n,k", [(14, 5), (17, 5), (13, 4), (16, 4)])
def test_dense_operators_on_matrix_cores(Q, n, k):
    """Dense operators applied one per sweep (k = 5 sweeps always; k = 4 with
    one operator per pass), both qubit orders mixed, against the oracle."""
    g, m = dense_records(n, k, 6, seed=n * 10 + k)
    print(f"mfma dense: n={n} k={k}", flush=True)
    psi0 = W.random_state(n, k)
    want, _, _ = oracle.run(n, g, psi=psi0, mats=m)
    sv = Q.StateVector(n, "complex64")
    sv.qsim_set_state(psi0)
    flags = Q.F_ONE_OP_PER_PASS if k == 4 else 0
    sv.qsim_apply(g, mats=m, max_width=5, flags=flags)
    got = sv.qsim_get_state()
    sv.close()
    assert oracle.infidelity(want, got) < 1e-5
    np.testing.assert_allclose(got, want, atol=1e-5 * np.abs(want).max())


def test_dense_fused_brickwork_width5(Q):
    """Brick-wall layers of random two-qubit unitaries fused up to 5 qubits
    with a high per-operator cost (dense 5-qubit operators), complex64."""
    n = 16
    g, m = W.dense_brickwork_circuit(n, 24, seed=3)
    want, _, _ = oracle.run(n, g, mats=m)
    sv = Q.StateVector(n, "complex64")
    sv.qsim_apply(g, mats=m, max_width=5, op_cost=40.0)
    st = sv.qsim_last_stats()
    got = sv.qsim_get_state()
    sv.close()
    assert st["max_width"] == 5
    assert oracle.infidelity(want, got) < 1e-5


def test_dense_operators_in_a_batch(Q):
    """The batched path hands strided operators to the same kernels, per state."""
    n = 13
    g, m = dense_records(n, 5, 3, seed=77)
    b = Q.Batch([{"n": n, "n_states": 3, "gates": g, "mats": m}], dtype="complex64", max_width=5)
    b.qsim_batch_run()
    want, _, _ = oracle.run(n, g, mats=m)
    for s in range(3):
        assert oracle.infidelity(want, b.qsim_batch_get_state(0, s)) < 1e-5
    b.close()
