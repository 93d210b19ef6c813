"""GPU parity of the register-resident tile kernel (QSIM_F_REG_ENGINE),
against the CPU oracle: every tile width it serves (10..13 qubits), both
precisions, circuits whose operators need lane/register exchanges and LDS
re-layouts, and the batched path with per-state coefficients."""
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


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("tile", [10, 11, 12, 13])
@pytest.mark.parametrize("gen", ["pauli", "all_kinds"])
def test_reg_engine_matches_oracle(Q, dtype, tile, gen):
    n = 17
    if gen == "pauli":
        g, _, _ = W.pauli_exponential_circuit(n, 400, seed=tile)
    else:
        g = W.random_all_kinds(n, 400, seed=tile, max_arity=4)
    print(f"reg engine: {gen} n={n} tile={tile} {dtype}", flush=True)
    st = Q.qsim_debug_plan(n, g, dtype, tile_qubits=tile, flags=Q.F_REG_ENGINE)
    assert st["reg_passes"] == st["passes"] > 0
    want, _, _ = oracle.run(n, g)
    sv = Q.StateVector(n, dtype)
    sv.qsim_apply(g, tile_qubits=tile, flags=Q.F_REG_ENGINE)
    got = sv.qsim_get_state()
    sv.close()
    tol = 1e-12 if dtype == "complex128" else 1e-5
    assert oracle.infidelity(want, got) < tol


def test_reg_engine_batched_templates(Q):
    w = 15
    rng = np.random.default_rng(21)
    strings = W.pauli_strings(w, 80, rng)
    recs = []
    for e, (qs, letters) in enumerate(strings):
        W.compile_pauli_exponential(qs, letters, 0.0, e, recs)
    g = W.gates(recs)
    H = W.pauli_sum(w, 30, seed=4)
    th = rng.normal(0, 0.6, size=(5, 80))
    print("reg engine: batched templates", flush=True)
    b = Q.Batch([{"n": w, "n_states": 5, "gates": g, "params": th, "terms": H}], dtype="complex64",
                tile_qubits=10, flags=Q.F_REG_ENGINE)
    b.qsim_batch_run()
    res = b.qsim_batch_results(0)
    for s in range(5):
        psi, _, _ = oracle.run(w, g, params=th[s])
        assert oracle.infidelity(psi, b.qsim_batch_get_state(0, s)) < 1e-5
        assert abs(res["expvals"][s] - oracle.expval(w, psi, H)) <= 1e-6 * np.abs(H["coeff"]).sum()
    b.close()
