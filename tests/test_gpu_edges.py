"""GPU edge cases: empty circuits, one qubit, and the largest states the
configurations use (30 qubits complex64, 29 qubits complex128 = 8 GiB),
where the oracle cannot hold the state and outputs are checked one by one
against closed forms and against properties that hold at any size."""
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


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_empty_circuit_and_program(Q, dtype):
    n = 9
    sv = Q.StateVector(n, dtype)
    sv.qsim_apply(W.gates([]))
    st = sv.qsim_get_state()
    assert st[0] == 1 and np.count_nonzero(st) == 1
    prog = Q.Program(n, W.gates([]), dtype)
    assert prog.qsim_program_stats()["passes"] == 0
    sv.qsim_apply(W.gates([(W.KIND_H, (3,), ())]))
    prog.qsim_run(sv)                       # nothing to apply: state unchanged
    want, _, _ = oracle.run(n, W.gates([(W.KIND_H, (3,), ())]))
    np.testing.assert_allclose(sv.qsim_get_state(), want, atol=1e-7)
    assert abs(sv.qsim_norm() - 1) < 1e-6


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_one_qubit(Q, dtype):
    kinds = [W.KIND_H, W.KIND_X, W.KIND_Y, W.KIND_Z, W.KIND_S, W.KIND_SDG, W.KIND_T, W.KIND_TDG,
             W.KIND_SX, W.KIND_RX, W.KIND_RY, W.KIND_RZ, W.KIND_U1, W.KIND_U2, W.KIND_U3]
    rng = np.random.default_rng(5)
    recs = [(k, (0,), tuple(rng.uniform(0, 2 * math.pi, size=W.KIND_NPARAMS.get(k, 0)))) for k in kinds * 3]
    g = W.gates(recs)
    for level in (0, 5):
        sv = Q.StateVector(1, dtype)
        sv.qsim_apply(g, level=level)
        want, _, _ = oracle.run(1, g)
        assert oracle.infidelity(want, sv.qsim_get_state()) < (1e-12 if dtype == "complex128" else 1e-6)
    o, p = sv.qsim_measure(0, 0.25)
    assert o in (0, 1) and 0 < p <= 1


def product_circuit(n, seed):
    """Ry, Rz on every qubit, then CZ on (0,1), (2,3), ...: amplitude x is
    prod_j f_j(x_j) * (-1)^{#pairs with both bits set}."""
    rng = np.random.default_rng(seed)
    ay = rng.uniform(0, math.pi, size=n)
    az = rng.uniform(0, 2 * math.pi, size=n)
    recs = [(W.KIND_RY, (j,), (float(ay[j]),)) for j in range(n)]
    recs += [(W.KIND_RZ, (j,), (float(az[j]),)) for j in range(n)]
    recs += [(W.KIND_CZ, (j, j + 1), ()) for j in range(0, n - 1, 2)]
    return W.gates(recs), ay, az


def product_amplitudes(n, ay, az, xs):
    """Closed form of product_circuit, one amplitude at a time: Ry(a)|0> =
    (cos a/2, sin a/2); Rz(b) = diag(e^{-ib/2}, e^{ib/2})."""
    out = np.empty(len(xs), dtype=np.complex128)
    for i, x in enumerate(xs):
        a = 1.0 + 0j
        for j in range(n):
            bit = (int(x) >> j) & 1
            a *= (math.sin(ay[j] / 2) if bit else math.cos(ay[j] / 2)) * np.exp(1j * az[j] / 2 * (1 if bit else -1))
        pairs = sum(((int(x) >> j) & 1) & ((int(x) >> (j + 1)) & 1) for j in range(0, n - 1, 2))
        out[i] = a * (-1) ** pairs
    return out


@pytest.mark.parametrize("dtype,n", [("complex64", 30), ("complex128", 29)])
def test_largest_state_sampled_amplitudes(Q, dtype, n):
    """8 GiB states: 4096 sampled amplitudes of a closed-form circuit, the
    FP64 norm, and a Pauli-exponential circuit followed by its inverse."""
    import torch
    say("largest state", dtype, n)
    g, ay, az = product_circuit(n, seed=n)
    sv = Q.StateVector(n, dtype)
    sv.qsim_apply(g)
    xs = np.random.default_rng(n + 1).integers(0, 1 << n, size=4096)
    got = sv.tensor[torch.as_tensor(xs, device=sv.tensor.device)].cpu().numpy().astype(np.complex128)
    want = product_amplitudes(n, ay, az, xs)
    scale = np.abs(want).max()
    tol = 1e-12 if dtype == "complex128" else 2e-6
    assert np.abs(got - want).max() <= tol * max(scale, 1e-300) * 10 + (1e-15 if dtype == "complex128" else 0)
    assert abs(sv.qsim_norm() - 1) < (1e-10 if dtype == "complex128" else 1e-4)
    # probabilities of single qubits: (cos^2, sin^2)(ay_j / 2)
    for j in (0, n // 2, n - 1):
        p = sv.qsim_probs([j])
        assert abs(p[0] - math.cos(ay[j] / 2) ** 2) < (1e-10 if dtype == "complex128" else 1e-5)
    # a deep circuit and its inverse return the product state
    h, _, _ = W.pauli_exponential_circuit(n, 150, seed=n + 2)
    sv.qsim_apply(h)
    sv.qsim_apply(W.inverse_circuit(h))
    got2 = sv.tensor[torch.as_tensor(xs, device=sv.tensor.device)].cpu().numpy().astype(np.complex128)
    assert np.abs(got2 - want).max() <= (1e-10 if dtype == "complex128" else 1e-3) * scale
    sv.close()


def test_out_of_memory_leaves_state_unchanged(Q):
    """qsim_apply failing on any of its allocations (the compile, the pinned
    staging buffer, the device tables) returns QSIM_E_NOMEM and leaves the
    state as it was; the next call works."""
    n = 12
    g1, _, _ = W.pauli_exponential_circuit(n, 30, seed=1)
    g2, _, _ = W.pauli_exponential_circuit(n, 60, seed=2)
    for after in range(4):
        print("out of memory at allocation", after, flush=True)
        sv = Q.StateVector(n, "complex128")
        sv.qsim_apply(g1[:5])
        before = sv.qsim_get_state()
        Q.qsim_debug_fail_alloc(after)
        try:
            sv.qsim_apply(g2)
            failed = False
        except Q.QsimError as e:
            assert e.code == Q.E_NOMEM
            failed = True
        Q.qsim_debug_fail_alloc(-1)
        if failed:
            assert np.array_equal(sv.qsim_get_state(), before)
        sv.qsim_apply(g1)
        want, _, _ = oracle.run(n, np.concatenate([g1[:5]] + ([] if failed else [g2]) + [g1]))
        assert oracle.infidelity(want, sv.qsim_get_state()) < 1e-12
        sv.close()
