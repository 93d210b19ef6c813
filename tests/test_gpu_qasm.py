"""GPU parity for circuits that arrive as OpenQASM 2.0 text (Section 4.1).

The text is parsed by qsim_parse_qasm and the records run through the HIP
path; the FP64 oracle runs the records the text was written from.  Same
tolerances as the other parity tests: complex128 within infidelity 1e-12,
complex64 within 1e-5; measurement outcomes bit-exact for the same draws.
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


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_parsed_pauli_circuit(Q, dtype):
    n = 16
    g, _, _ = W.pauli_exponential_circuit(n, 300, seed=21)
    got, nq, _ = Q.qsim_parse_qasm(W.to_qasm(g, n))
    assert nq == n
    say("qasm pauli", dtype)
    sv = Q.StateVector(n, dtype)
    sv.qsim_apply(got)
    want, _, _ = oracle.run(n, g)
    inf = oracle.infidelity(want, sv.qsim_get_state())
    assert inf < (1e-12 if dtype == "complex128" else 1e-5), inf


def test_parsed_definitions_and_broadcast(Q):
    """A user gate definition applied by broadcast over a register."""
    n = 12
    src = ["OPENQASM 2.0;", 'include "qelib1.inc";', "qreg q[6];", "qreg r[6];",
           "gate layer(a, b) x, y { ry(a) x; rz(b/2) y; cx x, y; rzz(a*b) x, y; }",
           "h q;", "layer(0.3, -1.1) q, r;", "cz r[0], q[5];", "layer(pi/7, 2.5) r, q;"]
    got, nq, _ = Q.qsim_parse_qasm("\n".join(src) + "\n")
    assert nq == n and len(got) == 6 + 4 * 6 + 1 + 4 * 6
    say("qasm definitions")
    sv = Q.StateVector(n, "complex128")
    sv.qsim_apply(got)
    want, _, _ = oracle.run(n, got)
    assert oracle.infidelity(want, sv.qsim_get_state()) < 1e-12


def test_parsed_trajectory_program(Q):
    """Measure and reset records from text: outcomes equal the oracle's for
    the same uniform draws, in complex128."""
    n_sys, rounds, ntraj = 5, 12, 16
    n = n_sys + 2
    g = W.trajectory_round_program(n_sys, rounds, seed=8)
    slots = 2 * rounds
    got, nq, nc = Q.qsim_parse_qasm(W.to_qasm(g, n, n_clbits=slots))
    assert (nq, nc) == (n, slots)
    u = W.uniforms((ntraj, slots), seed=9)
    say("qasm trajectories")
    b = Q.Batch([{"n": n, "n_states": ntraj, "gates": got, "uniforms": u, "n_slots": slots}],
                dtype="complex128")
    b.qsim_batch_run()
    res = b.qsim_batch_results(0)
    assert (res["status"] == 0).all()
    for t in range(ntraj):
        psi, oo, op = oracle.run(n, g, uniforms=u[t], n_slots=slots)
        np.testing.assert_array_equal(res["outcomes"][t], oo)
        np.testing.assert_allclose(res["probs"][t], op, atol=1e-12)
        assert oracle.infidelity(psi, b.qsim_batch_get_state(0, t)) < 1e-12
