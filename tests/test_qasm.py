"""Host-only checks of the OpenQASM 2.0 frontend (qsim_parse_qasm).

The paper ingests its circuits as QASM text (Section 4.1) with the gate set
of its Table 3.  Records parsed from text must equal the records the text
was written from; parameter expressions follow ordinary arithmetic; gate
definitions expand with parameter substitution; errors name their line; and
a parsed circuit simulated by the oracle equals the original.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from paper_2310_17739_amd import qsim


def same_records(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        assert int(x["kind"]) == int(y["kind"])
        assert int(x["nq"]) == int(y["nq"])
        k = int(x["nq"])
        assert list(x["q"][:k]) == list(y["q"][:k])
        if int(x["kind"]) in (W.KIND_MEASURE,):
            assert int(x["slot"]) == int(y["slot"])
        npar = W.KIND_NPARAMS.get(int(x["kind"]), 0)
        np.testing.assert_array_equal(x["theta"][:npar], y["theta"][:npar])


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_round_trip_all_kinds(seed):
    n = 7
    g = W.random_all_kinds(n, 300, seed=seed)
    txt = W.to_qasm(g, n)
    got, nq, nc = qsim.qsim_parse_qasm(txt)
    assert nq == n and nc == 0
    same_records(got, g)     # 17 significant digits round-trip exactly


def test_round_trip_pauli_circuit_and_measurements():
    n = 9
    g, _, _ = W.pauli_exponential_circuit(n, 40, seed=4)
    m = W.trajectory_round_program(3, 2, seed=5)        # 5 qubits, measure / reset records
    txt = W.to_qasm(np.concatenate([g, m]), n, n_clbits=4)
    got, nq, nc = qsim.qsim_parse_qasm(txt)
    assert (nq, nc) == (n, 4)
    same_records(got, np.concatenate([g, m]))


def test_expressions():
    cases = ["pi/2", "-pi", "2*pi^2", "2^3^2", "-(1+2)*3", "sin(pi/6)+cos(0)", "exp(1)-ln(2)",
             "sqrt(2)/2", "1e-3*4", ".5", "tan(0.3)", "3-2-1", "8/4/2"]
    want = [math.pi / 2, -math.pi, 2 * math.pi ** 2, 2 ** 9, -9, 1.5, math.e - math.log(2),
            math.sqrt(2) / 2, 4e-3, 0.5, math.tan(0.3), 0, 1]
    body = "".join(f"rz({c}) q[0];\n" for c in cases)
    got, _, _ = qsim.qsim_parse_qasm("OPENQASM 2.0;\nqreg q[1];\n" + body)
    np.testing.assert_allclose(got["theta"][:, 0], want, rtol=0, atol=1e-15)


def test_gate_definitions_broadcast_and_registers():
    src = """OPENQASM 2.0;
include "qelib1.inc";
qreg a[2];
qreg b[3];
creg m[3];
gate inner(t) x { ry(t) x; }
gate outer(s, u) x, y { inner(2*s) y; cx x, y; inner(-u) x; barrier x, y; }
outer(0.25, pi) a[1], b[0];
h b;
cz a, b[1:0];
"""
    # 'b[1:0]' is not QASM: a syntax error, reported with its line
    with pytest.raises(qsim.QsimError) as e:
        qsim.qsim_parse_qasm(src)
    assert "line 10" in str(e.value)
    src = src.replace("cz a, b[1:0];", "cz a, b[1];\nmeasure b -> m;")
    got, nq, nc = qsim.qsim_parse_qasm(src)
    assert (nq, nc) == (5, 3)
    K = W
    want = W.gates([(K.KIND_RY, (2,), (0.5,)), (K.KIND_CX, (1, 2), ()), (K.KIND_RY, (1,), (-math.pi,)),
                    (K.KIND_H, (2,), ()), (K.KIND_H, (3,), ()), (K.KIND_H, (4,), ()),
                    (K.KIND_CZ, (0, 3), ()), (K.KIND_CZ, (1, 3), ()),
                    (K.KIND_MEASURE, (2,), (), 0), (K.KIND_MEASURE, (3,), (), 1),
                    (K.KIND_MEASURE, (4,), (), 2)])
    same_records(got, want)


@pytest.mark.parametrize("src,code,line", [
    ("OPENQASM 2.0;\nqreg q[2];\nh q[0]\ncx q[0], q[1];\n", "E_ARG", 4),            # missing ';'
    ("OPENQASM 2.0;\nqreg q[2];\ncreg c[1];\nif (c==1) x q[0];\n", "E_UNSUPPORTED", 4),
    ("OPENQASM 2.0;\nqreg q[2];\nopaque g a;\n", "E_UNSUPPORTED", 3),
    ("OPENQASM 2.0;\nqreg q[2];\nrccx q[0], q[1], q[0];\n", "E_QUBIT", 3),         # repeated qubit
    ("OPENQASM 2.0;\nqreg q[2];\nrx q[0];\n", "E_ARG", 3),                          # missing angle
    ("OPENQASM 2.0;\nqreg q[2];\nx q[2];\n", "E_QUBIT", 3),
    ("OPENQASM 2.0;\nqreg q[2];\ncx q[1], q[1];\n", "E_QUBIT", 3),
    ("OPENQASM 2.0;\nqreg q[2];\nqreg r[3];\ncx q, r;\n", "E_ARG", 4),              # unequal broadcast
    ("OPENQASM 3.0;\nqreg q[2];\n", "E_UNSUPPORTED", 1),
    ("OPENQASM 2.0;\nqreg q[2];\nrz(foo) q[0];\n", "E_ARG", 3),
])
def test_errors_name_their_line(src, code, line):
    with pytest.raises(qsim.QsimError) as e:
        qsim.qsim_parse_qasm(src)
    assert e.value.code == getattr(qsim, code)
    assert f"line {line}" in str(e.value)


def test_parsed_circuit_equals_original_on_the_oracle():
    """Parsing is exact: the oracle gives the same state from the text's
    records as from the records the text was written from."""
    n = 8
    g = W.random_all_kinds(n, 200, seed=9)
    got, _, _ = qsim.qsim_parse_qasm(W.to_qasm(g, n))
    a, _, _ = oracle.run(n, g)
    b, _, _ = oracle.run(n, got)
    np.testing.assert_array_equal(a, b)


def test_empty_program():
    got, nq, nc = qsim.qsim_parse_qasm("OPENQASM 2.0;\n")
    assert len(got) == 0 and nq == 0 and nc == 0
