"""qsim_probs_noalloc, the entry point for callers that cannot allocate,
against qsim_probs through the C ABI: calls in a row on one device (the
second with a smaller input, the third a wide marginal), each checked
against the allocating call on the same state."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_probs_noalloc_matches_probs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_17739_amd import qsim
    out = torch.empty(4096 + 64, dtype=torch.float64, device="cuda")
    # (width, dtype, qubits): up to 8 qubits the reduction order is that of
    # qsim_probs, so the results must agree bit for bit; the second input is
    # smaller than the first
    cases = [(18, "complex128", [3, 17, 0, 9, 4, 11, 6, 14]), (12, "complex64", [5, 0, 9]),
             (20, "complex128", list(range(4, 16)))]
    for n, dtype, qs in cases:
        print(f"noalloc: n={n} {dtype} qubits={qs}", flush=True)
        g, _, _ = W.pauli_exponential_circuit(n, 300, seed=n)
        sv = qsim.StateVector(n, dtype)
        sv.qsim_apply(g)
        want = sv.qsim_probs(qs)
        out.fill_(-1.0)
        sv.qsim_probs_noalloc(qs, out)
        torch.cuda.synchronize()
        host = out.cpu().numpy()
        m = 1 << len(qs)
        got = host[:m]
        assert (host[m:] == -1.0).all()
        if len(qs) <= 8:
            assert np.array_equal(got, want)
        else:
            np.testing.assert_allclose(got, want, rtol=1e-12, atol=0)
        assert abs(got.sum() - 1.0) < 1e-12
        sv.close()


def test_probs_noalloc_rejects_bad_input():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_17739_amd import qsim
    out = torch.empty(16, dtype=torch.float64, device="cuda")
    sv = qsim.StateVector(6, "complex128")
    for qs, code in (([0, 0], qsim.E_QUBIT), ([6], qsim.E_QUBIT)):
        with pytest.raises(qsim.QsimError) as e:
            sv.qsim_probs_noalloc(qs, out)
        assert e.value.code == code
    sv.close()
