"""GPU checks of the serving form (qsim_server_*): continuous batching with
HBM-byte admission.  Every result matches the oracle; a request's result is
bit-identical alone and in a mix of concurrent requests."""
import sys
import time

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


def collect(srv, count, timeout=60.0):
    got = {}
    t0 = time.time()
    while len(got) < count:
        for r in srv.qsim_server_poll(wait_ms=50):
            got[r["id"]] = r
        assert time.time() - t0 < timeout, f"only {len(got)} of {count} results"
    return got


def requests(seed, count, wmin=8, wmax=17):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        w = int(rng.integers(wmin, wmax + 1))
        g, _, _ = W.pauli_exponential_circuit(w, int(rng.integers(10, 120)), seed=1000 * seed + i)
        out.append((w, g, W.pauli_sum(w, 20, seed=2000 * seed + i)))
    return out


@pytest.mark.parametrize("dtype", ["complex64", "complex128"])
def test_served_results_match_oracle(Q, dtype):
    reqs = requests(1, 24)
    srv = Q.Server(dtype=dtype, slots=6, compile_threads=3, pool_bytes=64 << 20)
    ids = [srv.qsim_server_submit(w, g, terms=H, want_state=True) for (w, g, H) in reqs]
    got = collect(srv, len(ids))
    tol = 1e-12 if dtype == "complex128" else 1e-5
    for rid, (w, g, H) in zip(ids, reqs):
        r = got[rid]
        assert r["status"] == 0
        psi, _, _ = oracle.run(w, g)
        assert oracle.infidelity(psi, r["state"]) < tol
        assert abs(r["expval"] - oracle.expval(w, psi, H)) <= 1e-6 * np.abs(H["coeff"]).sum()
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
    st = srv.qsim_server_stats()
    assert st["completed"] == len(ids) and st["in_flight"] == 0 and st["pool_in_use"] == 0
    srv.close()


def test_alone_equals_in_mix(Q):
    """The probe's state, <H> and norm are bit-identical run alone and in a
    mix.  The mix starts with a long anchor request (19 qubits, 20,000
    exponentials); the probe and the others are submitted once the anchor
    is admitted, so the probe runs while the anchor is resident."""
    reqs = requests(2, 16, 10, 19)
    probe = reqs[7]
    alone = Q.Server(dtype="complex64", slots=1, compile_threads=1, pool_bytes=64 << 20)
    a_id = alone.qsim_server_submit(probe[0], probe[1], terms=probe[2], want_state=True)
    a = collect(alone, 1)[a_id]
    alone.close()
    mix = Q.Server(dtype="complex64", slots=8, compile_threads=4, pool_bytes=64 << 20)
    anchor = W.pauli_exponential_circuit(19, 20000, seed=77)[0]
    anchor_id = mix.qsim_server_submit(19, anchor)
    t0 = time.time()
    while mix.qsim_server_stats()["in_flight"] < 1:
        assert time.time() - t0 < 60, "the anchor was not admitted"
        time.sleep(0.0005)
    order = [7] + [i for i in range(len(reqs)) if i != 7]
    ids = {i: mix.qsim_server_submit(reqs[i][0], reqs[i][1], terms=reqs[i][2], want_state=(i == 7))
           for i in order}
    got = collect(mix, len(ids) + 1)
    m = got[ids[7]]
    assert np.array_equal(m["state"], a["state"])
    assert m["expval"] == a["expval"] and m["norm"] == a["norm"]
    # the probe shared the device: its admit..done interval lies inside the
    # anchor's, and several requests were resident at once
    an = got[anchor_id]
    assert an["status"] == 0
    assert an["t_admit"] < m["t_admit"] and m["t_done"] < an["t_done"], "the probe ran alone in the mix"
    assert mix.qsim_server_stats()["peak_in_flight"] > 1
    mix.close()


def test_admission_by_pool_bytes(Q):
    # a 2 MiB pool holds one 18-qubit complex64 state (2 MiB) at a time
    srv = Q.Server(dtype="complex64", slots=4, compile_threads=2, pool_bytes=2 << 20)
    with pytest.raises(Q.QsimError) as e:
        srv.qsim_server_submit(19, W.gates([(W.KIND_H, (0,), ())]))
    assert e.value.code == Q.E_CAPACITY
    reqs = [(18, W.pauli_exponential_circuit(18, 30, seed=s)[0]) for s in range(4)]
    ids = [srv.qsim_server_submit(w, g) for w, g in reqs]
    got = collect(srv, len(ids))
    st = srv.qsim_server_stats()
    assert st["rejected"] == 1 and st["pool_peak"] <= 2 << 20
    # one at a time: admission intervals do not overlap
    spans = sorted((got[i]["t_admit"], got[i]["t_done"]) for i in ids)
    for (a0, d0), (a1, d1) in zip(spans, spans[1:]):
        assert a1 >= d0 - 1e-3
    for i in ids:
        assert got[i]["status"] == 0 and abs(got[i]["norm"] - 1) < 1e-5
    srv.close()
