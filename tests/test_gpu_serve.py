"""Serving on the GPU: requests that run together give the results they give alone.

A burst of small requests is served with three slots (their work overlaps on the
device) on the BF16-split mixed path; each request is then served alone.  P(q, i nu),
Sigma(k, i omega) and the electron count must agree within the mixed path's tolerance (1e-5 relative, the
kernels being deterministic the difference is expected to be zero), the requests
must have overlapped in time, and one request is checked against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
import synthcell as sc
from synthcell import Request

pytestmark = pytest.mark.gpu

TOL = 1e-5


def relmax(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def executor():
    from paper_1911_05633_amd import serve
    from synthcell.device import ServingInputs
    return serve.GWExecutor(ServingInputs(), prec="bf16x3", capacity=16 << 30, slots=3, keep=("P", "S"))


MIX = [Request(0, 0.0, "si24", 16), Request(1, 0.0, "tiny2", 16), Request(2, 0.0, "si8", 16),
       Request(3, 0.0, "tiny2", 24), Request(4, 0.0, "si24", 24), Request(5, 0.0, "tiny2", 16)]


@pytest.fixture(scope="module")
def mixed(executor):
    from paper_1911_05633_amd import serve
    print("serve: burst of", len(MIX), "requests, 3 slots", flush=True)
    srv = serve.Server(executor, executor.capacity, slots=3)
    return srv.run(MIX)


def test_mix_completes_and_overlaps(mixed):
    assert [r.status for r in mixed] == ["done"] * len(MIX), [(r.status, r.error) for r in mixed]
    for r in mixed:
        assert abs(r.result["n"] - r.result["n_expected"]) < 1e-8 * r.result["n_expected"]
    spans = [(r.result["t_start"], r.result["t_end"]) for r in mixed]
    overlap = any(a0 < b1 and b0 < a1 for i, (a0, a1) in enumerate(spans) for (b0, b1) in spans[i + 1:])
    assert overlap, f"no two requests overlapped on the device: {spans}"


def test_each_result_alone_equals_result_in_the_mix(executor, mixed):
    from paper_1911_05633_amd import serve
    for req, rm in zip(MIX, mixed):
        print("serve: alone", req, flush=True)
        ra = serve.Server(executor, executor.capacity, slots=1).run([req])[0]
        assert ra.status == "done"
        for name in ("P", "S"):
            e = relmax(rm.result[name].numpy(), ra.result[name].numpy())
            assert e <= TOL, (req, name, e)
        assert rm.result["n"] == pytest.approx(ra.result["n"], rel=1e-12)


def test_served_tiny_request_matches_the_oracle(mixed):
    rec = mixed[1]  # tiny2, 16 tau points
    spec = sc.serving_cell("tiny2", 16, 0)
    b = sc.bands(spec, sc.hoppings(spec))
    Gk = sc.green_ktau(spec, b)
    C = sc.coefficients(spec)
    tau = sc.tau_grid(spec)
    WR = sc.w_tensor(spec)
    Pq = oracle.polarizability_q(Gk, spec, C, spec.spin)
    Pw = oracle.apply_tau_to_omega(oracle.filon_matrix(tau, oracle.bosonic_frequencies(spec.n_tau, spec.beta)), Pq)
    Sk = oracle.r_to_k(oracle.self_energy_r(oracle.k_to_r(Gk, spec.mesh), WR, spec, C), spec.mesh)
    Sw = oracle.apply_tau_to_omega(oracle.filon_matrix(tau, oracle.fermionic_frequencies(spec.n_tau, spec.beta)), Sk)
    eP = relmax(rec.result["P"].numpy().astype(np.complex128), Pw)
    eS = relmax(rec.result["S"].numpy(), Sw)
    print(f"served tiny2 vs oracle: P {eP:.2e}, Sigma {eS:.2e}", flush=True)
    assert eP <= TOL and eS <= TOL
