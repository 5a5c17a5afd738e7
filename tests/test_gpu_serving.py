"""GPU: the continuous-batching server. Requests of mixed sizes and dtypes
arrive while others run; each result equals the same circuit run alone
(bitwise: the same plan and tile arithmetic) and matches the oracle."""
import numpy as np
import pytest

import oracle
import paper_1801_01037_amd as sv
from paper_1801_01037_amd import serving
from tests.gpu_helpers import assert_close

pytestmark = pytest.mark.gpu


def _alone(r):
    """The request run alone with SV_FUSE, which makes the plan the server
    uses."""
    h = sv.sv_create(r.n, r.dtype)
    try:
        sv.sv_run_circuit(h, r.gates, sv.SV_FUSE)
        return sv.sv_copy_out(h)
    finally:
        sv.sv_destroy(h)


@pytest.mark.parametrize("persist,solo", [(0, 2048), (1, 8)], ids=["default", "three-streams"])
def test_each_result_is_the_same_alone_and_in_the_mix(persist, solo):
    """Also with each step's batch split three ways: circuits of one tile per
    pass (n <= 12) in the persistent launch, of 8 tiles or more (n >= 15) pass
    by pass on the third stream, the rest in levels."""
    reqs = serving.poisson_requests(rate=400.0, count=24, seed=3, n_lo=10, n_hi=17,
                                    d_lo=5, d_hi=40)
    srv = serving.Server(chunk=3, keep_results=True, persist_tiles=persist, solo_tiles=solo)
    try:
        stats = srv.run(reqs)
    finally:
        srv.close()
    assert stats["requests"] == len(reqs)
    assert stats["steps"] > 1
    for r in reqs:
        assert r.t_done >= r.t_admit >= 0 and r.latency > 0
        assert np.array_equal(r.result, _alone(r)), r.rid
        ref = oracle.simulate(r.n, r.gates)
        assert_close(r.result, ref, r.dtype, len(r.gates), f"served request {r.rid}")


def test_admission_respects_the_memory_budget():
    """A budget of two 2^16 complex128 states: requests queue for memory and
    all complete."""
    reqs = serving.poisson_requests(rate=1000.0, count=8, seed=5, n_lo=16, n_hi=16,
                                    d_lo=4, d_hi=8)
    budget = 2 * (1 << 16) * 16
    srv = serving.Server(budget_bytes=budget, chunk=2)
    peak = []
    orig = srv._admit

    def admit(r, now):
        orig(r, now)
        peak.append(srv.in_use)
    srv._admit = admit
    try:
        stats = srv.run(reqs)
    finally:
        srv.close()
    assert stats["requests"] == 8
    assert max(peak) <= budget
    assert all(abs(r.norm - 1.0) <= 1e-5 for r in reqs)
