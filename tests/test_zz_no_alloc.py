"""GPU: sv_sample_device_noalloc, the sampling entry point that allocates
nothing (its scratch is a static device array), against sv_sample_device.

Both run the same kernels on the same state; the draws are integers, so they
must agree bit for bit. Two calls in a row go through the static array, the
second on a smaller state with fewer draws, so it must not depend on what the
first left there. States above the array's 30-qubit limit are rejected before
anything is queued.
"""
import numpy as np
import pytest

import oracle
import paper_1801_01037_amd as sv
import qcircuits as qc
from tests.gpu_helpers import rounded, state_from_host

pytestmark = pytest.mark.gpu


def _draws(fn, h, u):
    import torch
    ud = torch.as_tensor(np.ascontiguousarray(u, dtype=np.float64)).cuda()
    out = torch.full((len(u),), -1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    fn(h, ud.data_ptr(), len(u), out.data_ptr())
    sv.sv_synchronize(h)
    return out.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("dtype", [sv.SV_C128, sv.SV_C64], ids=["c128", "c64"])
def test_noalloc_draws_equal_the_allocating_call(dtype):
    # (n, draws): the second call is smaller in both
    for n, m, seed in ((22, 200000, 1), (13, 3000, 2)):
        psi = rounded(qc.random_state(n, 40 + n), dtype)
        u = qc.sorted_uniforms(seed, m)
        h = state_from_host(n, dtype, psi)
        try:
            want = _draws(sv.sv_sample_device, h, u)
            got = _draws(sv.sv_sample_device_noalloc, h, u)
        finally:
            sv.sv_destroy(h)
        print(f"n={n} draws={m}: {int(np.sum(got != want))} differ", flush=True)
        assert np.array_equal(got, want), f"n={n}"
        # and they are the oracle's draws up to CDF rounding
        ref = oracle.sample_indices(psi, u)
        assert np.mean(got == ref) > 0.999


def test_noalloc_in_a_fresh_handle_after_a_larger_state():
    """A basis state after a random one: every draw must give its index, so
    nothing of the earlier call's block sums may leak into this one."""
    u = qc.sorted_uniforms(9, 10000)
    psi = qc.random_state(20, 3)
    h = state_from_host(20, sv.SV_C128, psi)
    try:
        _draws(sv.sv_sample_device_noalloc, h, u)
    finally:
        sv.sv_destroy(h)
    for n, x in ((16, 40000), (5, 17)):
        h = sv.sv_create(n, sv.SV_C64)
        try:
            sv.sv_reset(h, x)
            assert (_draws(sv.sv_sample_device_noalloc, h, u) == x).all(), (n, x)
        finally:
            sv.sv_destroy(h)


def test_noalloc_rejects_states_above_its_limit():
    import torch
    n = 31
    t = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    h = sv.sv_wrap(t.data_ptr(), n, sv.SV_C64)
    try:
        ud = torch.zeros(4, dtype=torch.float64, device="cuda")
        out = torch.zeros(4, dtype=torch.int64, device="cuda")
        with pytest.raises(sv.SVError) as e:
            sv.sv_sample_device_noalloc(h, ud.data_ptr(), 4, out.data_ptr())
        assert e.value.status == sv.SV_EINVAL
        assert "30 qubits" in str(e.value)
        assert (out == 0).all().item()
    finally:
        sv.sv_destroy(h)
    del t
    torch.cuda.empty_cache()
