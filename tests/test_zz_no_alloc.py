"""dh_conservation_noalloc (the entry point for callers that cannot allocate) against
dh_conservation on the same states, through the C ABI: two calls in a row, the second on a
smaller grid, and a two-sample batch; results equal bit for bit (same kernels and summation
order)."""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dhp():
    import paper_2502_02294_amd as dhp
    return dhp


def _state(dhp, n, seed, batch=1):
    s = dhp.Sim(dhp.default_config(n=n, box=10.0 * n / 64, a_init=0.05, subgrid=2, batch=batch))
    s.init_from_seed(seed)
    s.run_steps(2)
    return s


def test_noalloc_sums_equal_the_handle_sums_on_two_calls(dhp):
    m_dm = 1.0 - 0.05 / 0.3
    for n, seed in ((64, 3), (32, 4)):
        s = _state(dhp, n, seed)
        q, mom = s.get("q"), s.get("mom")
        out = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
        dhp.conservation_noalloc(q, mom, n, m_dm, out)
        got = out.cpu().numpy()
        ref = np.array(s.conservation())
        print(f"n={n}: {got}")
        assert np.array_equal(got, ref), (n, got, ref)
        s.close()


def test_noalloc_batch_and_limits(dhp):
    from paper_2502_02294_amd import _lib
    n, m_dm = 32, 1.0 - 0.05 / 0.3
    s = _state(dhp, n, 5, batch=2)
    q, mom = s.get("q"), s.get("mom")
    out = torch.zeros(16, dtype=torch.float64, device="cuda")
    dhp.conservation_noalloc(q, mom, n, m_dm, out, batch=2)
    assert np.array_equal(out.cpu().numpy().reshape(2, 8), np.array(s.conservation()))
    s.close()
    # beyond the scratch limit: a host-side error before any launch
    import ctypes
    rc = _lib.lib().dh_conservation_noalloc(ctypes.c_void_p(q.data_ptr()),
                                            ctypes.c_void_p(mom.data_ptr()), 512, 1, m_dm,
                                            ctypes.c_void_p(out.data_ptr()), None)
    assert rc == -1
    assert "scratch limit" in _lib.lib().dh_last_error(None).decode()
