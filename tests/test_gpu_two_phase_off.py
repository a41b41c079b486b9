"""The two-phase device path is switched off: evp_set_two_phase with parameters returns
EVP_ERR_DISABLED, launches nothing and leaves the grid a single-phase one that steps bit for bit
like a grid it was never called on."""
import numpy as np
import pytest

from paper_1803_09563_amd import inputs

from harness import gpu_grid, gpu_state, to_dev
from test_gpu_parity import _wl

pytestmark = pytest.mark.gpu

EVP_ERR_DISABLED = -6


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1803_09563_amd  # noqa: F401  (fails loudly without libevp.so)
    yield


def test_set_two_phase_is_disabled_and_changes_nothing():
    import paper_1803_09563_amd as evp
    wl = _wl(32, 24, 16, False, "oldroyd_b")
    fields = inputs.random_state(wl.shape, 81, amp_u=0.1)
    a, b = gpu_grid(wl), gpu_grid(wl)
    with pytest.raises(evp.EvpError) as e:
        a.set_two_phase(rho1=1.0, rho2=0.5, mu_s1=0.02, mu_s2=0.05, mu_p1=0.03, mu_p2=0.01,
                        lam1=0.5, lam2=0.8, sigma=0.05)
    assert e.value.status == EVP_ERR_DISABLED
    a.set_two_phase(None)        # switching back to a single phase is still accepted
    for G in (a, b):
        G.write_fields(*to_dev(*fields))
        G.step(1e-3, 5)
    sa, sb = gpu_state(a), gpu_state(b)
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k
