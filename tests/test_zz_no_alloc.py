"""The allocation-free reduction (tslb_reduce_noalloc) against tslb_reduce.

Both launch the same two-pass FP64 reduction with the same number of
partial blocks, so the sums must agree bit for bit.  Two calls in a row on
different handles, the second on a smaller grid with 16-bit storage, show
that the shared scratch array carries nothing over from one call to the
next."""
import numpy as np
import pytest

import workloads as W
from helpers import gpu_solver, to_device_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2401_17074_amd  # noqa: F401
    torch.cuda.set_device(0)


def _check_against_reduce(s):
    import torch
    from paper_2401_17074_amd import capi as C
    want, rc = C.tslb_reduce(s.h)
    assert rc == C.TSLB_OK
    shear = C.tslb_objective(s.h, C.TSLB_OBJ_WALL_SHEAR)
    out = torch.full((C.TSLB_REDUCE_VALUES,), float("nan"), dtype=torch.float64, device="cuda")
    C.tslb_reduce_noalloc(s.h, out)
    got = out.cpu().numpy()
    print("noalloc reduce %s: %s" % (s.h, got.tolist()), flush=True)
    np.testing.assert_array_equal(got[:5], np.array(want))
    assert got[5] == 0.0
    assert got[6] == shear


def test_noalloc_reduce_matches_reduce_twice():
    big = W.channel_case(nx=96, ny=34, nz=40, re_tau=20)
    small = W.channel_case(nx=24, ny=10, nz=12, re_tau=10)
    s1 = gpu_solver(big, storage=0)
    s1.set_state(to_device_state(W.channel_state(big)))
    s1.step(3)
    s2 = gpu_solver(small, storage=1)
    s2.set_state(to_device_state(W.channel_state(small)))
    s2.step(2)
    try:
        _check_against_reduce(s1)
        _check_against_reduce(s2)
        # and back: the larger grid again after the smaller one
        _check_against_reduce(s1)
    finally:
        s1.close()
        s2.close()
