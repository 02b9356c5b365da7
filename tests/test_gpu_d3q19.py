"""GPU parity of the D3Q19 update (the tiled kernel with the D3Q19 weights
and the restricted third-order reconstruction) against the FP64 oracle,
through the C ABI, with the same bars as the D3Q27 parity tests."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import abs_err, from_device_state, gpu_solver, oracle_grid, rel_err, to_device_state

pytestmark = pytest.mark.gpu
EPS32 = float(np.finfo(np.float32).eps)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2401_17074_amd  # noqa: F401
    torch.cuda.set_device(0)


def pi_tol(want):
    return 32 * EPS32 * max(float(np.abs(want[1:4]).max()) ** 2, float(np.abs(want[4:]).max()))


CASES = [("periodic", (0, 0, 0, 0, 0, 0)), ("walls_y", (0, 0, 1, 1, 0, 0)), ("walls_xz", (1, 1, 0, 0, 1, 1)),
         ("ghosts", (3, 3, 3, 3, 3, 3))]


@pytest.mark.parametrize("order", [3, 2])
@pytest.mark.parametrize("name,faces", CASES)
def test_random_state_ragged_grid(name, faces, order):
    case = W.Case(name, 71, 37, 23, 0.57, faces=faces, order=order, lattice=19)
    st0 = W.to_fp32(W.random_state(case.shape, seed=501))
    g = W.random_force(case.shape, seed=502, amp=1e-5).astype(np.float32).astype(np.float64)
    G = oracle_grid(case)
    st0 = oracle.ghost_fill(G, st0, 0)
    kinds = oracle.node_kinds(G)
    fl = kinds == 0
    s = gpu_solver(case)
    s.set_force_field(g)
    s.set_state(to_device_state(st0))
    s.step(1)
    got1 = from_device_state(s.get_state())
    want1 = oracle.step(G, st0, g)
    assert abs_err(got1[0], want1[0], fl) < 1e-7
    assert rel_err(got1[1:4], want1[1:4], fl) < 2e-6
    assert abs_err(got1[4:], want1[4:], fl) < pi_tol(want1[:, fl])
    s.step(6)
    got = from_device_state(s.get_state())
    s.close()
    want = oracle.run(G, st0, 7, g)
    assert rel_err(got[1:4], want[1:4], fl) < 1e-5
    assert abs_err(got[0], want[0], fl) < 1e-6


def test_taylor_green_100_steps():
    case = W.tgv_case()
    case.lattice = 19
    st0 = W.to_fp32(W.tgv_state(case.nx, case.extra["u0"]))
    G = oracle_grid(case)
    want = oracle.run(G, st0, case.steps)
    s = gpu_solver(case)
    s.set_state(to_device_state(st0))
    s.step(case.steps)
    got = from_device_state(s.get_state())
    s.close()
    assert rel_err(got[1:4], want[1:4]) <= 1e-5 and rel_err(got[0], want[0]) <= 1e-5


def test_channel_full_size_sampled():
    """The 384x192x192 channel on D3Q19 in the benchmark launch: 20 steps,
    then one step checked at sampled fluid nodes."""
    case = W.channel_case()
    case.lattice = 19
    st0 = W.to_fp32(W.channel_state(case))
    s = gpu_solver(case)
    s.set_state(to_device_state(st0))
    s.step(20)
    pre = from_device_state(s.get_state())
    s.step(1)
    post = from_device_state(s.get_state())
    s.close()
    G = oracle_grid(case)
    kinds = oracle.node_kinds(G)
    idx = W.sample_nodes(case, 3000, 11, fluid_mask=(kinds == 0))
    want = oracle.update_nodes(G, pre, idx)
    got = post.reshape(10, -1)[:, idx]
    assert np.abs(got[0] - want[0]).max() < 1e-7
    assert np.abs(got[1:4] - want[1:4]).max() < 2e-6 * np.abs(want[1:4]).max()
    assert np.abs(got[4:] - want[4:]).max() < pi_tol(want)


def test_d3q19_argument_checks():
    import torch
    from paper_2401_17074_amd import Solver, TslbError
    s = Solver(16, 12, 10, 0.7, lattice=19)
    with pytest.raises(TslbError):
        s.set_kernel(1)
    raw = s.save_raw()
    lam = torch.zeros((10, 10, 12, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(TslbError):
        s.adjoint_step(raw, raw, lam)
    s.close()
