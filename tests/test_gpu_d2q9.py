"""GPU parity of the D2Q9 update (the two-dimensional counterpart of
D3Q27, one wavefront-marching kernel) against the FP64 oracle, through the
C ABI, with the same bars as the D3Q27 parity tests."""
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
    return 32 * EPS32 * max(float(np.abs(want[1:3]).max()) ** 2, float(np.abs(want[[4, 5, 7]]).max()))


def _state2d(shape, seed, **kw):
    st = W.random_state(shape, seed=seed, **kw)
    st[[3, 6, 8, 9]] = 0.0
    return W.to_fp32(st)


CASES = [("periodic", (0, 0, 0, 0, 0, 0)), ("walls_y", (0, 0, 1, 1, 0, 0)), ("walls_xy", (1, 1, 1, 1, 0, 0)),
         ("ghosts_x", (3, 3, 0, 0, 0, 0))]


@pytest.mark.parametrize("order", [3, 2])
@pytest.mark.parametrize("name,faces", CASES)
def test_random_state_ragged_grid(name, faces, order):
    """A grid that spans several strips and row segments with ragged tails;
    random moments and force field; 1 step, then 9 more."""
    case = W.Case(name, 203, 131, 1, 0.57, faces=faces, order=order, lattice=9)
    st0 = _state2d(case.shape, 401)
    g = W.random_force(case.shape, seed=402, amp=1e-5).astype(np.float32).astype(np.float64)
    g[2] = 0.0
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
    assert rel_err(got1[1:3], want1[1:3], fl) < 2e-6
    assert abs_err(got1[[4, 5, 7]], want1[[4, 5, 7]], fl) < pi_tol(want1[:, fl])
    assert np.all(got1[[3, 6, 8, 9]] == 0.0)
    s.step(9)
    got = from_device_state(s.get_state())
    s.close()
    want = oracle.run(G, st0, 10, g)
    assert rel_err(got[1:3], want[1:3], fl) < 1e-5
    assert abs_err(got[0], want[0], fl) < 1e-6


def test_taylor_green_2d_100_steps():
    """The 2D Taylor-Green vortex on 64^2 (tau = 0.8, u0 = 0.01): 100 steps
    against the oracle within 1e-5 (normwise relative)."""
    n = 64
    case = W.Case("tgv2d", n, n, 1, 0.8, lattice=9)
    st0 = W.to_fp32(W.tgv_state(n, 0.01)[:, :1])
    G = oracle_grid(case)
    want = oracle.run(G, st0, 100)
    s = gpu_solver(case)
    s.set_state(to_device_state(st0))
    s.step(100)
    got = from_device_state(s.get_state())
    s.close()
    assert rel_err(got[1:3], want[1:3]) <= 1e-5
    assert rel_err(got[0], want[0]) <= 1e-5


def test_channel_2d_full_size_sampled():
    """The 8192 x 4096 2D channel (walls at y = 0, ny - 1) of the benchmark,
    in the launch it times: 20 steps, then one step checked at sampled nodes,
    and FP64 mass conservation."""
    case = W.channel2d_case()
    st0 = W.to_fp32(W.channel2d_state(case))
    G = oracle_grid(case)
    kinds = oracle.node_kinds(G)
    s = gpu_solver(case)
    s.set_state(to_device_state(st0))
    r0, _ = s.reduce()
    s.step(20)
    pre = from_device_state(s.get_state())
    s.step(1)
    post = from_device_state(s.get_state())
    r1, _ = s.reduce()
    s.close()
    idx = W.sample_nodes(case, 4000, 10, fluid_mask=(kinds == 0))
    want = oracle.update_nodes(G, pre, idx)
    got = post.reshape(10, -1)[:, idx]
    assert np.abs(got[0] - want[0]).max() < 1e-7
    assert np.abs(got[1:3] - want[1:3]).max() < 2e-6 * np.abs(want[1:3]).max()
    assert np.abs(got[[4, 5, 7]] - want[[4, 5, 7]]).max() < pi_tol(want)
    assert abs(r1[0] - r0[0]) < 1e-6 * r0[0]


def test_d2q9_argument_checks():
    from paper_2401_17074_amd import Solver, TslbError
    with pytest.raises(TslbError):
        Solver(16, 16, 2, 0.7, lattice=9)                   # nz must be 1
    with pytest.raises(TslbError):
        Solver(16, 16, 1, 0.7, force=(0, 0, 1e-6), lattice=9)  # no z force
    s = Solver(16, 16, 1, 0.7, lattice=9)
    with pytest.raises(TslbError):
        s.set_kernel(1)
    import torch
    raw = s.save_raw()
    lam = torch.zeros((10, 1, 16, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(TslbError):
        s.adjoint_step(raw, raw, lam)
    s.close()
