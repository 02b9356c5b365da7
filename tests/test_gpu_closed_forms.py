"""Closed forms checked on the GPU path itself (not only through the
oracle): the laminar Poiseuille profile between half-way walls and the
decay of a linear shear wave, both exact for this scheme's linear
dynamics, and the Taylor-Green decay rate 2 nu k^2 (the same closed forms
pin the oracle)."""
import numpy as np
import pytest

import workloads as W
from helpers import from_device_state, gpu_solver, to_device_state

pytestmark = pytest.mark.gpu
CS2 = 1.0 / 3.0


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2401_17074_amd  # noqa: F401
    torch.cuda.set_device(0)


# (kernel variant, lattice): the three D3Q27 variants, D3Q19 and D2Q9
VARIANTS = [(0, 27), (1, 27), (2, 27), (0, 19), (0, 9)]


@pytest.mark.parametrize("kernel,lattice", VARIANTS)
@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_poiseuille_steady_state(kernel, lattice, tau):
    """Forced flow between the walls y = 1/2 and y = ny - 3/2 from rest to
    its steady state: u(y) = g/(2 nu) [(y - 1/2)(ny - 3/2 - y) - 1/4] + g/2
    and Pi_xy = -cs2 tau du/dy at the bulk nodes (the same profile on the
    three lattices, whose y-marginal is the same three-point set)."""
    nx, ny, g = 64, 18, 1e-6
    nz = 1 if lattice == 9 else 4
    case = W.Case("poiseuille", nx, ny, nz, tau, faces=(0, 0, 1, 1, 0, 0), force=(g, 0.0, 0.0), lattice=lattice)
    nu = CS2 * (float(np.float32(tau)) - 0.5)
    # slowest mode decays as exp(-nu (pi / (ny - 2))^2 t): 5000 steps leave < 1e-8 of it
    s = gpu_solver(case, kernel=kernel)
    s.set_state(to_device_state(W.rest_state(case.shape)))
    s.step(5000)
    st = from_device_state(s.get_state())
    s.close()
    y = np.arange(1, ny - 1)
    ua = g / (2 * nu) * ((y - 0.5) * (ny - 1.5 - y) - 0.25) + g / 2
    u = st[1][:, 1:-1, :]
    assert np.abs(u - ua[None, :, None]).max() < 1e-4 * ua.max()
    assert np.abs(st[2:4][:, :, 1:-1, :]).max() < 1e-6 * ua.max()
    dudy = (st[1][:, 3:-1, :] - st[1][:, 1:-3, :]) / 2
    pxy = st[7][:, 2:-2, :]
    assert np.abs(pxy + CS2 * float(np.float32(tau)) * dudy).max() < 1e-3 * np.abs(pxy).max()


@pytest.mark.parametrize("kernel,lattice", VARIANTS)
@pytest.mark.parametrize("order", [3, 2])
def test_shear_wave_decay(kernel, lattice, order):
    """u_x = A sin(k y) with its eigen-stress Pi_xy = s A cos(k y) decays by
    the dominant eigenvalue of the one-step map per step (the linear mode
    reaches no third-order term, so both orders share it, and the three
    lattices share the map)."""
    nx, ny, tau, A, steps = 64, 64, 0.8, 1e-3, 50
    nz = 1 if lattice == 9 else 4
    tau32 = float(np.float32(tau))
    om = 1.0 / tau32
    k = 2 * np.pi / ny
    T = (2 + np.cos(k)) / 3 + (1 - om) * np.cos(k)
    D = (1 - om) * (1 + 2 * np.cos(k)) / 3
    lam = (T + np.sqrt(T * T - 4 * D)) / 2
    sc = -(np.sin(k) / 3) / (lam - (1 - om) * np.cos(k))
    case = W.Case("shear", nx, ny, nz, tau, order=order, lattice=lattice)
    st0 = W.rest_state(case.shape)
    yy = np.arange(ny)[None, :, None]
    st0[1] = A * np.sin(k * yy) + 0 * st0[1]
    st0[7] = sc * A * np.cos(k * yy) + 0 * st0[7]
    st0 = W.to_fp32(st0)
    s = gpu_solver(case, kernel=kernel)
    s.set_state(to_device_state(st0))
    s.step(steps)
    st = from_device_state(s.get_state())
    s.close()
    mode = np.sin(k * yy) + 0 * st[1]
    amp = (st[1] * mode).sum() / (mode * mode).sum()
    amp0 = (st0[1] * mode).sum() / (mode * mode).sum()
    assert amp / amp0 == pytest.approx(lam ** steps, rel=2e-5)


@pytest.mark.parametrize("kernel,lattice", VARIANTS)
def test_taylor_green_decay_rate(kernel, lattice):
    """The z-invariant Taylor-Green vortex (32^3, tau = 0.8, u0 = 0.01) decays
    as exp(-2 nu k^2 t): the rate fitted over t in [20, 100] on the GPU path
    is within 1e-3 of 2 nu k^2 (the initial Pi = 0 transient is over by
    t = 20)."""
    import torch
    n, tau, u0 = 32, 0.8, 0.01
    nz = 1 if lattice == 9 else n
    case = W.Case("tgv", n, n, nz, tau, lattice=lattice)
    st0 = W.rest_state(case.shape)
    st0[1:3] = W.tgv_state(n, u0)[1:3, :nz]
    st0 = W.to_fp32(st0)
    mode = st0[1]
    s = gpu_solver(case, kernel=kernel)
    s.set_state(to_device_state(st0))
    s.step(20)
    ts, amps = [], []
    for t in range(20, 101, 20):
        if t > 20:
            s.step(20)
        st = from_device_state(s.get_state())
        ts.append(t)
        amps.append((st[1] * mode).sum() / (mode * mode).sum())
    s.close()
    torch.cuda.synchronize()
    rate = -np.polyfit(ts, np.log(amps), 1)[0]
    nu = CS2 * (float(np.float32(tau)) - 0.5)
    k = 2 * np.pi / n
    assert rate / (2 * nu * k * k) == pytest.approx(1.0, abs=1e-3)
