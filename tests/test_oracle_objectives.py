"""Closed-form pins of the oracle's objective values and of the outlet sponge.

- The kinetic energy L = 1/2 sum over fluid nodes of rho |u|^2 (the loss of
  the differentiable workload; the conservation sums of Section 2) is
  checked, as returned by both oracle entry points that form it (the FP64
  reductions and the adjoint seed), against values fixed by the fields
  alone: a uniform flow gives 1/2 rho0 |u0|^2 times the number of fluid
  nodes, and the discrete Taylor-Green vortex at t = 0 gives n^3 u0^2 / 4
  exactly, since sin^2 and cos^2 each sum to n/2 over a full period of n
  nodes.  A wrong 1/2, a missing rho, or wall and ghost nodes counted as
  fluid all fail one of them.
- The sponge of the jet of Section 3.2 (the garbled formula's reading: the
  viscosity rises as nu (1 + K xi^3) over the last w planes) is checked at
  the three points the reading fixes: nu at the sponge start, nu (1 + K/8)
  half-way, (K + 1) nu at the outflow layer.
"""
import numpy as np
import pytest

import workloads as W

PERIODIC, WALL, INLET, OUTLET = 0, 1, 2, 3


def _uniform(shape, rho0, u0):
    st = np.zeros((10,) + tuple(shape))
    st[0] = rho0
    for a in range(3):
        st[1 + a] = u0[a]
    return st


FACES = {
    "periodic": ((PERIODIC,) * 6, lambda nx, ny, nz: nx * ny * nz),
    "y_walls": ((PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC), lambda nx, ny, nz: nx * (ny - 2) * nz),
    "xz_walls": ((WALL, WALL, PERIODIC, PERIODIC, WALL, WALL), lambda nx, ny, nz: (nx - 2) * ny * (nz - 2)),
    "outlets": ((OUTLET,) * 6, lambda nx, ny, nz: (nx - 2) * (ny - 2) * (nz - 2)),
    "walls_and_outlets": ((OUTLET, OUTLET, WALL, WALL, PERIODIC, PERIODIC),
                          lambda nx, ny, nz: (nx - 2) * (ny - 2) * nz),
}


@pytest.mark.parametrize("kind", sorted(FACES))
def test_kinetic_energy_of_uniform_flow(oracle, kind):
    faces, fluid = FACES[kind]
    nx, ny, nz = 7, 6, 5
    rho0, u0 = 1.0372, (0.031, -0.017, 0.0045)
    G = oracle.make_grid(nx, ny, nz, 0.8, faces=faces)
    st = _uniform(G.shape, rho0, u0)
    nf = fluid(nx, ny, nz)
    u2 = sum(v * v for v in u0)
    want = 0.5 * rho0 * u2 * nf
    sums, bad = oracle.reduce(G, st)
    assert bad == 0
    assert sums[4] == pytest.approx(want, rel=1e-14)
    assert sums[0] == pytest.approx(rho0 * nf, rel=1e-14)
    for a in range(3):
        assert sums[1 + a] == pytest.approx(rho0 * u0[a] * nf, rel=1e-14)
    L, lam = oracle.ke_seed(G, st)
    assert L == pytest.approx(want, rel=1e-14)
    # dL/dM: |u|^2 / 2 on rho, rho u on u, nothing on Pi; zero off the fluid
    fl = oracle.node_kinds(G) == 0
    assert fl.sum() == nf
    assert np.allclose(lam[0][fl], 0.5 * u2, rtol=1e-14, atol=0)
    for a in range(3):
        assert np.allclose(lam[1 + a][fl], rho0 * u0[a], rtol=1e-14, atol=0)
    assert not lam[4:].any()
    assert not lam[:, ~fl].any()


def test_kinetic_energy_of_taylor_green_start(oracle):
    n, u0 = 32, 0.01
    case = W.tgv_case(n=n, u0=u0)
    st = W.tgv_state(n, u0)
    G = oracle.make_grid(n, n, n, case.tau)
    want = n ** 3 * u0 * u0 / 4.0
    sums, bad = oracle.reduce(G, st)
    assert bad == 0
    assert sums[4] == pytest.approx(want, rel=1e-13)
    assert sums[0] == pytest.approx(float(n ** 3), rel=1e-15)
    assert np.abs(sums[1:4]).max() < 1e-15 * n ** 3
    L, _ = oracle.ke_seed(G, st)
    assert L == pytest.approx(want, rel=1e-13)


def test_kinetic_energy_weights_rho(oracle):
    """A density field varying in space with a uniform velocity: L is
    1/2 |u|^2 times the total mass, whatever the density pattern."""
    nx, ny, nz = 8, 5, 6
    G = oracle.make_grid(nx, ny, nz, 0.9)
    st = _uniform(G.shape, 1.0, (0.02, 0.01, -0.03))
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    st[0] = 1.0 + 0.1 * ((x + 2 * y + 3 * z) % 4)
    u2 = 0.02 ** 2 + 0.01 ** 2 + 0.03 ** 2
    sums, _ = oracle.reduce(G, st)
    assert sums[4] == pytest.approx(0.5 * u2 * st[0].sum(), rel=1e-14)
    L, _ = oracle.ke_seed(G, st)
    assert L == pytest.approx(0.5 * u2 * st[0].sum(), rel=1e-14)


def test_sponge_profile_reading():
    case = W.paper_jet_case()
    K, power, width = case.sponge
    assert (K, power, width) == (1000.0, 3.0, 50)
    tau = W.tau_profile(case)
    assert tau.shape == (case.nz,)
    nu0 = (case.tau - 0.5) / 3.0
    nu = (tau - 0.5) / 3.0
    zs = case.nz - 1 - width
    # untouched up to the sponge start
    assert np.allclose(nu[: zs + 1], nu0, rtol=1e-14, atol=0)
    # half-way: xi = 1/2, nu (1 + K / 8)
    assert nu[zs + width // 2] == pytest.approx(nu0 * (1.0 + K / 8.0), rel=1e-12)
    # the outflow layer: (K + 1) nu
    assert nu[case.nz - 1] == pytest.approx((K + 1.0) * nu0, rel=1e-12)
    # smooth and monotone in between
    assert np.all(np.diff(nu) >= 0)
    assert np.all(tau > 0.5)


def test_no_sponge_without_a_sponge_case():
    assert W.tau_profile(W.jet_case(nx=16, ny=12, nz=10)) is None
