"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the lattice Boltzmann method: it only
builds initial moment fields, force fields and case parameters, in float64
numpy arrays (one generator draws on the GPU, for grids too large for the
host) of shape (10, nz, ny, nx) (rho, u_x, u_y, u_z, Pi^neq xx, yy, zz,
xy, xz, yz) or (3, nz, ny, nx) for a body-force field.  Both the HIP path and
the FP64 oracle consume what it returns; neither is imported here.

The cases stand in for the paper's workloads (Montessori et al.,
arXiv:2401.17074): the turbulent channel of Section 3.1 and the round jet of
Section 3.2 are replaced by seeded synthetic states of the same shape,
boundary kinds, relaxation time and forcing; no DNS or experimental data is
used or needed.
"""
from dataclasses import dataclass, field

import numpy as np

PERIODIC, WALL, INLET, OUTLET = 0, 1, 2, 3


@dataclass
class Case:
    """Geometry, relaxation time, forcing and boundary kinds of one workload."""
    name: str
    nx: int
    ny: int
    nz: int
    tau: float
    faces: tuple = (PERIODIC,) * 6
    force: tuple = (0.0, 0.0, 0.0)
    inlet_u: tuple = (0.0, 0.0, 0.0)
    inlet_center: tuple = (0.0, 0.0)
    inlet_radius: float = 0.0
    inlet_noise: float = 0.0
    seed: int = 0
    steps: int = 100
    order: int = 3  # Hermite order of the rebuilt populations (2: regularised collision)
    noise_kind: int = 0  # inlet perturbation: 0 uniform, 1 Gaussian
    sponge: tuple = ()  # (K, power, width) of an outlet sponge on the +z face, or ()
    lattice: int = 27  # 27 (D3Q27) or 9 (D2Q9, nz = 1)
    extra: dict = field(default_factory=dict)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def nodes(self):
        return self.nx * self.ny * self.nz


def _rng(seed):
    return np.random.default_rng(np.random.SeedSequence(seed))


def rest_state(shape):
    st = np.zeros((10,) + tuple(shape))
    st[0] = 1.0
    return st


# --------------------------------------------------------------------------
# Taylor-Green vortex, 32^3 periodic, tau = 0.8, u0 = 0.01: the z-invariant
# vortex u = u0 sin(kx) cos(ky), v = -u0 cos(kx) sin(ky), k = 2 pi / n, whose
# velocity decays as exp(-2 nu k^2 t) in the incompressible limit.
def tgv_case(n=32, tau=0.8, u0=0.01, steps=100):
    return Case("taylor_green_%d" % n, n, n, n, tau, steps=steps, extra={"u0": u0})


def tgv_state(n=32, u0=0.01):
    k = 2.0 * np.pi / n
    x = np.arange(n)
    X, Y = np.meshgrid(x, x, indexing="xy")  # X varies along the last (x) axis
    st = rest_state((n, n, n))
    st[1] = (u0 * np.sin(k * X) * np.cos(k * Y))[None]
    st[2] = (-u0 * np.cos(k * X) * np.sin(k * Y))[None]
    return st


# --------------------------------------------------------------------------
# Channel: walls are the node layers y = 0 and y = ny - 1 (solid), x and z
# periodic.  Friction Reynolds number 180 with tau = 0.5045 (nu = 0.0015):
# half-width h = (ny - 2) / 2, u_tau = Re_tau nu / h, g = u_tau^2 / h along x.
def channel_case(nx=384, ny=192, nz=192, re_tau=180.0, tau=0.5045, steps=1000, seed=1234, uc=None, lattice=27):
    nu = (tau - 0.5) / 3.0
    h = (ny - 2) / 2.0
    u_tau = re_tau * nu / h
    g = u_tau * u_tau / h
    if uc is None:
        uc = 20.0 * u_tau  # centreline of the initial parabola: a low-Mach stand-in
    name = "channel_%dx%dx%d" % (nx, ny, nz) + ("" if lattice == 27 else "_d3q%d" % lattice)
    return Case(name, nx, ny, nz, tau,
                faces=(PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC),
                force=(g, 0.0, 0.0), seed=seed, steps=steps, lattice=lattice,
                extra={"u_tau": u_tau, "h": h, "uc": uc, "perturb": 0.05})


def channel_state(case):
    """Parabolic streamwise profile vanishing on the half-way walls
    (y = 1/2 and y = ny - 3/2) with centreline case.extra['uc'], plus seeded
    uniform perturbations of +-5 % of the centreline speed per component."""
    nz, ny, nx = case.shape
    uc = case.extra["uc"]
    h = case.extra["h"]
    yc = (ny - 1) / 2.0
    y = np.arange(ny)
    prof = uc * np.clip(1.0 - ((y - yc) / h) ** 2, 0.0, None)
    st = rest_state(case.shape)
    st[1] = prof[None, :, None]
    rng = _rng(case.seed)
    amp = case.extra["perturb"] * uc
    st[1:4] += rng.uniform(-amp, amp, size=(3,) + case.shape)
    st[1:4, :, 0, :] = 0.0
    st[1:4, :, ny - 1, :] = 0.0
    return st


# --------------------------------------------------------------------------
# Round jet: inflow disc of diameter 20 on the x = 0 face, top-hat velocity
# 0.05 along +x with 2 % seeded perturbation, zero-gradient outflow on every
# other boundary node, Re = U D / nu = 7000 through tau = 0.5 + 3 U D / Re.
def jet_case(nx=512, ny=256, nz=256, U=0.05, D=20.0, re=7000.0, steps=2000, seed=4321, noise=0.02):
    tau = 0.5 + 3.0 * U * D / re
    return Case("jet_%dx%dx%d" % (nx, ny, nz), nx, ny, nz, tau,
                faces=(INLET, OUTLET, OUTLET, OUTLET, OUTLET, OUTLET),
                inlet_u=(U, 0.0, 0.0), inlet_center=((ny - 1) / 2.0, (nz - 1) / 2.0),
                inlet_radius=D / 2.0, inlet_noise=noise, seed=seed, steps=steps)


def jet_state(case):
    return rest_state(case.shape)


# --------------------------------------------------------------------------
# The jet as the paper sets it up (Section 3.2): 440 x 440 x 600, inlet disc
# D = 20 centred on the z = 0 face with U = 0.05 along z and time-varying
# Gaussian noise, periodic crossflow faces, outflow at the top, and a sponge
# of the last 50 planes where nu grows as nu (1 + K xi^3), K = 1000.
def paper_jet_case(nx=440, ny=440, nz=600, U=0.05, D=20.0, re=7000.0, steps=2000, seed=4321, noise=0.02,
                   sponge=(1000.0, 3.0, 50)):
    tau = 0.5 + 3.0 * U * D / re
    return Case("paper_jet_%dx%dx%d" % (nx, ny, nz), nx, ny, nz, tau,
                faces=(PERIODIC, PERIODIC, PERIODIC, PERIODIC, INLET, OUTLET),
                inlet_u=(0.0, 0.0, U), inlet_center=((nx - 1) / 2.0, (ny - 1) / 2.0),
                inlet_radius=D / 2.0, inlet_noise=noise, seed=seed, steps=steps, noise_kind=1, sponge=sponge)


# --------------------------------------------------------------------------
# Two-dimensional channel for the D2Q9 lattice: 8192 x 4096 nodes (nz = 1),
# walls at y = 0 and y = ny - 1, x periodic; the laminar parabola of
# centreline 0.05 plus seeded uniform 5 % perturbations; the body force of
# that Poiseuille profile.
def channel2d_case(nx=8192, ny=4096, tau=0.5045, uc=0.05, seed=5678):
    nu = (tau - 0.5) / 3.0
    h = (ny - 2) / 2.0
    g = 2.0 * nu * uc / (h * h)
    return Case("channel2d_%dx%d" % (nx, ny), nx, ny, 1, tau, faces=(PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC),
                force=(g, 0.0, 0.0), seed=seed, lattice=9, extra={"h": h, "uc": uc})


def channel2d_state(case):
    h, uc = case.extra["h"], case.extra["uc"]
    y = np.arange(case.ny) - 0.5  # walls half-way between the solid and first fluid layers
    prof = np.clip(uc * (1.0 - ((y - h) / h) ** 2), 0.0, None)
    st = rest_state(case.shape)
    noise = _rng(case.seed).uniform(-1.0, 1.0, size=(case.ny, case.nx))
    st[1, 0] = prof[:, None] * (1.0 + 0.05 * noise)
    st[:, 0, 0, :] = rest_state((1,))[:, 0:1]
    st[:, 0, -1, :] = rest_state((1,))[:, 0:1]
    return st


def tau_profile(case):
    """Relaxation time of each z plane for a case with an outlet sponge, else
    None.  With nu = (tau - 1/2)/3, the planes z >= z_s = nz - 1 - width get
    nu_s = nu (1 + K xi^p), xi = (z - z_s) / width in [0, 1]."""
    if not case.sponge:
        return None
    K, pw, width = case.sponge
    nu = (case.tau - 0.5) / 3.0
    z = np.arange(case.nz, dtype=np.float64)
    zs = case.nz - 1 - width
    xi = np.clip((z - zs) / width, 0.0, 1.0)
    return 0.5 + 3.0 * nu * (1.0 + K * xi ** pw)


# --------------------------------------------------------------------------
# Differentiable case: 64^3 periodic, body-force field with seeded Gaussian
# components of standard deviation 1e-6, initial Taylor-Green velocity
# (u0 = 0.01) plus seeded Gaussian noise of 1e-3, tau = 0.8.
def adjoint_case(n=64, tau=0.8, steps=400, ckpt=20, seed=777, g_amp=1e-6, u_noise=1e-3):
    return Case("forced_periodic_%d" % n, n, n, n, tau, seed=seed, steps=steps,
                extra={"ckpt": ckpt, "g_amp": g_amp, "u_noise": u_noise})


def adjoint_inputs(case):
    n = case.nx
    rng = _rng(case.seed)
    g = rng.normal(0.0, case.extra["g_amp"], size=(3,) + case.shape)
    st = tgv_state(n, 0.01)
    st[1:4] += rng.normal(0.0, case.extra["u_noise"], size=(3,) + case.shape)
    return st, g


# --------------------------------------------------------------------------
# Generic seeded random states for parity tests: rho near 1, low-Mach
# velocity and small non-equilibrium stress, on any grid.
def random_state(shape, seed, u_amp=0.03, rho_amp=0.01, pi_amp=1e-3):
    rng = _rng(seed)
    st = np.empty((10,) + tuple(shape))
    st[0] = 1.0 + rng.uniform(-rho_amp, rho_amp, size=shape)
    st[1:4] = rng.uniform(-u_amp, u_amp, size=(3,) + tuple(shape))
    st[4:10] = rng.uniform(-pi_amp, pi_amp, size=(6,) + tuple(shape))
    return st


def random_state_device(shape, seed, u_amp=0.03, rho_amp=0.01, pi_amp=1e-3):
    """The same distributions as random_state, drawn on the current GPU with a
    seeded torch generator, as float32 (rho - 1, u, Pi): for grids whose
    state is too large to build on the host."""
    import torch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    st = torch.empty((10,) + tuple(shape), dtype=torch.float32, device="cuda")
    st[0].uniform_(-rho_amp, rho_amp, generator=gen)
    st[1:4].uniform_(-u_amp, u_amp, generator=gen)
    st[4:10].uniform_(-pi_amp, pi_amp, generator=gen)
    return st


def random_force(shape, seed, amp=1e-5):
    return _rng(seed).uniform(-amp, amp, size=(3,) + tuple(shape))


def sample_nodes(case, count, seed, fluid_mask=None):
    """Seeded sample of node indices (x fastest) from the fluid mask."""
    rng = _rng(seed)
    if fluid_mask is None:
        return np.sort(rng.choice(case.nodes, size=min(count, case.nodes), replace=False))
    idx = np.flatnonzero(fluid_mask.reshape(-1))
    return np.sort(rng.choice(idx, size=min(count, idx.size), replace=False))


def to_fp32(st):
    """Round a float64 state to what binary32 storage holds (rho stored as rho - 1)."""
    out = st.astype(np.float32).astype(np.float64)
    out[0] = 1.0 + (st[0] - 1.0).astype(np.float32).astype(np.float64)
    return out


def gradient_directions(case, seed, count=2):
    """Seeded probe directions for directional-derivative checks of the
    differentiable case: `count` standard-normal fields of shape
    (3, nz, ny, nx), one list for the force field and one for the initial
    velocity."""
    rng = _rng(seed)
    shape = (3,) + case.shape
    dg = [rng.standard_normal(shape) for _ in range(count)]
    du = [rng.standard_normal(shape) for _ in range(count)]
    return dg, du


def precision_subcase():
    """64^3 channel subcase of the precision workload (h = 31, tau = 0.5045)
    with the body force set for a laminar centreline velocity of 0.05:
    g = 2 nu U_c / h^2 along x, nu = (tau - 1/2) / 3."""
    case = channel_case(nx=64, ny=64, nz=64, tau=0.5045)
    nu = (case.tau - 0.5) / 3
    h = case.extra["h"]
    case.name = "channel_64_laminar"
    case.force = (0.05 * 2 * nu / h ** 2, 0.0, 0.0)
    case.extra["uc"] = 0.05
    return case
