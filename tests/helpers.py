"""Shared test plumbing: build matching oracle grids and GPU solvers for a
workloads.Case, move states between them, and measure errors.

Parameters reach the GPU as binary32, so the oracle is given the same
binary32-rounded tau, force and inlet values (the comparison is then about
the arithmetic, not about parameter rounding)."""
import numpy as np

import oracle

F32 = np.float32


def f32(x):
    return float(F32(x))


def _tau_z32(case):
    import workloads as W
    prof = W.tau_profile(case)
    return None if prof is None else [f32(v) for v in prof]


def oracle_grid(case):
    return oracle.make_grid(case.nx, case.ny, case.nz, f32(case.tau), faces=case.faces,
                            force=[f32(v) for v in case.force], inlet_u=[f32(v) for v in case.inlet_u],
                            inlet_center=[f32(v) for v in case.inlet_center], inlet_radius=f32(case.inlet_radius),
                            inlet_noise=_amp_ratio(case), seed=case.seed, order=case.order,
                            noise_kind=case.noise_kind, tau_z=_tau_z32(case), lattice=case.lattice)


def _amp_ratio(case):
    """The library forms amp = noise * |u| in double from binary32 inputs and
    rounds it to binary32; give the oracle a noise value that reproduces the
    same amp exactly."""
    u = np.array([f32(v) for v in case.inlet_u])
    mag = float(np.sqrt((u * u).sum()))
    if mag == 0.0:
        return 0.0
    amp32 = f32(f32(case.inlet_noise) * mag)
    return amp32 / mag


def gpu_solver(case, storage=0, kernel=None, scale=(0.0, 0.0, 0.0)):
    from paper_2401_17074_amd import Solver
    s = Solver(case.nx, case.ny, case.nz, f32(case.tau), force=[f32(v) for v in case.force], faces=case.faces,
               storage=storage, scale=scale, inlet_u=case.inlet_u, inlet_center=case.inlet_center,
               inlet_radius=case.inlet_radius, inlet_noise=case.inlet_noise, seed=case.seed, kernel=kernel,
               order=case.order, inlet_noise_kind=case.noise_kind, lattice=case.lattice)
    tz = _tau_z32(case)
    if tz is not None:
        s.set_relaxation_profile(tz)
    return s


def to_device_state(st64):
    """float64 (rho, u, Pi) -> float32 (rho - 1, u, Pi) as the solver stores it."""
    dev = np.empty(st64.shape, dtype=np.float32)
    dev[0] = (st64[0] - 1.0).astype(np.float32)
    dev[1:] = st64[1:].astype(np.float32)
    return dev


def from_device_state(t):
    st = t.double().cpu().numpy()
    st[0] += 1.0
    return st


def rel_err(got, want, mask=None):
    """max |got - want| / max |want| over the masked nodes (normwise relative)."""
    if mask is not None:
        got = got[..., mask]
        want = want[..., mask]
    den = np.abs(want).max()
    return float(np.abs(got - want).max() / (den if den > 0 else 1.0))


def abs_err(got, want, mask=None):
    if mask is not None:
        got = got[..., mask]
        want = want[..., mask]
    return float(np.abs(got - want).max())
