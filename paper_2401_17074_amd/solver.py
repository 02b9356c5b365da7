"""Object wrapper over the C ABI and the autograd bridge of the adjoint.

Marshalling only: tensors are allocated with torch on the solver's device and
passed by pointer; every number is produced by the library's kernels.
"""
import torch

from . import _binding as C


class Solver:
    """One TSLB solver handle (tslb_create) on the current CUDA/HIP device.

    State tensors exchanged by ``set_state`` / ``get_state`` are float32 of
    shape (10, nz, ny, nx): rho - 1, u_x, u_y, u_z, Pi^neq xx, yy, zz, xy, xz, yz
    (with lattice=TSLB_D2Q9, nz = 1 and the z components are zero).
    """

    def __init__(self, nx, ny, nz, tau, force=(0.0, 0.0, 0.0), faces=(C.TSLB_PERIODIC,) * 6,
                 storage=C.TSLB_FP32, scale=(0.0, 0.0, 0.0), inlet_u=(0.0, 0.0, 0.0), inlet_center=(0.0, 0.0),
                 inlet_radius=0.0, inlet_noise=0.0, seed=0, kernel=None, order=3, inlet_noise_kind=0,
                 lattice=C.TSLB_D3Q27):
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        self.device = torch.device("cuda", torch.cuda.current_device())
        bc = C.make_bc(faces=faces, inlet_u=inlet_u, inlet_center=inlet_center, inlet_radius=inlet_radius,
                       inlet_noise=inlet_noise, seed=seed, storage=storage, scale=scale, order=order,
                       inlet_noise_kind=inlet_noise_kind)
        self.h = C.tslb_create(nx, ny, nz, lattice, tau, force, bc)
        if kernel is not None:
            C.tslb_set_kernel(self.h, kernel)

    def close(self):
        if self.h is not None:
            C.tslb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bind_state_to_torch(self):
        """Move the two state buffers into tensors from PyTorch's allocator
        (kept on the Solver as `state_buffers`)."""
        nb = C.tslb_state_bytes(self.h)
        bufs = [torch.empty(nb, dtype=torch.uint8, device=self.device) for _ in range(2)]
        C.tslb_bind_state(self.h, bufs[0], bufs[1])
        self.state_buffers = bufs

    def set_kernel(self, variant):
        C.tslb_set_kernel(self.h, variant)

    def set_state(self, st):
        st = torch.as_tensor(st, dtype=torch.float32).to(self.device).contiguous()
        assert st.shape == (10,) + self.shape
        C.tslb_set_moments(self.h, st[0], st[1:4], st[4:10], C.TSLB_DEVICE | C.TSLB_RHO_DEVIATION)

    def get_state(self):
        st = torch.empty((10,) + self.shape, dtype=torch.float32, device=self.device)
        C.tslb_get_moments(self.h, st[0], st[1:4], st[4:10], C.TSLB_DEVICE | C.TSLB_RHO_DEVIATION)
        return st

    def set_force_field(self, g):
        if g is None:
            C.tslb_set_force_field(self.h, None)
            return
        g = torch.as_tensor(g, dtype=torch.float32).to(self.device).contiguous()
        assert g.shape == (3,) + self.shape
        C.tslb_set_force_field(self.h, g)

    def step(self, n=1):
        C.tslb_step(self.h, n)

    # ---- velocity statistics (FP64 sums on the device)
    def stats_begin(self, profile_axis=None, field=False):
        """Start accumulating: profile sums along `profile_axis` (0 x, 1 y,
        2 z) and/or per-node sums (field=True)."""
        kinds = (C.TSLB_STATS_PROFILE if profile_axis is not None else 0) | (C.TSLB_STATS_FIELD if field else 0)
        self._stats_axis = profile_axis
        C.tslb_stats_begin(self.h, kinds, profile_axis if profile_axis is not None else 0)

    def stats_sample(self):
        C.tslb_stats_sample(self.h)

    def stats_profile(self):
        """(sums (n_axis, 13) float64 tensor on the host, number of samples)."""
        n_axis = (self.shape[2], self.shape[1], self.shape[0])[self._stats_axis]
        rows, ns = C.tslb_stats_profile(self.h, n_axis)
        return torch.tensor(rows, dtype=torch.float64), ns

    def stats_field(self):
        """Per-node mean velocity (3, nz, ny, nx) and covariances (6, ...)."""
        mean = torch.empty((3,) + self.shape, dtype=torch.float32, device=self.device)
        cov = torch.empty((6,) + self.shape, dtype=torch.float32, device=self.device)
        C.tslb_stats_field(self.h, mean, cov)
        return mean, cov

    def stats_jet(self, axis, center):
        """Centreline velocity and half-width of every cross-section along
        `axis` from the time-averaged field."""
        n_axis = (self.shape[2], self.shape[1], self.shape[0])[axis]
        uc = torch.empty(n_axis, dtype=torch.float32, device=self.device)
        rh = torch.empty(n_axis, dtype=torch.float32, device=self.device)
        C.tslb_stats_jet(self.h, axis, center, uc, rh)
        return uc, rh

    def set_relaxation_profile(self, tau_z):
        """Relaxation time per z plane (nz values), or None for the uniform tau."""
        if tau_z is not None:
            assert len(tau_z) == self.shape[0]
        C.tslb_set_relaxation_profile(self.h, tau_z)

    def step_timed(self, n):
        """n steps; returns (ms in the main update kernel, ms in the per-step
        auxiliary launches), summed over the steps."""
        return C.tslb_step_timed(self.h, n)

    @property
    def t(self):
        return C.tslb_get_time(self.h)

    @t.setter
    def t(self, value):
        C.tslb_set_time(self.h, value)

    def reduce(self, check=True):
        """FP64 (mass, momentum x3, kinetic energy) over fluid nodes; synchronises."""
        out, rc = C.tslb_reduce(self.h, check=check)
        return out, rc

    def state_bytes(self):
        return C.tslb_state_bytes(self.h)

    def save_raw(self, dst=None):
        if dst is None:
            dst = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        C.tslb_save_state(self.h, dst)
        return dst

    def load_raw(self, src):
        C.tslb_load_state(self.h, src)

    def adjoint_step(self, raw_t, raw_t1, lam_t1, dg=None):
        lam_t = torch.empty_like(lam_t1)
        C.tslb_adjoint_step(self.h, raw_t, raw_t1, lam_t1, lam_t, dg)
        return lam_t

    def adjoint_seed(self, raw, objective=C.TSLB_OBJ_KINETIC_ENERGY):
        lam = torch.empty((10,) + self.shape, dtype=torch.float32, device=self.device)
        C.tslb_adjoint_seed(self.h, raw, lam, objective)
        return lam

    def objective(self, objective=C.TSLB_OBJ_KINETIC_ENERGY):
        """Value of an objective at the current level (FP64)."""
        return C.tslb_objective(self.h, objective)


class TslbRollout(torch.autograd.Function):
    """L after `nsteps` steps from (rho = 1, u0, Pi = 0) under the force field
    g, with checkpoints every `every` steps; L is the kinetic energy
    1/2 sum rho |u|^2 (TSLB_OBJ_KINETIC_ENERGY, the default) or the wall
    shear force on the y and z walls (TSLB_OBJ_WALL_SHEAR).

    forward(g (3, nz, ny, nx), u0 (3, nz, ny, nx), solver, nsteps, every
    [, objective]) -> L (float64 scalar); backward returns dL/dg and dL/du0
    from the library's discrete adjoint, recomputing each checkpointed
    segment once.
    """

    @staticmethod
    def forward(ctx, g, u0, solver, nsteps, every, objective=C.TSLB_OBJ_KINETIC_ENERGY):
        st = torch.zeros((10,) + solver.shape, dtype=torch.float32, device=solver.device)
        st[1:4] = u0.detach().to(torch.float32)
        solver.t = 0
        solver.set_force_field(g.detach())
        solver.set_state(st)
        nbytes = C.tslb_rollout_workspace_bytes(solver.h, nsteps, every)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=solver.device)
        C.tslb_rollout_forward(solver.h, nsteps, every, ws)
        final = solver.save_raw()
        loss = solver.objective(objective)
        ctx.solver, ctx.nsteps, ctx.every, ctx.objective = solver, nsteps, every, objective
        ctx.save_for_backward(ws, final)
        return torch.tensor(loss, dtype=torch.float64, device=solver.device)

    @staticmethod
    def backward(ctx, dL):
        ws, final = ctx.saved_tensors
        solver = ctx.solver
        lam = solver.adjoint_seed(final, ctx.objective)
        dg = torch.zeros((3,) + solver.shape, dtype=torch.float32, device=solver.device)
        C.tslb_rollout_backward(solver.h, ctx.nsteps, ctx.every, ws, lam, dg)
        scale = dL.to(torch.float32)
        return dg * scale, lam[1:4] * scale, None, None, None, None
