"""FP64 CPU oracle for the moment-only high-order thread-safe LB update.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  The product path
(``paper_2401_17074_amd``) never imports this package, and this package never
imports the product.  The arithmetic lives in ``tslb_oracle.c`` (plain C99,
double precision, explicit Hermite tensors per population; Montessori et al.,
arXiv:2401.17074, Section 2); this module only marshals numpy arrays.

State arrays are float64 of shape (10, nz, ny, nx): rho, u_x, u_y, u_z and
Pi^neq in the order xx, yy, zz, xy, xz, yz.  Note the oracle keeps rho itself
(the paper's variable), not rho - 1.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "tslb_oracle.c")

PERIODIC, WALL, INLET, OUTLET = 0, 1, 2, 3
FLUID, SOLID, GHOST = 0, 1, 2


def build():
    """Compile the oracle (gcc, OpenMP).  Building the checker is not using it."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-fcx-limited-range",
           _SRC, "-o", _LIB_PATH + ".tmp", "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)


class Grid(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("face", ctypes.c_int * 6),
        ("tau", ctypes.c_double),
        ("force", ctypes.c_double * 3),
        ("inlet_u", ctypes.c_double * 3),
        ("inlet_center", ctypes.c_double * 2),
        ("inlet_radius", ctypes.c_double),
        ("inlet_noise", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("order", ctypes.c_int),
        ("noise_kind", ctypes.c_int),
        ("tau_z", ctypes.POINTER(ctypes.c_double)),
        ("lattice", ctypes.c_int),
    ]

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def n(self):
        return self.nx * self.ny * self.nz


def make_grid(nx, ny, nz, tau, faces=(PERIODIC,) * 6, force=(0.0, 0.0, 0.0), inlet_u=(0.0, 0.0, 0.0),
              inlet_center=(0.0, 0.0), inlet_radius=0.0, inlet_noise=0.0, seed=0, order=3, noise_kind=0,
              tau_z=None, lattice=27):
    """order: 3 = the recursive third-order update (Section 2.2), 2 = the
    regularised second-order update (Eq. (fullstrcoll)).
    noise_kind: inlet perturbation, 0 uniform in [-1, 1), 1 standard Gaussian.
    tau_z: optional relaxation time per z plane (nz values; the outlet sponge
    of Section 3.2); every node relaxes with the value of its own plane.
    lattice: 27 (D3Q27) or 9 (D2Q9: nz = 1 with periodic z faces; the state
    keeps ten fields, u_z and the Pi components with a z index are zero)."""
    if lattice == 9:
        assert nz == 1 and faces[4] == PERIODIC and faces[5] == PERIODIC
    g = Grid()
    g.nx, g.ny, g.nz = nx, ny, nz
    for k in range(6):
        g.face[k] = faces[k]
    g.tau = tau
    for a in range(3):
        g.force[a] = force[a]
        g.inlet_u[a] = inlet_u[a]
    g.inlet_center[0], g.inlet_center[1] = inlet_center
    g.inlet_radius = inlet_radius
    g.inlet_noise = inlet_noise
    g.seed = seed
    g.order = order
    g.noise_kind = noise_kind
    g.lattice = lattice
    if tau_z is not None:
        arr = np.ascontiguousarray(tau_z, dtype=np.float64)
        assert arr.shape == (nz,)
        g._tau_z = arr  # keeps the buffer alive as long as the grid
        g.tau_z = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return g


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_L = ctypes.POINTER(ctypes.c_long)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    G = ctypes.POINTER(Grid)
    sig = {
        "or_lattice": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), _D, ctypes.POINTER(ctypes.c_int)]),
        "or_hermite": (ctypes.c_double, [ctypes.c_int] * 6),
        "or_feq": (ctypes.c_double, [ctypes.c_int, ctypes.c_int, ctypes.c_double, _D, ctypes.c_int]),
        "or_fneq": (ctypes.c_double, [ctypes.c_int, ctypes.c_int, _D, _D, ctypes.c_int]),
        "or_fpost": (ctypes.c_double, [ctypes.c_int, ctypes.c_int, _D, _D, ctypes.c_double, ctypes.c_int]),
        "or_moments": (None, [ctypes.c_int, _D, _D]),
        "or_node_kind": (ctypes.c_int, [G, ctypes.c_long]),
        "or_node_kinds": (None, [G, ctypes.c_void_p]),
        "or_ghost_fill": (None, [G, _D, ctypes.c_long]),
        "or_step": (None, [G, _D, _D, _D, ctypes.c_long]),
        "or_round_storage": (None, [G, _D, ctypes.c_int, _D]),
        "or_run": (ctypes.c_int, [G, _D, _D, ctypes.c_long, ctypes.c_int, ctypes.c_int, _D]),
        "or_update_nodes": (None, [G, _D, _D, _L, ctypes.c_long, _D]),
        "or_reduce": (ctypes.c_long, [G, _D, _D]),
        "or_num_threads": (ctypes.c_int, []),
        "or_splitmix64": (ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_uint64]),
        "or_inlet_xi": (ctypes.c_double, [ctypes.c_uint64, ctypes.c_long, ctypes.c_long, ctypes.c_long,
                                          ctypes.c_int]),
        "or_inlet_gauss": (ctypes.c_double, [ctypes.c_uint64, ctypes.c_long, ctypes.c_long, ctypes.c_long,
                                             ctypes.c_int]),
        "or_round_fp16": (ctypes.c_double, [ctypes.c_double]),
        "or_round_bf16": (ctypes.c_double, [ctypes.c_double]),
        "or_jvp_step": (ctypes.c_int, [G, _D, _D, _D, _D, ctypes.c_long, _D]),
        "or_adjoint_step": (ctypes.c_int, [G, _D, _D, _D, _D, _D]),
        "or_adjoint_nodes": (ctypes.c_int, [G, _D, _D, _D, _L, ctypes.c_long, _D, _D]),
        "or_ke_seed": (ctypes.c_double, [G, _D, _D]),
        "or_wall_shear_seed": (ctypes.c_double, [G, _D, _D]),
        "or_rollout_grad": (ctypes.c_int, [G, _D, _D, ctypes.c_long, ctypes.c_int, ctypes.c_int, _D, _D, _D]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _state(grid, st):
    st = np.ascontiguousarray(st, dtype=np.float64)
    assert st.shape == (10,) + grid.shape, st.shape
    return st


def _field(grid, g):
    if g is None:
        return None
    g = np.ascontiguousarray(g, dtype=np.float64)
    assert g.shape == (3,) + grid.shape
    return g


def lattice(lattice=27):
    """(c (q, 3), w (q,), opp (q,)) of lattice 27 (D3Q27) or 9 (D2Q9)."""
    lib = _load()
    c = (ctypes.c_int * 81)()
    w = (ctypes.c_double * 27)()
    opp = (ctypes.c_int * 27)()
    q = lib.or_lattice(lattice, c, w, opp)
    return (np.array(c[:3 * q], dtype=np.int64).reshape(q, 3), np.array(w[:q]),
            np.array(opp[:q], dtype=np.int64))


def hermite(i, order, a=0, b=0, g=0, lattice=27):
    return _load().or_hermite(lattice, i, order, a, b, g)


def feq(i, rho, u, order=3, lattice=27):
    u = np.ascontiguousarray(u, dtype=np.float64)
    return _load().or_feq(lattice, i, rho, _p(u), order)


def fneq(i, pi6, u, order=3, lattice=27):
    pi6 = np.ascontiguousarray(pi6, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    return _load().or_fneq(lattice, i, _p(pi6), _p(u), order)


def fpost(i, m, g, omega, order=3, lattice=27):
    m = np.ascontiguousarray(m, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    return _load().or_fpost(lattice, i, _p(m), _p(g), omega, order)


def moments(f, lattice=27):
    f = np.ascontiguousarray(f, dtype=np.float64)
    m = np.zeros(10)
    _load().or_moments(lattice, _p(f), _p(m))
    return m


def node_kinds(grid):
    """Node classes (0 fluid, 1 solid, 2 ghost), shape (nz, ny, nx)."""
    out = np.empty(grid.shape, dtype=np.int8)
    _load().or_node_kinds(ctypes.byref(grid), out.ctypes.data)
    return out


def ghost_fill(grid, st, t=0):
    st = _state(grid, st).copy()
    _load().or_ghost_fill(ctypes.byref(grid), _p(st), t)
    return st


def step(grid, st, g=None, t=0):
    st = _state(grid, st)
    out = np.empty_like(st)
    g = _field(grid, g)
    _load().or_step(ctypes.byref(grid), _p(st), _p(out), _p(g), t)
    return out


def run(grid, st, nsteps, g=None, t0=0, storage=0, scale=(1.0, 1.0, 1.0)):
    st = _state(grid, st).copy()
    g = _field(grid, g)
    sc = np.ascontiguousarray(scale, dtype=np.float64)
    rc = _load().or_run(ctypes.byref(grid), _p(st), _p(g), t0, nsteps, storage, _p(sc))
    if rc != 0:
        raise MemoryError("oracle run failed")
    return st


def round_storage(grid, st, kind, scale):
    st = _state(grid, st).copy()
    sc = np.ascontiguousarray(scale, dtype=np.float64)
    _load().or_round_storage(ctypes.byref(grid), _p(st), kind, _p(sc))
    return st


def update_nodes(grid, st, idx, g=None):
    st = _state(grid, st)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty((10, idx.size))
    g = _field(grid, g)
    _load().or_update_nodes(ctypes.byref(grid), _p(st), _p(g), idx.ctypes.data_as(_L), idx.size, _p(out))
    return out


def reduce(grid, st):
    st = _state(grid, st)
    out = np.zeros(5)
    bad = _load().or_reduce(ctypes.byref(grid), _p(st), _p(out))
    return out, bad


def num_threads():
    """OpenMP threads the oracle's parallel loops use."""
    return _load().or_num_threads()


def splitmix64(seed, k):
    return _load().or_splitmix64(seed, k)


def inlet_xi(seed, t, n, N, a):
    return _load().or_inlet_xi(seed, t, n, N, a)


def inlet_gauss(seed, t, n, N, a):
    return _load().or_inlet_gauss(seed, t, n, N, a)


def round_fp16(x):
    return _load().or_round_fp16(float(x))


def round_bf16(x):
    return _load().or_round_bf16(float(x))


def jvp_step(grid, st, dst, g=None, dg=None, t=0):
    st = _state(grid, st)
    dst = _state(grid, dst)
    g = _field(grid, g)
    dg = _field(grid, dg)
    out = np.empty_like(st)
    if _load().or_jvp_step(ctypes.byref(grid), _p(st), _p(g), _p(dst), _p(dg), t, _p(out)) != 0:
        raise MemoryError
    return out


def adjoint_step(grid, st, lam1, g=None):
    st = _state(grid, st)
    lam1 = _state(grid, lam1)
    g = _field(grid, g)
    lam0 = np.empty_like(st)
    dg = np.zeros((3,) + grid.shape)
    if _load().or_adjoint_step(ctypes.byref(grid), _p(st), _p(g), _p(lam1), _p(lam0), _p(dg)) != 0:
        raise ValueError("oracle adjoint: unsupported lattice or out of memory")
    return lam0, dg


def adjoint_nodes(grid, st, lam1, idx, g=None):
    st = _state(grid, st)
    lam1 = _state(grid, lam1)
    g = _field(grid, g)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    lam = np.empty((10, idx.size))
    dg = np.empty((3, idx.size))
    if _load().or_adjoint_nodes(ctypes.byref(grid), _p(st), _p(g), _p(lam1), idx.ctypes.data_as(_L), idx.size,
                                _p(lam), _p(dg)) != 0:
        raise ValueError("oracle adjoint: unsupported lattice or out of memory")
    return lam, dg


def ke_seed(grid, st):
    st = _state(grid, st)
    lam = np.empty_like(st)
    L = _load().or_ke_seed(ctypes.byref(grid), _p(st), _p(lam))
    return L, lam


def wall_shear_seed(grid, st):
    """Wall shear objective (x force on the y and z walls) and dL/dM."""
    st = _state(grid, st)
    lam = np.empty_like(st)
    L = _load().or_wall_shear_seed(ctypes.byref(grid), _p(st), _p(lam))
    return L, lam


OBJ_KINETIC_ENERGY, OBJ_WALL_SHEAR = 0, 1


def rollout_grad(grid, st0, nsteps, g=None, t0=0, objective=OBJ_KINETIC_ENERGY):
    """Loss L after nsteps (objective 0: 1/2 sum rho |u|^2; 1: the wall shear
    force), dL/dM_0 and dL/dg (FP64)."""
    st0 = _state(grid, st0)
    g = _field(grid, g)
    loss = ctypes.c_double(0.0)
    lam0 = np.empty_like(st0)
    dg = np.zeros((3,) + grid.shape)
    if _load().or_rollout_grad(ctypes.byref(grid), _p(st0), _p(g), t0, nsteps, objective, ctypes.byref(loss),
                               _p(lam0), _p(dg)) != 0:
        raise ValueError("oracle adjoint: unsupported lattice or out of memory")
    return loss.value, lam0, dg
