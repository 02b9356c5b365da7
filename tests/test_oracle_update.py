"""Pins of the oracle's full update (Section 2.2, the recursive thread-safe
step with the forcing of Section 3.1 and the boundaries of Section 2.3).

Fixed by the method and by mathematics: exact fixed points, closed-form
relaxation, conservation laws, the tau = 1 reduction to a streamed
equilibrium, the closed-form linear shear-mode eigenvalue, laminar
Poiseuille flow between half-way walls, Taylor-Green decay at
nu = cs2 (tau - 1/2), cube-symmetry equivariance, and an independent
population-push implementation on tiny grids.
"""
import itertools

import numpy as np
import pytest

import workloads as W

CS2 = 1.0 / 3.0


@pytest.mark.parametrize("order", [3, 2])
def test_uniform_equilibrium_is_a_fixed_point(oracle, order):
    G = oracle.make_grid(4, 5, 3, 0.7, order=order)
    st = W.rest_state(G.shape)
    st[0] = 1.13
    st[1:4] = np.array([0.07, -0.04, 0.02])[:, None, None, None]
    out = oracle.step(G, st)
    assert np.abs(out - st).max() < 1e-15


@pytest.mark.parametrize("order", [3, 2])
def test_homogeneous_relaxation_closed_form(oracle, order):
    """Uniform rho, u and Pi: rho and u are kept, Pi -> (1 - omega) Pi."""
    tau = 0.62
    G = oracle.make_grid(3, 4, 5, tau, order=order)
    st = W.rest_state(G.shape)
    st[0] = 0.98
    st[1:4] = np.array([0.03, 0.05, -0.02])[:, None, None, None]
    st[4:] = np.array([1e-3, -2e-3, 5e-4, 7e-4, -3e-4, 2e-4])[:, None, None, None]
    out = oracle.step(G, st)
    want = st.copy()
    want[4:] *= 1.0 - 1.0 / tau
    assert np.abs(out - want).max() < 1e-15


@pytest.mark.parametrize("order", [3, 2])
def test_conservation_periodic_and_forced(oracle, order):
    G = oracle.make_grid(5, 4, 6, 0.55, order=order)
    st = W.random_state(G.shape, seed=11)
    r0, _ = oracle.reduce(G, st)
    r1, _ = oracle.reduce(G, oracle.step(G, st))
    assert abs(r1[0] - r0[0]) < 1e-12 * r0[0]
    assert np.abs(r1[1:4] - r0[1:4]).max() < 1e-14
    g = W.random_force(G.shape, seed=12, amp=1e-3)
    r2, _ = oracle.reduce(G, oracle.step(G, st, g))
    assert abs(r2[0] - r0[0]) < 1e-12 * r0[0]
    # the local forcing adds exactly sum_y rho_y g_y of momentum per step
    assert np.allclose(r2[1:4] - r0[1:4], (st[0] * g).sum(axis=(1, 2, 3)), rtol=0, atol=1e-15)


def test_mass_conserved_with_bounce_back_walls(oracle):
    G = oracle.make_grid(4, 7, 5, 0.7, faces=(0, 0, 1, 1, 1, 1), force=(1e-4, 0, 0))
    st = W.random_state(G.shape, seed=13)
    kinds = oracle.node_kinds(G)
    m0 = st[0][kinds == 0].sum()
    out = st
    for t in range(5):
        out = oracle.step(G, out, t=t)
    assert abs(out[0][kinds == 0].sum() - m0) < 1e-12 * m0


def test_tau_one_is_a_streamed_equilibrium(oracle):
    """At omega = 1 the non-equilibrium input drops out and every population is
    the third-order equilibrium of its upstream node (BGK with full relaxation)."""
    G = oracle.make_grid(4, 3, 5, 1.0)
    st = W.random_state(G.shape, seed=14, pi_amp=1e-2)
    c, w, _ = oracle.lattice()
    nz, ny, nx = G.shape
    fe = np.zeros((27,) + G.shape)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        for i in range(27):
            fe[i, z, y, x] = oracle.feq(i, st[0, z, y, x], st[1:4, z, y, x])
    fin = np.stack([np.roll(fe[i], shift=(c[i, 2], c[i, 1], c[i, 0]), axis=(0, 1, 2)) for i in range(27)])
    rho = fin.sum(0)
    j = np.einsum("izyx,ia->azyx", fin, c)
    out = oracle.step(G, st)
    assert np.abs(out[0] - rho).max() < 1e-15
    assert np.abs(out[1:4] - j / rho).max() < 1e-15


def _push_reference(oracle, G, st, g, tau_z=None):
    """Independent population-push implementation: every node emits its 27
    post-collision populations along c_i, relaxed with its own tau (that of
    its z plane when a profile is given); a population aimed at a solid node
    is returned to its emitter in the opposite direction; moments are summed
    from the arrived sets.  Walls/periodic only."""
    c, w, opp = oracle.lattice()
    nz, ny, nx = G.shape
    kinds = oracle.node_kinds(G)
    fin = np.zeros((27,) + G.shape)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        if kinds[z, y, x] != 0:
            continue
        omega = 1.0 / (G.tau if tau_z is None else tau_z[z])
        m = st[:, z, y, x]
        gg = g[:, z, y, x] if g is not None else np.array(G.force[:])
        for i in range(27):
            f = oracle.fpost(i, m, gg, omega, G.order)
            X, Y, Z = x + c[i, 0], y + c[i, 1], z + c[i, 2]
            X, Y, Z = X % nx, Y % ny, Z % nz  # wall layers sit inside the array
            if kinds[Z, Y, X] == 1:
                fin[opp[i], z, y, x] += f
            else:
                fin[i, Z, Y, X] += f
    out = st.copy()
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        if kinds[z, y, x] == 0:
            out[:, z, y, x] = oracle.moments(fin[:, z, y, x])
    return out


@pytest.mark.parametrize("order", [3, 2])
@pytest.mark.parametrize("faces", [(0,) * 6, (0, 0, 1, 1, 0, 0), (1, 1, 0, 0, 1, 1)])
def test_pull_update_matches_population_push(oracle, faces, order):
    G = oracle.make_grid(4, 5, 6, 0.66, faces=faces, order=order)
    st = W.random_state(G.shape, seed=15)
    g = W.random_force(G.shape, seed=16, amp=1e-4)
    want = _push_reference(oracle, G, st, g)
    got = oracle.step(G, st, g)
    kinds = oracle.node_kinds(G)
    assert np.abs((got - want)[:, kinds == 0]).max() < 1e-15


@pytest.mark.parametrize("faces", [(0,) * 6, (0, 0, 1, 1, 1, 1)])
def test_relaxation_profile_matches_population_push(oracle, faces):
    """A relaxation time that varies with z (the jet's outlet sponge,
    Section 3.2): each population relaxes with the tau of the node that
    emits it."""
    tau_z = [0.55, 0.6, 0.72, 0.9, 1.3, 2.0]
    G = oracle.make_grid(4, 5, 6, 0.66, faces=faces, tau_z=tau_z)
    st = W.random_state(G.shape, seed=35)
    g = W.random_force(G.shape, seed=36, amp=1e-4)
    want = _push_reference(oracle, G, st, g, tau_z)
    got = oracle.step(G, st, g)
    kinds = oracle.node_kinds(G)
    assert np.abs((got - want)[:, kinds == 0]).max() < 1e-15
    # a constant profile is the scalar tau, bit for bit
    G1 = oracle.make_grid(4, 5, 6, 0.66, faces=faces, tau_z=[0.66] * 6)
    G0 = oracle.make_grid(4, 5, 6, 0.66, faces=faces)
    assert np.array_equal(oracle.step(G1, st, g), oracle.step(G0, st, g))
    # mass and momentum stay conserved (periodic box)
    if faces == (0,) * 6:
        r0, _ = oracle.reduce(G, st)
        r1, _ = oracle.reduce(G, got)
        assert abs(r1[0] - r0[0]) < 1e-12 * r0[0]
        assert np.allclose(r1[1:4] - r0[1:4], (st[0] * g).sum(axis=(1, 2, 3)), rtol=0, atol=1e-15)


def _rotate(st, perm, sign):
    """Apply x'_a = sign[a] x_{perm[a]} to a state (scalar, vector, tensor)."""
    n = st.shape[-1]
    arr = st.transpose(0, 3, 2, 1)  # (q, x, y, z) spatial order
    arr = np.transpose(arr, (0,) + tuple(1 + p for p in perm))
    for a in range(3):
        if sign[a] < 0:
            arr = np.flip(arr, axis=1 + a)
            arr = np.roll(arr, 1, axis=1 + a)  # x -> -x mod n keeps node 0 fixed
    arr = arr.transpose(0, 3, 2, 1)
    out = np.empty_like(arr)
    out[0] = arr[0]
    R = np.zeros((3, 3))
    for a in range(3):
        R[a, perm[a]] = sign[a]
    out[1:4] = np.einsum("ab,bzyx->azyx", R, arr[1:4])
    P = np.zeros((3, 3) + arr.shape[1:])
    idx = {(0, 0): 4, (1, 1): 5, (2, 2): 6, (0, 1): 7, (0, 2): 8, (1, 2): 9}
    for (a, b), q in idx.items():
        P[a, b] = arr[q]
        P[b, a] = arr[q]
    P2 = np.einsum("ac,bd,cdzyx->abzyx", R, R, P)
    for (a, b), q in idx.items():
        out[q] = P2[a, b]
    assert n == st.shape[-1]
    return out


@pytest.mark.parametrize("order", [3, 2])
def test_cube_symmetry_equivariance(oracle, order):
    """The 48 symmetries of the cube commute with the update (isotropy of the
    Hermite tensors and the lattice), tested on a tiny periodic grid."""
    G = oracle.make_grid(4, 4, 4, 0.58, order=order)
    st = W.random_state(G.shape, seed=17, u_amp=0.05, pi_amp=3e-3)
    base = oracle.step(G, st)
    worst = 0.0
    for perm in itertools.permutations(range(3)):
        for sign in itertools.product((1, -1), repeat=3):
            a = oracle.step(G, _rotate(st, perm, sign))
            b = _rotate(base, perm, sign)
            worst = max(worst, np.abs(a - b).max())
    assert worst < 1e-15


@pytest.mark.parametrize("order", [3, 2])
def test_shear_wave_closed_form_eigenvalue(oracle, order):
    """Linear shear mode u_x = A sin(k y), Pi_xy = s A cos(k y): one step is the
    2x2 map [[(2 + cos k)/3, (1-w) sin k], [-sin k / 3, (1-w) cos k]] (derived
    from the update with the D3Q27 weights); its dominant eigenvalue gives the
    decay, and -ln(lambda) -> nu k^2 with nu = cs2 (tau - 1/2)."""
    n, tau, A, steps = 32, 0.8, 1e-6, 50
    om = 1.0 / tau
    k = 2 * np.pi / n
    T = (2 + np.cos(k)) / 3 + (1 - om) * np.cos(k)
    D = (1 - om) * (1 + 2 * np.cos(k)) / 3
    lam = (T + np.sqrt(T * T - 4 * D)) / 2
    s = -(np.sin(k) / 3) / (lam - (1 - om) * np.cos(k))
    G = oracle.make_grid(1, n, 1, tau, order=order)
    y = np.arange(n)
    st = W.rest_state(G.shape)
    st[1, 0, :, 0] = A * np.sin(k * y)
    st[7, 0, :, 0] = s * A * np.cos(k * y)
    out = oracle.run(G, st, steps)
    amp = (out[1, 0, :, 0] * np.sin(k * y)).sum() / (np.sin(k * y) ** 2).sum()
    assert amp / A == pytest.approx(lam ** steps, rel=1e-8)
    nu = CS2 * (tau - 0.5)
    assert -np.log(lam) == pytest.approx(nu * k * k, rel=1e-3)


@pytest.mark.parametrize("tau", [0.8, 1.0, 1.5])
def test_poiseuille_between_halfway_walls(oracle, tau):
    """Steady forced flow between walls at y = 1/2 and y = ny - 3/2:
    u(y) = g/(2 nu) [(y - 1/2)(ny - 3/2 - y) - 1/4] + g/2 (exact for this
    scheme's linear steady state; the +g/2 - g/(8 nu) is the discrete offset)."""
    ny, g = 12, 1e-6
    G = oracle.make_grid(1, ny, 1, tau, faces=(0, 0, 1, 1, 0, 0), force=(g, 0, 0))
    out = oracle.run(G, W.rest_state(G.shape), 6000)
    nu = CS2 * (tau - 0.5)
    y = np.arange(1, ny - 1)
    ua = g / (2 * nu) * ((y - 0.5) * (ny - 1.5 - y) - 0.25) + g / 2
    assert np.abs(out[1, 0, 1:-1, 0] - ua).max() < 1e-9 * ua.max()
    # steady shear stress: Pi_xy = -cs2 tau du/dy exactly at the bulk nodes
    uy = out[1, 0, :, 0]
    dudy = (uy[3:-1] - uy[1:-3]) / 2
    assert np.allclose(out[7, 0, 2:-2, 0], -CS2 * tau * dudy, rtol=1e-6, atol=1e-16)


def test_taylor_green_decay_rate_and_conservation(oracle):
    """The z-invariant Taylor-Green vortex decays as exp(-2 nu k^2 t); the
    fitted rate over t in [20, 100] matches within 1e-3 and mass and momentum
    are conserved to round-off."""
    case = W.tgv_case()
    G = oracle.make_grid(case.nx, case.ny, case.nz, case.tau)
    st = W.tgv_state(case.nx, case.extra["u0"])
    r0, _ = oracle.reduce(G, st)
    mode = st[1]
    ts, amps = [], []
    cur = oracle.run(G, st, 20)
    for t in range(20, 101, 20):
        if t > 20:
            cur = oracle.run(G, cur, 20, t0=t - 20)
        ts.append(t)
        amps.append((cur[1] * mode).sum() / (mode * mode).sum())
    rate = -np.polyfit(ts, np.log(amps), 1)[0]
    nu = CS2 * (case.tau - 0.5)
    k = 2 * np.pi / case.nx
    assert rate / (2 * nu * k * k) == pytest.approx(1.0, abs=1e-3)
    r1, bad = oracle.reduce(G, cur)
    assert bad == 0
    assert abs(r1[0] - r0[0]) < 1e-12 * r0[0]
    assert np.abs(r1[1:4] - r0[1:4]).max() < 1e-12


def test_update_nodes_equals_full_step(oracle):
    G = oracle.make_grid(6, 5, 4, 0.7, faces=(0, 0, 1, 1, 0, 0), force=(1e-5, 0, 0))
    st = W.random_state(G.shape, seed=18)
    full = oracle.step(G, st)
    kinds = oracle.node_kinds(G).reshape(-1)
    idx = np.flatnonzero(kinds == 0)[::3]
    part = oracle.update_nodes(G, st, idx)
    assert np.array_equal(part, full.reshape(10, -1)[:, idx])


def test_order_two_drops_third_order_moments(oracle):
    """The higher-order update differs from the regularised one exactly in the
    third-order Hermite content: from a uniform moving state with Pi = 0 both
    keep (rho, u), but their post-collision populations differ by
    w H3:(rho u u u) / (6 cs6) (Eq. (eqts) minus Eq. (lbequil))."""
    c, w, _ = oracle.lattice()
    m = np.array([1.03, 0.05, -0.04, 0.02, 0, 0, 0, 0, 0, 0], dtype=float)
    rho, u = m[0], m[1:4]
    for i in range(27):
        d = oracle.fpost(i, m, np.zeros(3), 1.3, 3) - oracle.fpost(i, m, np.zeros(3), 1.3, 2)
        cu = c[i] @ u
        h3uuu = cu ** 3 - 3 * CS2 * cu * (u @ u)
        assert d == pytest.approx(w[i] * rho * h3uuu / (6 * CS2 ** 3), rel=1e-10, abs=1e-18)
