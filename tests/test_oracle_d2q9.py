"""Pins of the oracle's D2Q9 update, the two-dimensional counterpart of
D3Q27 (Section 2.2).  D2Q9 runs on an nz = 1 grid with the ten-field state
(u_z and the Pi components with a z index held at zero).

Fixed by mathematics: the unique isotropic shell weights, the Hermite
coefficients of the equilibrium and non-equilibrium parts, fixed points,
closed-form relaxation, conservation, an independent population push, the
eight symmetries of the square, the closed-form shear-mode eigenvalue, and
the marginal identity: a z-invariant D3Q27 state (u_z = Pi_xz = Pi_yz = 0,
any Pi_zz) on an nz = 1 grid steps its x-y moments exactly as D2Q9 does,
because the D3Q27 weights are the product of the D2Q9 weights and W(c_z),
and every term that depends on c_z sums to zero over c_z."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import workloads as W

CS2 = 1.0 / 3.0
L9 = 9


def _state2d(shape, seed, u_amp=0.05, pi_amp=2e-3):
    st = W.random_state(shape, seed=seed, u_amp=u_amp, pi_amp=pi_amp)
    st[3] = 0.0   # u_z
    st[6] = 0.0   # Pi_zz
    st[8] = 0.0   # Pi_xz
    st[9] = 0.0   # Pi_yz
    return st


def test_weights_are_the_unique_isotropic_set(oracle):
    c, w, opp = oracle.lattice(L9)
    assert c.shape == (9, 3) and np.all(c[:, 2] == 0)
    # shells 0, 1, 2: sum w = 1, sum w cx^2 = 1/3, sum w cx^2 cy^2 = 1/9
    # -> W0 + 4 W1 + 4 W2 = 1, 2 W1 + 4 W2 = 1/3, 4 W2 = 1/9
    W2 = Fraction(1, 36)
    W1 = (Fraction(1, 3) - 4 * W2) / 2
    W0 = 1 - 4 * W1 - 4 * W2
    assert (W0, W1, W2) == (Fraction(4, 9), Fraction(1, 9), Fraction(1, 36))
    for i in range(9):
        assert w[i] == pytest.approx(float((W0, W1, W2)[int(np.abs(c[i]).sum())]), rel=1e-15)
        assert (c[opp[i]] == -c[i]).all()


def test_isotropy_to_fourth_order(oracle):
    c, w, _ = oracle.lattice(L9)
    c = c[:, :2]
    d = np.eye(2)
    assert np.sum(w) == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), CS2 * d, atol=1e-15)
    iso4 = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                       + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), iso4, atol=1e-15)


def _H3(c):
    d = np.eye(2)
    return (np.einsum("ia,ib,ig->iabg", c, c, c)
            - CS2 * (np.einsum("ig,ab->iabg", c, d) + np.einsum("ia,bg->iabg", c, d)
                     + np.einsum("ib,ag->iabg", c, d)))


@pytest.mark.parametrize("order", [3, 2])
def test_hermite_coefficients(oracle, order):
    """Projections on H0..H3 return rho, rho u, rho u u, rho u u u (the xxx
    and yyy components are not supported and vanish), and for the
    non-equilibrium part 0, 0, Pi, symmetrised Pi u (order 3) or 0."""
    c, w, _ = oracle.lattice(L9)
    c2 = c[:, :2].astype(float)
    rng = np.random.default_rng(5)
    rho, u = 1.04, np.array([0.06, -0.03, 0.0])
    pi6 = np.array([2e-3, -1e-3, 0.0, 7e-4, 0.0, 0.0])
    P = np.array([[pi6[0], pi6[3]], [pi6[3], pi6[1]]])
    fe = np.array([oracle.feq(i, rho, u, order, lattice=L9) for i in range(9)])
    fn = np.array([oracle.fneq(i, pi6, u, order, lattice=L9) for i in range(9)])
    H2 = np.einsum("ia,ib->iab", c2, c2) - CS2 * np.eye(2)
    H3 = _H3(c2)
    u2 = u[:2]
    assert fe.sum() == pytest.approx(rho, rel=1e-14)
    assert np.allclose(fe @ c2, rho * u2, rtol=1e-13)
    assert np.allclose(np.einsum("i,iab->ab", fe, H2), rho * np.outer(u2, u2), rtol=1e-12, atol=1e-16)
    a3 = np.einsum("i,iabg->abg", fe, H3)
    for a, b, g in itertools.product(range(2), repeat=3):
        want = 0.0 if (a == b == g or order == 2) else rho * u2[a] * u2[b] * u2[g]
        assert a3[a, b, g] == pytest.approx(want, abs=1e-15)
    assert abs(fn.sum()) < 1e-17 and np.allclose(fn @ c2, 0.0, atol=1e-17)
    assert np.allclose(np.einsum("i,iab->ab", fn, H2), P, rtol=1e-12, atol=1e-17)
    n3 = np.einsum("i,iabg->abg", fn, H3)
    for a, b, g in itertools.product(range(2), repeat=3):
        full = P[a, b] * u2[g] + P[b, g] * u2[a] + P[a, g] * u2[b]
        want = 0.0 if (a == b == g or order == 2) else full
        assert n3[a, b, g] == pytest.approx(want, abs=1e-17)


@pytest.mark.parametrize("order", [3, 2])
def test_fixed_point_relaxation_and_conservation(oracle, order):
    G = oracle.make_grid(5, 6, 1, 0.7, order=order, lattice=L9)
    st = W.rest_state(G.shape)
    st[0] = 1.1
    st[1:3] = np.array([0.05, -0.03])[:, None, None, None]
    assert np.abs(oracle.step(G, st) - st).max() < 1e-15
    st[4], st[5], st[7] = 1e-3, -2e-3, 5e-4
    want = st.copy()
    want[4:] *= 1.0 - 1.0 / 0.7
    assert np.abs(oracle.step(G, st) - want).max() < 1e-15
    rnd = _state2d(G.shape, 21)
    g = W.random_force(G.shape, seed=22, amp=1e-4)
    g[2] = 0.0
    r0, _ = oracle.reduce(G, rnd)
    out = oracle.step(G, rnd, g)
    r1, _ = oracle.reduce(G, out)
    assert abs(r1[0] - r0[0]) < 1e-12 * r0[0]
    assert np.allclose(r1[1:3] - r0[1:3], (rnd[0] * g[:2]).sum(axis=(1, 2, 3)), rtol=0, atol=1e-15)
    assert np.all(out[[3, 6, 8, 9]] == 0.0)


def _push_reference(oracle, G, st, g):
    c, w, opp = oracle.lattice(L9)
    _, ny, nx = G.shape
    kinds = oracle.node_kinds(G)
    omega = 1.0 / G.tau
    fin = np.zeros((9,) + G.shape)
    for y, x in itertools.product(range(ny), range(nx)):
        if kinds[0, y, x] != 0:
            continue
        for i in range(9):
            f = oracle.fpost(i, st[:, 0, y, x], g[:, 0, y, x], omega, G.order, lattice=L9)
            X, Y = (x + c[i, 0]) % nx, (y + c[i, 1]) % ny
            if kinds[0, Y, X] == 1:
                fin[opp[i], 0, y, x] += f
            else:
                fin[i, 0, Y, X] += f
    out = st.copy()
    for y, x in itertools.product(range(ny), range(nx)):
        if kinds[0, y, x] == 0:
            out[:, 0, y, x] = oracle.moments(fin[:, 0, y, x], lattice=L9)
    return out


@pytest.mark.parametrize("order", [3, 2])
@pytest.mark.parametrize("faces", [(0,) * 6, (0, 0, 1, 1, 0, 0), (1, 1, 1, 1, 0, 0)])
def test_pull_update_matches_population_push(oracle, faces, order):
    G = oracle.make_grid(6, 7, 1, 0.64, faces=faces, order=order, lattice=L9)
    st = _state2d(G.shape, 23)
    g = W.random_force(G.shape, seed=24, amp=1e-4)
    g[2] = 0.0
    want = _push_reference(oracle, G, st, g)
    got = oracle.step(G, st, g)
    kinds = oracle.node_kinds(G)
    assert np.abs((got - want)[:, kinds == 0]).max() < 1e-15


def _square_map(st, swap, sx, sy):
    """Apply a symmetry of the square (optional x <-> y swap, then sign flips)
    to a 2D state on an n x n grid (node 0 kept fixed)."""
    out = st.copy()
    arr = st[:, 0]  # (q, y, x)
    if swap:
        arr = np.transpose(arr, (0, 2, 1))
    if sx < 0:
        arr = np.roll(np.flip(arr, axis=2), 1, axis=2)
    if sy < 0:
        arr = np.roll(np.flip(arr, axis=1), 1, axis=1)
    R = np.array([[0, 1], [1, 0]]) if swap else np.eye(2)
    R = np.diag([sx, sy]) @ R
    u = np.einsum("ab,b...->a...", R, arr[1:3])
    P = np.array([[arr[4], arr[7]], [arr[7], arr[5]]])
    P2 = np.einsum("ac,bd,cd...->ab...", R, R, P)
    out[0, 0] = arr[0]
    out[1:3, 0] = u
    out[4, 0], out[5, 0], out[7, 0] = P2[0, 0], P2[1, 1], P2[0, 1]
    return out


@pytest.mark.parametrize("order", [3, 2])
def test_square_symmetry_equivariance(oracle, order):
    G = oracle.make_grid(6, 6, 1, 0.58, order=order, lattice=L9)
    st = _state2d(G.shape, 25)
    base = oracle.step(G, st)
    worst = 0.0
    for swap, sx, sy in itertools.product((False, True), (1, -1), (1, -1)):
        a = oracle.step(G, _square_map(st, swap, sx, sy))
        b = _square_map(base, swap, sx, sy)
        worst = max(worst, np.abs(a - b).max())
    assert worst < 1e-15


@pytest.mark.parametrize("order", [3, 2])
def test_shear_wave_closed_form_eigenvalue(oracle, order):
    """Same linear shear-mode map as on D3Q27 (the y-marginal of both
    lattices is the same three-point weight set)."""
    n, tau, A, steps = 32, 0.8, 1e-6, 50
    om = 1.0 / tau
    k = 2 * np.pi / n
    M = np.array([[(2 + np.cos(k)) / 3, (1 - om) * np.sin(k)], [-np.sin(k) / 3, (1 - om) * np.cos(k)]])
    G = oracle.make_grid(1, n, 1, tau, order=order, lattice=L9)
    y = np.arange(n)
    st = W.rest_state(G.shape)
    st[1, 0, :, 0] = A * np.sin(k * y)
    v = np.array([A, 0.0])
    for _ in range(steps):
        st = oracle.step(G, st)
        v = M @ v
    amp = 2 * (st[1, 0, :, 0] * np.sin(k * y)).sum() / n
    assert amp == pytest.approx(v[0], rel=1e-8)


@pytest.mark.parametrize("order", [3, 2])
@pytest.mark.parametrize("faces", [(0,) * 6, (0, 0, 1, 1, 0, 0), (1, 1, 0, 0, 0, 0)])
def test_marginal_of_a_z_invariant_d3q27_step(oracle, faces, order):
    st2 = _state2d((1, 7, 9), 26)
    g = W.random_force((1, 7, 9), seed=27, amp=1e-4)
    g[2] = 0.0
    G9 = oracle.make_grid(9, 7, 1, 0.61, faces=faces, order=order, lattice=L9)
    G27 = oracle.make_grid(9, 7, 1, 0.61, faces=faces, order=order)
    st3 = st2.copy()
    st3[6] = np.random.default_rng(28).uniform(-2e-3, 2e-3, st3[6].shape)  # any Pi_zz
    a = oracle.step(G9, st2, g)
    b = oracle.step(G27, st3, g)
    kinds = oracle.node_kinds(G9)
    xy = [0, 1, 2, 4, 5, 7]
    assert np.abs((a[xy] - b[xy])[:, kinds == 0]).max() < 1e-15


@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_poiseuille_between_halfway_walls(oracle, tau):
    """The D3Q27 steady Poiseuille profile (its y-marginal weights are the
    same): u(y) = g/(2 nu) [(y - 1/2)(ny - 3/2 - y) - 1/4] + g/2."""
    ny, g = 12, 1e-6
    G = oracle.make_grid(1, ny, 1, tau, faces=(0, 0, 1, 1, 0, 0), force=(g, 0, 0), lattice=L9)
    out = oracle.run(G, W.rest_state(G.shape), 6000)
    nu = (tau - 0.5) / 3.0
    y = np.arange(1, ny - 1)
    ua = g / (2 * nu) * ((y - 0.5) * (ny - 1.5 - y) - 0.25) + g / 2
    assert np.abs(out[1, 0, 1:-1, 0] - ua).max() < 1e-9 * ua.max()
