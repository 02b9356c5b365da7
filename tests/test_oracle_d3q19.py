"""Pins of the oracle's D3Q19 update: the same recursive reconstruction
restricted to the third-order Hermite content the 19-velocity lattice
supports.

Fixed by mathematics: the unique shell weights (exact rationals), fourth-
order isotropy (and the missing sixth-order moment that removes H_xyz),
the exact reproduction of every supported Hermite moment by the equilibrium
and non-equilibrium parts (rho, rho u, rho u u and the six third-order
combinations a_xxy +- a_yzz, a_xzz +- a_xyy, a_yyz +- a_xxz), fixed
points, closed-form relaxation, conservation, an independent population
push, the 48 cube symmetries and the closed-form shear eigenvalue."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import workloads as W

CS2 = 1.0 / 3.0
L19 = 19
PAIRS = (((0, 0, 1), (1, 2, 2)), ((0, 2, 2), (0, 1, 1)), ((1, 1, 2), (0, 0, 2)))


def test_weights_are_the_unique_shell_set(oracle):
    c, w, opp = oracle.lattice(L19)
    assert c.shape == (19, 3)
    assert sorted(map(tuple, c.tolist())) == sorted(v for v in itertools.product((-1, 0, 1), repeat=3)
                                                  if sum(map(abs, v)) <= 2)
    # shells 0, 1, 2: W0 + 6 W1 + 12 W2 = 1, 2 W1 + 8 W2 = 1/3, 4 W2 = 1/9
    W2 = Fraction(1, 36)
    W1 = (Fraction(1, 3) - 8 * W2) / 2
    W0 = 1 - 6 * W1 - 12 * W2
    assert (W0, W1, W2) == (Fraction(1, 3), Fraction(1, 18), Fraction(1, 36))
    for i in range(19):
        assert w[i] == pytest.approx(float((W0, W1, W2)[int(np.abs(c[i]).sum())]), rel=1e-15)
        assert (c[opp[i]] == -c[i]).all()


def test_isotropy_and_the_missing_sixth_moment(oracle):
    c, w, _ = oracle.lattice(L19)
    d = np.eye(3)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), CS2 * d, atol=1e-15)
    iso4 = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                       + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), iso4, atol=1e-15)
    # no corners: sum w cx^2 cy^2 cz^2 = 0 instead of cs2^3, so H_xyz is zero
    assert np.einsum("i,i,i,i->", w, c[:, 0] ** 2, c[:, 1] ** 2, c[:, 2] ** 2) == 0.0
    assert all(oracle.hermite(i, 3, 0, 1, 2, lattice=L19) == 0.0 for i in range(19))


def _H3(oracle, a, b, g):
    return np.array([oracle.hermite(i, 3, a, b, g, lattice=L19) for i in range(19)])


@pytest.mark.parametrize("seed", [0, 1])
def test_supported_hermite_moments_are_reproduced(oracle, seed):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.05 * rng.standard_normal()
    u = 0.08 * rng.standard_normal(3)
    pi6 = 2e-3 * rng.standard_normal(6)
    P = np.array([[pi6[0], pi6[3], pi6[4]], [pi6[3], pi6[1], pi6[5]], [pi6[4], pi6[5], pi6[2]]])
    c, w, _ = oracle.lattice(L19)
    fe = np.array([oracle.feq(i, rho, u, 3, lattice=L19) for i in range(19)])
    fn = np.array([oracle.fneq(i, pi6, u, 3, lattice=L19) for i in range(19)])
    H2 = np.einsum("ia,ib->iab", c, c) - CS2 * np.eye(3)
    assert fe.sum() == pytest.approx(rho, rel=1e-14)
    assert np.allclose(fe @ c, rho * u, rtol=1e-13, atol=1e-17)
    assert np.allclose(np.einsum("i,iab->ab", fe, H2), rho * np.outer(u, u), rtol=1e-12, atol=1e-16)
    assert abs(fn.sum()) < 1e-16 and np.allclose(fn @ c, 0.0, atol=1e-16)
    assert np.allclose(np.einsum("i,iab->ab", fn, H2), P, rtol=1e-12, atol=1e-17)
    a3e = rho * np.einsum("a,b,g->abg", u, u, u)
    a3n = np.einsum("ab,g->abg", P, u) + np.einsum("bg,a->abg", P, u) + np.einsum("ag,b->abg", P, u)
    for p, q in PAIRS:
        hp = _H3(oracle, *p) + _H3(oracle, *q)
        hm = _H3(oracle, *p) - _H3(oracle, *q)
        for f, a3 in ((fe, a3e), (fn, a3n)):
            assert f @ hp == pytest.approx(a3[p] + a3[q], rel=1e-11, abs=1e-17)
            assert f @ hm == pytest.approx(a3[p] - a3[q], rel=1e-11, abs=1e-17)


@pytest.mark.parametrize("order", [3, 2])
def test_fixed_point_relaxation_and_conservation(oracle, order):
    G = oracle.make_grid(4, 5, 3, 0.7, order=order, lattice=L19)
    st = W.rest_state(G.shape)
    st[0] = 1.1
    st[1:4] = np.array([0.05, -0.03, 0.02])[:, None, None, None]
    assert np.abs(oracle.step(G, st) - st).max() < 1e-15
    st[4:] = np.array([1e-3, -2e-3, 5e-4, 7e-4, -3e-4, 2e-4])[:, None, None, None]
    want = st.copy()
    want[4:] *= 1.0 - 1.0 / 0.7
    assert np.abs(oracle.step(G, st) - want).max() < 1e-15
    rnd = W.random_state(G.shape, seed=31)
    g = W.random_force(G.shape, seed=32, amp=1e-4)
    r0, _ = oracle.reduce(G, rnd)
    r1, _ = oracle.reduce(G, oracle.step(G, rnd, g))
    assert abs(r1[0] - r0[0]) < 1e-12 * r0[0]
    assert np.allclose(r1[1:4] - r0[1:4], (rnd[0] * g).sum(axis=(1, 2, 3)), rtol=0, atol=1e-15)


def _push_reference(oracle, G, st, g):
    c, w, opp = oracle.lattice(L19)
    nz, ny, nx = G.shape
    kinds = oracle.node_kinds(G)
    omega = 1.0 / G.tau
    fin = np.zeros((19,) + G.shape)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        if kinds[z, y, x] != 0:
            continue
        for i in range(19):
            f = oracle.fpost(i, st[:, z, y, x], g[:, z, y, x], omega, G.order, lattice=L19)
            X, Y, Z = (x + c[i, 0]) % nx, (y + c[i, 1]) % ny, (z + c[i, 2]) % nz
            if kinds[Z, Y, X] == 1:
                fin[opp[i], z, y, x] += f
            else:
                fin[i, Z, Y, X] += f
    out = st.copy()
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        if kinds[z, y, x] == 0:
            out[:, z, y, x] = oracle.moments(fin[:, z, y, x], lattice=L19)
    return out


@pytest.mark.parametrize("order", [3, 2])
@pytest.mark.parametrize("faces", [(0,) * 6, (0, 0, 1, 1, 0, 0), (1, 1, 0, 0, 1, 1)])
def test_pull_update_matches_population_push(oracle, faces, order):
    G = oracle.make_grid(4, 5, 6, 0.66, faces=faces, order=order, lattice=L19)
    st = W.random_state(G.shape, seed=33)
    g = W.random_force(G.shape, seed=34, amp=1e-4)
    want = _push_reference(oracle, G, st, g)
    got = oracle.step(G, st, g)
    kinds = oracle.node_kinds(G)
    assert np.abs((got - want)[:, kinds == 0]).max() < 1e-15


def _rotate(st, perm, sign):
    arr = st.transpose(0, 3, 2, 1)
    arr = np.transpose(arr, (0,) + tuple(1 + p for p in perm))
    for a in range(3):
        if sign[a] < 0:
            arr = np.roll(np.flip(arr, axis=1 + a), 1, axis=1 + a)
    arr = arr.transpose(0, 3, 2, 1)
    out = np.empty_like(arr)
    out[0] = arr[0]
    R = np.zeros((3, 3))
    for a in range(3):
        R[a, perm[a]] = sign[a]
    out[1:4] = np.einsum("ab,bzyx->azyx", R, arr[1:4])
    idx = {(0, 0): 4, (1, 1): 5, (2, 2): 6, (0, 1): 7, (0, 2): 8, (1, 2): 9}
    P = np.zeros((3, 3) + arr.shape[1:])
    for (a, b), q in idx.items():
        P[a, b] = arr[q]
        P[b, a] = arr[q]
    P2 = np.einsum("ac,bd,cdzyx->abzyx", R, R, P)
    for (a, b), q in idx.items():
        out[q] = P2[a, b]
    return out


def test_cube_symmetry_equivariance(oracle):
    G = oracle.make_grid(4, 4, 4, 0.58, lattice=L19)
    st = W.random_state(G.shape, seed=35, u_amp=0.05, pi_amp=3e-3)
    base = oracle.step(G, st)
    worst = 0.0
    for perm in itertools.permutations(range(3)):
        for sign in itertools.product((1, -1), repeat=3):
            worst = max(worst, np.abs(oracle.step(G, _rotate(st, perm, sign)) - _rotate(base, perm, sign)).max())
    assert worst < 1e-15


def test_shear_wave_closed_form_eigenvalue(oracle):
    """The y-marginal of the D3Q19 weights is the same three-point set as for
    D3Q27, so the linear shear map is the same."""
    n, tau, A, steps = 32, 0.8, 1e-6, 50
    om = 1.0 / tau
    k = 2 * np.pi / n
    M = np.array([[(2 + np.cos(k)) / 3, (1 - om) * np.sin(k)], [-np.sin(k) / 3, (1 - om) * np.cos(k)]])
    G = oracle.make_grid(1, n, 1, tau, lattice=L19)
    y = np.arange(n)
    st = W.rest_state(G.shape)
    st[1, 0, :, 0] = A * np.sin(k * y)
    v = np.array([A, 0.0])
    for _ in range(steps):
        st = oracle.step(G, st)
        v = M @ v
    amp = 2 * (st[1, 0, :, 0] * np.sin(k * y)).sum() / n
    assert amp == pytest.approx(v[0], rel=1e-8)


@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_poiseuille_between_halfway_walls(oracle, tau):
    """The D3Q27 steady Poiseuille profile (its y-marginal weights are the
    same): u(y) = g/(2 nu) [(y - 1/2)(ny - 3/2 - y) - 1/4] + g/2."""
    ny, g = 12, 1e-6
    G = oracle.make_grid(1, ny, 1, tau, faces=(0, 0, 1, 1, 0, 0), force=(g, 0, 0), lattice=L19)
    out = oracle.run(G, W.rest_state(G.shape), 6000)
    nu = (tau - 0.5) / 3.0
    y = np.arange(1, ny - 1)
    ua = g / (2 * nu) * ((y - 0.5) * (ny - 1.5 - y) - 0.25) + g / 2
    assert np.abs(out[1, 0, 1:-1, 0] - ua).max() < 1e-9 * ua.max()
