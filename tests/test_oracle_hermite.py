"""Pins of the oracle's lattice, Hermite tensors and per-population formulas.

Each check is fixed by mathematics, not by the oracle itself: the weights are
the unique isotropic shell weights (solved here in exact rationals), the
Hermite tensors must be orthogonal under those weights, and projecting the
oracle's equilibrium / non-equilibrium populations back onto the Hermite
basis must return the coefficients of the recursion of Section 2.2
(a^n_eq = rho u^n; a^2_neq = Pi, a^3_neq = Pi u symmetrised).
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

CS2 = 1.0 / 3.0


def _shell_weights_exact():
    """Solve the isotropy conditions for the four D3Q27 shells in rationals:
    sum w = 1, sum w cx^2 = 1/3, sum w cx^2 cy^2 = 1/9, sum w cx^2 cy^2 cz^2 = 1/27."""
    vel = list(itertools.product((-1, 0, 1), repeat=3))
    rows, rhs = [], [Fraction(1), Fraction(1, 3), Fraction(1, 9), Fraction(1, 27)]
    feats = [lambda c: 1, lambda c: c[0] ** 2, lambda c: c[0] ** 2 * c[1] ** 2,
             lambda c: c[0] ** 2 * c[1] ** 2 * c[2] ** 2]
    for f in feats:
        row = [Fraction(0)] * 4
        for c in vel:
            row[sum(abs(x) for x in c)] += f(c)
        rows.append(row)
    # Gaussian elimination in exact arithmetic
    n = 4
    A = [rows[i] + [rhs[i]] for i in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        for r in range(n):
            if r != col and A[r][col] != 0:
                fac = A[r][col] / A[col][col]
                A[r] = [a - fac * b for a, b in zip(A[r], A[col])]
    return [A[i][n] / A[i][i] for i in range(n)]


def test_weights_are_the_unique_isotropic_set(oracle):
    c, w, opp = oracle.lattice()
    ws = _shell_weights_exact()
    assert ws == [Fraction(8, 27), Fraction(2, 27), Fraction(1, 54), Fraction(1, 216)]
    for i in range(27):
        shell = int(np.abs(c[i]).sum())
        assert w[i] == pytest.approx(float(ws[shell]), rel=1e-15, abs=0)
    assert sorted(map(tuple, c.tolist())) == sorted(itertools.product((-1, 0, 1), repeat=3))
    for i in range(27):
        assert (c[opp[i]] == -c[i]).all()


def test_lattice_isotropy_to_fourth_order(oracle):
    c, w, _ = oracle.lattice()
    d = np.eye(3)
    assert np.sum(w) == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(np.einsum("i,ia->a", w, c), 0.0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), CS2 * d, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0.0, atol=1e-16)
    iso4 = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                       + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), iso4, atol=1e-15)
    assert np.einsum("i,i,i,i->", w, c[:, 0] ** 2, c[:, 1] ** 2, c[:, 2] ** 2) == pytest.approx(CS2 ** 3)


def _H(oracle, order):
    """All components of the oracle's Hermite tensor of one order, per velocity."""
    out = np.zeros((27,) + (3,) * order)
    for i in range(27):
        for idx in itertools.product(range(3), repeat=order):
            a = idx + (0,) * (3 - order)
            out[(i,) + idx] = oracle.hermite(i, order, *a)
    return out


def test_hermite_tensors_match_definition_and_are_orthogonal(oracle):
    c, w, _ = oracle.lattice()
    H = [_H(oracle, n) for n in range(4)]
    d = np.eye(3)
    # the definitions (Section 2.2) built here from c, independently of the oracle
    assert np.allclose(H[1], c)
    assert np.allclose(H[2], np.einsum("ia,ib->iab", c, c) - CS2 * d)
    h3 = (np.einsum("ia,ib,ig->iabg", c, c, c) - CS2 * (np.einsum("ig,ab->iabg", c, d)
          + np.einsum("ia,bg->iabg", c, d) + np.einsum("ib,ag->iabg", c, d)))
    assert np.allclose(H[3], h3)
    # H_xxx vanishes on every D3Q27 velocity because c^3 = c there
    assert np.allclose(H[3][:, 0, 0, 0], 0.0) and np.allclose(H[3][:, 2, 2, 2], 0.0)
    # mutual orthogonality of orders 0..3 under the weights
    for m in range(4):
        for n in range(m + 1, 4):
            prod = np.einsum("i,i...,i...->...", w, H[m].reshape(27, -1)[:, :, None],
                             H[n].reshape(27, -1)[:, None, :])
            assert np.allclose(prod, 0.0, atol=1e-15), (m, n)
    # second-order normalisation: sum w H2_ab H2_cd = cs4 (d_ac d_bd + d_ad d_bc)
    g2 = np.einsum("i,iab,icd->abcd", w, H[2], H[2])
    assert np.allclose(g2, CS2 ** 2 * (np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)))
    # third-order norms of the two supported families
    assert np.einsum("i,i,i->", w, H[3][:, 0, 0, 1], H[3][:, 0, 0, 1]) == pytest.approx(2 * CS2 ** 3)
    assert np.einsum("i,i,i->", w, H[3][:, 0, 1, 2], H[3][:, 0, 1, 2]) == pytest.approx(CS2 ** 3)


@pytest.mark.parametrize("order", [3, 2])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_equilibrium_hermite_coefficients(oracle, seed, order):
    """Order 3: Eq. (eqts); order 2: Eq. (lbequil), whose third-order
    Hermite coefficients vanish."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.1 * rng.standard_normal()
    u = 0.1 * rng.standard_normal(3)
    c, w, _ = oracle.lattice()
    f = np.array([oracle.feq(i, rho, u, order) for i in range(27)])
    H2 = _H(oracle, 2)
    H3 = _H(oracle, 3)
    assert f.sum() == pytest.approx(rho, rel=1e-14)
    assert np.allclose(f @ c, rho * u, rtol=1e-13, atol=1e-16)
    # raw second moment: rho u u + rho cs2 delta (Navier-Stokes pressure term)
    assert np.allclose(np.einsum("i,ia,ib->ab", f, c, c), rho * np.outer(u, u) + rho * CS2 * np.eye(3),
                       rtol=1e-13, atol=1e-16)
    # Hermite coefficients: a2 = rho u u, a3 = rho u u u on the supported set
    assert np.allclose(np.einsum("i,iab->ab", f, H2), rho * np.outer(u, u), rtol=1e-12, atol=1e-16)
    a3 = np.einsum("i,iabg->abg", f, H3)
    for (a, b, g) in itertools.product(range(3), repeat=3):
        if len({a, b, g}) == 1 or order == 2:
            assert a3[a, b, g] == pytest.approx(0.0, abs=1e-15)  # Q_xxx not supported / not kept
        else:
            assert a3[a, b, g] == pytest.approx(rho * u[a] * u[b] * u[g], rel=1e-11, abs=1e-15)


@pytest.mark.parametrize("order", [3, 2])
@pytest.mark.parametrize("seed", [3, 4])
def test_nonequilibrium_hermite_coefficients(oracle, seed, order):
    rng = np.random.default_rng(seed)
    u = 0.1 * rng.standard_normal(3)
    pi6 = 1e-2 * rng.standard_normal(6)
    P = np.array([[pi6[0], pi6[3], pi6[4]], [pi6[3], pi6[1], pi6[5]], [pi6[4], pi6[5], pi6[2]]])
    c, w, _ = oracle.lattice()
    f = np.array([oracle.fneq(i, pi6, u, order) for i in range(27)])
    H2 = _H(oracle, 2)
    H3 = _H(oracle, 3)
    assert abs(f.sum()) < 1e-17
    assert np.allclose(f @ c, 0.0, atol=1e-17)
    assert np.allclose(np.einsum("i,iab->ab", f, H2), P, rtol=1e-12, atol=1e-17)
    a3 = np.einsum("i,iabg->abg", f, H3)
    for (a, b, g) in itertools.product(range(3), repeat=3):
        want = 0.0 if (len({a, b, g}) == 1 or order == 2) else P[a, b] * u[g] + P[b, g] * u[a] + P[a, g] * u[b]
        assert a3[a, b, g] == pytest.approx(want, rel=1e-11, abs=1e-15)


def test_post_collision_population_and_forcing(oracle):
    """fpost = feq + (1 - omega) fneq + w rho c.g / cs2: its moments are rho,
    rho u + rho g, and the second Hermite coefficient rho u u + (1 - omega) Pi."""
    rng = np.random.default_rng(5)
    m = np.concatenate([[1.02], 0.05 * rng.standard_normal(3), 1e-3 * rng.standard_normal(6)])
    g = 1e-4 * rng.standard_normal(3)
    omega = 1.0 / 0.7
    c, w, _ = oracle.lattice()
    f = np.array([oracle.fpost(i, m, g, omega) for i in range(27)])
    rho, u = m[0], m[1:4]
    P = np.array([[m[4], m[7], m[8]], [m[7], m[5], m[9]], [m[8], m[9], m[6]]])
    H2 = _H(oracle, 2)
    assert f.sum() == pytest.approx(rho, rel=1e-14)
    assert np.allclose(f @ c, rho * u + rho * g, rtol=1e-12, atol=1e-17)
    assert np.allclose(np.einsum("i,iab->ab", f, H2), rho * np.outer(u, u) + (1 - omega) * P,
                       rtol=1e-11, atol=1e-16)


def test_moments_inverse_of_reconstruction(oracle):
    """Moments of feq + fneq at (rho, u, Pi) return exactly (rho, u, Pi)."""
    rng = np.random.default_rng(6)
    rho = 0.97
    u = 0.04 * rng.standard_normal(3)
    pi6 = 1e-3 * rng.standard_normal(6)
    f = np.array([oracle.feq(i, rho, u) + oracle.fneq(i, pi6, u) for i in range(27)])
    m = oracle.moments(f)
    assert m[0] == pytest.approx(rho, rel=1e-15)
    assert np.allclose(m[1:4], u, rtol=1e-12, atol=1e-17)
    assert np.allclose(m[4:], pi6, rtol=1e-10, atol=1e-16)
