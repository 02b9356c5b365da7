"""Pins of the statistics oracle (oracle/stats.py): the channel moments of
Section 3.1 and the jet diagnostics of Section 3.2 on fields whose answers
are known in closed form."""
import numpy as np
import pytest

from oracle import stats as S


def _two_point_field(nx, ny, nz):
    """u_x' takes +4 on 2 of every 10 x positions and -1 on the other 8
    (zero mean, <u'^2> = 4, <u'^3> = 12, skewness 1.5); u_y' = -u_x' / 2;
    the mean profile U_x(y) = 0.01 y is added on top."""
    assert nx % 10 == 0
    pat = np.where(np.arange(nx) % 10 < 2, 4.0, -1.0)
    u = np.zeros((3, nz, ny, nx))
    u[0] = pat[None, None, :] + 0.01 * np.arange(ny)[None, :, None]
    u[1] = -0.5 * pat[None, None, :]
    return u


def test_channel_moments_closed_form():
    u = _two_point_field(20, 7, 5)
    mask = np.ones(u.shape[1:], dtype=bool)
    sums = S.profile_sums([u], axis=1, mask=mask)
    assert sums.shape == (7, 13)
    assert np.all(sums[:, 0] == 100.0)
    U, c2, c3 = S.profile_moments(sums)
    assert np.allclose(U[:, 0], 0.01 * np.arange(7), atol=1e-14)
    assert np.allclose(U[:, 1:], 0.0, atol=1e-15)
    assert np.allclose(c2[:, 0], 4.0, rtol=1e-13)            # <u'x u'x>
    assert np.allclose(c2[:, 1], 1.0, rtol=1e-13)            # <u'y u'y> = 4 / 4
    assert np.allclose(c2[:, 3], -2.0, rtol=1e-13)           # <u'x u'y> = -4 / 2
    assert np.allclose(c2[:, [2, 4, 5]], 0.0, atol=1e-15)
    assert np.allclose(c3[:, 0], 12.0, rtol=1e-12)
    assert np.allclose(c3[:, 1], -1.5, rtol=1e-12)           # (-1/2)^3 * 12
    sk = S.s3(c2, c3)
    assert np.allclose(sk[:, 0], 1.5, rtol=1e-12)
    assert np.allclose(sk[:, 1], -1.5, rtol=1e-12)
    assert np.allclose(S.s2(c2, 0.5)[:, 0], 16.0, rtol=1e-13)


def test_sine_wave_moments_and_time_average():
    """u_x = A sin(2 pi (x + t) / n): <u'^2> = A^2 / 2 and <u'^3> = 0 over a
    period, for every sample and for their average; a mask drops nodes."""
    n, A = 16, 0.3
    x = np.arange(n)
    samples = []
    for t in range(3):
        u = np.zeros((3, 4, 6, n))
        u[0] = A * np.sin(2 * np.pi * (x + t) / n)[None, None, :]
        samples.append(u)
    mask = np.ones((4, 6, n), dtype=bool)
    mask[:, 0, :] = False  # a wall row
    sums = S.profile_sums(samples, axis=1, mask=mask)
    assert sums[0, 0] == 0.0 and np.all(sums[1:, 0] == 3 * 4 * n)
    U, c2, c3 = S.profile_moments(sums[1:])
    assert np.allclose(U, 0.0, atol=1e-15)
    assert np.allclose(c2[:, 0], A * A / 2, rtol=1e-13)
    assert np.allclose(c3[:, 0], 0.0, atol=1e-15)
    # the same sums along z (every z plane sees the whole wave)
    sz = S.profile_sums(samples, axis=2, mask=mask)
    assert np.allclose(S.profile_moments(sz)[1][:, 0], A * A / 2, rtol=1e-13)


def test_field_sums_are_per_node_time_sums():
    rng = np.random.default_rng(3)
    samples = [rng.standard_normal((3, 2, 3, 4)) for _ in range(5)]
    s1, s2 = S.field_sums(samples)
    assert np.allclose(s1, sum(samples), rtol=1e-14)
    assert np.allclose(s2[3], sum(u[0] * u[1] for u in samples), rtol=1e-14)


@pytest.mark.parametrize("center", [(30.0, 30.0), (29.5, 31.5)])
def test_jet_half_width_of_a_cone_is_exact(center):
    """A linear (cone) profile U (1 - r / (2R)): the mean over any bin is the
    profile at the bin's mean radius, so the interpolated half-width is R
    exactly, whatever the binning."""
    R, U = 17.0, 0.05
    ny, nx, nz = 61, 61, 3
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((xx - center[0]) ** 2 + (yy - center[1]) ** 2)
    prof = U * (1.0 - r / (2 * R))
    field = np.broadcast_to(prof, (nz, ny, nx)) * np.array([1.0, 0.5, 2.0])[:, None, None]
    uc, rh = S.jet_axis(field, center, axis=2)
    rbin0 = r[r < 1].mean()
    assert np.allclose(uc, U * (1 - rbin0 / (2 * R)) * np.array([1.0, 0.5, 2.0]), rtol=1e-13)
    # the half of U_c, not of U: solve U (1 - r/2R) = U_c / 2 for r
    want = 2 * R * (1 - 0.5 * (1 - rbin0 / (2 * R)))
    assert np.allclose(rh, want, rtol=1e-12)


def test_jet_half_width_of_a_gaussian():
    """A Gaussian U exp(-r^2 / (2 s^2)) centred on a node: U_c = U and
    r_1/2 = s sqrt(2 ln 2) up to the binning (second-order in 1/s)."""
    n = 121
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    errs = []
    for s in (8.0, 16.0, 32.0):
        r2 = (xx - 60.0) ** 2 + (yy - 60.0) ** 2
        f = np.exp(-r2 / (2 * s * s))[None]
        uc, rh = S.jet_axis(f, (60.0, 60.0), axis=2)
        assert uc[0] == 1.0
        errs.append(abs(rh[0] / (s * np.sqrt(2 * np.log(2))) - 1))
    assert errs[0] < 0.02 and errs[2] < errs[0]


def test_jet_axis_along_x():
    """Transverse axes in x, y, z order: for a jet along x they are (y, z)."""
    nz, ny, nx = 41, 31, 5
    zz, yy = np.meshgrid(np.arange(nz), np.arange(ny), indexing="ij")
    r = np.sqrt((yy - 12.0) ** 2 + (zz - 20.0) ** 2)
    f = np.broadcast_to((1.0 - r / 20.0)[:, :, None], (nz, ny, nx))
    uc, rh = S.jet_axis(f, (12.0, 20.0), axis=0)
    assert uc.shape == (nx,) and np.allclose(uc, 1.0)
    assert np.allclose(rh, 10.0, rtol=1e-12)


def test_profile_that_never_halves():
    f = np.ones((2, 9, 9))
    uc, rh = S.jet_axis(f, (4.0, 4.0), axis=2)
    assert np.all(uc == 1.0) and np.all(rh == -1.0)
