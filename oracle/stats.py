"""Velocity statistics of the turbulence benchmarks, written out from their
definitions.  TEST INFRASTRUCTURE ONLY: used by tests/ to check the on-device
statistics of the HIP library; nothing in the product imports this module.

Channel (Section 3.1): averages over the homogeneous directions and over
time give, for every wall-normal position, the mean velocity U_a, the
second-order moments <u'_a u'_b> (normalised by u_tau^2 they are S_2,ab)
and the third-order moments <u'_a^3>, whose ratio to <u'_a^2>^(3/2) is the
skewness S_3,a.

Jet (Section 3.2): from the time-averaged axial velocity, the centreline
value U_c of every cross-section and the half-width r_1/2, the radius where
the azimuthally averaged mean axial velocity falls to U_c / 2.

All sums are plain float64 numpy reductions over the samples given.
"""
import numpy as np

PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def profile_sums(samples, axis, mask):
    """Raw sums along a profile axis (0 = x, 1 = y, 2 = z).

    samples: iterable of (3, nz, ny, nx) velocity fields (one per time level)
    mask:    (nz, ny, nx) bool, the nodes that count (fluid nodes)
    Returns (n_axis, 13) float64: for every index j along the axis, summed
    over the nodes of plane j and over the samples, the columns
      0        count
      1..3     u_a
      4..9     u_a u_b for (a, b) in xx, yy, zz, xy, xz, yz
      10..12   u_a^3
    """
    np_axis = 2 - axis  # array axes are (z, y, x)
    other = tuple(k for k in range(3) if k != np_axis)
    out = None
    for u in samples:
        u = np.asarray(u, dtype=np.float64)
        cols = [mask.astype(np.float64)]
        cols += [u[a] * mask for a in range(3)]
        cols += [u[a] * u[b] * mask for a, b in PAIRS]
        cols += [u[a] ** 3 * mask for a in range(3)]
        s = np.stack([c.sum(axis=other) for c in cols], axis=1)
        out = s if out is None else out + s
    return out


def profile_moments(sums):
    """Mean U (n, 3), central second moments <u'_a u'_b> (n, 6, PAIRS order)
    and central third moments <u'_a^3> (n, 3) from profile sums."""
    n = sums[:, 0:1]
    m1 = sums[:, 1:4] / n
    m2 = sums[:, 4:10] / n
    m3 = sums[:, 10:13] / n
    c2 = np.stack([m2[:, k] - m1[:, a] * m1[:, b] for k, (a, b) in enumerate(PAIRS)], axis=1)
    # <(u - U)^3> = <u^3> - 3 U <u^2> + 2 U^3
    c3 = np.stack([m3[:, a] - 3.0 * m1[:, a] * m2[:, a] + 2.0 * m1[:, a] ** 3 for a in range(3)], axis=1)
    return m1, c2, c3


def s2(c2, u_tau):
    """S_2,ab = <u'_a u'_b> / u_tau^2 (Section 3.1)."""
    return c2 / u_tau ** 2


def s3(c2, c3):
    """S_3,a = <u'_a^3> / <u'_a^2>^(3/2) (Section 3.1)."""
    return c3 / c2[:, 0:3] ** 1.5


def field_sums(samples):
    """Per-node sums over the samples of u_a (3, ...) and u_a u_b (6, ...)."""
    s1 = s2_ = None
    for u in samples:
        u = np.asarray(u, dtype=np.float64)
        a = u.copy()
        b = np.stack([u[i] * u[j] for i, j in PAIRS])
        s1 = a if s1 is None else s1 + a
        s2_ = b if s2_ is None else s2_ + b
    return s1, s2_


def jet_axis(mean_axial, center, axis=2):
    """Centreline velocity and half-width of every cross-section.

    mean_axial: (nz, ny, nx) time-averaged velocity along `axis`
    center:     (c1, c2) coordinates of the jet axis in the two transverse
                directions, in x, y, z order
    Bins: the nodes of a cross-section are grouped by k = floor(r), r their
    distance to the axis; bin k has mean radius rbar_k and mean axial
    velocity P_k.  U_c = P_0 (the nodes within one spacing of the axis);
    r_1/2 interpolates linearly between the first bin k >= 1 with
    P_k <= U_c / 2 and bin k - 1 (-1 when the profile never falls that far).
    Returns (uc, rhalf), one value per cross-section.
    """
    arr = np.moveaxis(np.asarray(mean_axial, dtype=np.float64), 2 - axis, 0)  # (n_axis, t2, t1)
    n_axis, n2, n1 = arr.shape
    t1, t2 = np.meshgrid(np.arange(n1), np.arange(n2))
    r = np.sqrt((t1 - center[0]) ** 2 + (t2 - center[1]) ** 2)
    k = np.floor(r).astype(np.int64)
    nb = k.max() + 1
    cnt = np.bincount(k.ravel(), minlength=nb).astype(np.float64)
    rbar = np.bincount(k.ravel(), weights=r.ravel(), minlength=nb) / np.maximum(cnt, 1)
    uc = np.empty(n_axis)
    rh = np.empty(n_axis)
    for j in range(n_axis):
        prof = np.bincount(k.ravel(), weights=arr[j].ravel(), minlength=nb) / np.maximum(cnt, 1)
        uc[j] = prof[0]
        half = 0.5 * prof[0]
        rh[j] = -1.0
        for b in range(1, nb):
            if cnt[b] > 0 and prof[b] <= half:
                pb = b - 1
                while cnt[pb] == 0:
                    pb -= 1
                rh[j] = rbar[pb] + (rbar[b] - rbar[pb]) * (prof[pb] - half) / (prof[pb] - prof[b])
                break
    return uc, rh
