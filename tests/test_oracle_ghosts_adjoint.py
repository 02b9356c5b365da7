"""Pins of the oracle's ghost layers (Section 2.3), inlet random numbers,
storage rounding, and its tangent and adjoint.

- The ghost rule is checked value by value against its definition; the
  random stream against the published SplitMix64 outputs.
- Binary16 / bfloat16 rounding is checked against numpy's and torch's
  conversions (library routines) on inputs where they are exact references.
- The adjoint is pinned twice: by the dot-product identity against the
  complex-step tangent of the whole step, and by central finite differences
  in FP64 of the kinetic-energy loss through a short rollout.
"""
import os

import numpy as np
import pytest

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def test_splitmix64_published_outputs(oracle):
    rows = [ln.split() for ln in open(os.path.join(HERE, "golden", "splitmix64_seed0.txt"))
            if ln.strip() and not ln.startswith("#")]
    for k, hexval in rows:
        assert oracle.splitmix64(0, int(k)) == int(hexval, 16)


def test_inlet_variate_bits(oracle):
    """xi = 2 * (top 24 bits of output k) / 2^24 - 1, k = 1 + 3 (t N + n) + a."""
    seed, N = 987654321, 1000
    for (t, n, a) in [(0, 0, 0), (3, 17, 2), (1999, 999, 1)]:
        k = 1 + 3 * (t * N + n) + a
        h = oracle.splitmix64(seed, k)
        assert oracle.inlet_xi(seed, t, n, N, a) == (h >> 40) / 2.0 ** 24 * 2 - 1
    xs = np.array([oracle.inlet_xi(seed, 5, n, N, 0) for n in range(4000)])
    assert xs.min() >= -1 and xs.max() < 1 and abs(xs.mean()) < 0.05


def test_ghost_fill_rule(oracle):
    case = W.jet_case(nx=9, ny=12, nz=11, D=4.0)
    G = oracle.make_grid(case.nx, case.ny, case.nz, case.tau, faces=case.faces, inlet_u=case.inlet_u,
                         inlet_center=case.inlet_center, inlet_radius=case.inlet_radius,
                         inlet_noise=case.inlet_noise, seed=case.seed)
    st = W.random_state(G.shape, seed=21)
    t = 7
    out = oracle.ghost_fill(G, st, t)
    kinds = oracle.node_kinds(G)
    nz, ny, nx = G.shape
    N = G.n
    U = np.array(case.inlet_u)
    amp = case.inlet_noise * np.linalg.norm(U)
    n_inlet = 0
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if kinds[z, y, x] == 0:
                    assert np.array_equal(out[:, z, y, x], st[:, z, y, x])
                    continue
                xf, yf, zf = min(max(x, 1), nx - 2), min(max(y, 1), ny - 2), min(max(z, 1), nz - 2)
                src = st[:, zf, yf, xf]
                r2 = (y - case.inlet_center[0]) ** 2 + (z - case.inlet_center[1]) ** 2
                if x == 0 and r2 <= case.inlet_radius ** 2:
                    n_inlet += 1
                    n = x + nx * (y + ny * z)
                    ub = U + amp * np.array([oracle.inlet_xi(case.seed, t, n, N, a) for a in range(3)])
                    assert out[0, z, y, x] == src[0]
                    assert np.array_equal(out[4:, z, y, x], src[4:])
                    assert np.allclose(out[1:4, z, y, x], ub, rtol=0, atol=1e-17)
                    assert np.all(np.abs(out[1:4, z, y, x] - U) <= amp)
                else:
                    assert np.array_equal(out[:, z, y, x], src)
    # lattice points of the disc (y - 5.5)^2 + (z - 5)^2 <= 4: dy = +-0.5, +-1.5 with |dz| <= 1
    assert n_inlet == 12


def test_ghost_layers_do_not_leak_mass_when_uniform(oracle):
    """A uniform rest state with zero-gradient ghosts everywhere is a fixed point."""
    G = oracle.make_grid(6, 7, 5, 0.51, faces=(3,) * 6)
    st = oracle.ghost_fill(G, W.rest_state(G.shape), 0)
    out = oracle.run(G, st, 5)
    assert np.abs(out - st).max() < 1e-15


def test_fp16_rounding_matches_numpy(oracle):
    rng = np.random.default_rng(22)
    xs = np.concatenate([rng.standard_normal(3000) * 10.0 ** rng.integers(-9, 5, 3000),
                         [0.0, 6.1e-5, 5.96e-8, 2.98e-8, 65504.0, 65519.0, 65520.0, -1e-9]])
    for x in xs:
        assert oracle.round_fp16(x) == float(np.float64(x).astype(np.float16)), x


def test_bf16_rounding_matches_torch(oracle):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(23)
    xs = (rng.standard_normal(3000) * 10.0 ** rng.integers(-30, 30, 3000)).astype(np.float32)
    ref = torch.from_numpy(xs).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([oracle.round_bf16(float(x)) for x in xs])
    assert np.array_equal(got, ref)


def test_storage_rounding_emulation(oracle):
    G = oracle.make_grid(3, 3, 3, 0.7)
    st = W.random_state(G.shape, seed=24)
    sc = (2.0 ** 10, 2.0 ** 12, 2.0 ** 16)
    r = oracle.round_storage(G, st, 1, sc)
    assert np.array_equal(((r[0] - 1) * sc[0]).astype(np.float16).astype(np.float64), (r[0] - 1) * sc[0])
    assert np.array_equal((r[4:] * sc[2]).astype(np.float16).astype(np.float64), r[4:] * sc[2])
    assert np.abs(r[1:4] - st[1:4]).max() <= 2.0 ** -11 * 0.03


@pytest.mark.parametrize("sponge", [False, True])
@pytest.mark.parametrize("faces", [(0,) * 6, (0, 0, 1, 1, 0, 0)])
def test_adjoint_dot_product_identity(oracle, faces, sponge):
    """<lam, J v> = <J^T lam, v> with J v from the complex-step tangent (also
    with a relaxation time that varies from plane to plane)."""
    tau_z = [0.61, 0.7, 0.95, 1.4] if sponge else None
    G = oracle.make_grid(5, 6, 4, 0.61, faces=faces, tau_z=tau_z)
    st = W.random_state(G.shape, seed=25, u_amp=0.05, pi_amp=2e-3)
    g = W.random_force(G.shape, seed=26, amp=1e-4)
    rng = np.random.default_rng(27)
    v = rng.standard_normal(st.shape)
    dg = rng.standard_normal(g.shape)
    lam1 = rng.standard_normal(st.shape)
    kinds = oracle.node_kinds(G)
    lam1[:, kinds != 0] = 0.0  # the loss only sees fluid nodes
    jv = oracle.jvp_step(G, st, v, g, dg)
    lam0, gg = oracle.adjoint_step(G, st, lam1, g)
    lhs = (lam1 * jv).sum()
    rhs = (lam0 * v).sum() + (gg * dg).sum()
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_adjoint_nodes_match_full_adjoint(oracle):
    G = oracle.make_grid(4, 6, 5, 0.7, faces=(0, 0, 1, 1, 0, 0))
    st = W.random_state(G.shape, seed=28)
    lam1 = np.random.default_rng(29).standard_normal(st.shape)
    lam0, dg = oracle.adjoint_step(G, st, lam1)
    idx = np.arange(0, G.n, 7)
    lam_s, dg_s = oracle.adjoint_nodes(G, st, lam1, idx)
    assert np.allclose(lam_s, lam0.reshape(10, -1)[:, idx], rtol=1e-13, atol=1e-14)
    assert np.allclose(dg_s, dg.reshape(3, -1)[:, idx], rtol=1e-13, atol=1e-14)


def test_rollout_gradient_matches_central_differences(oracle):
    """FP64 central differences (h = 1e-4 relative) of L = 1/2 sum rho |u|^2
    after 8 steps, along random directions of g and of the initial velocity."""
    case = W.adjoint_case(n=6, steps=8)
    G = oracle.make_grid(case.nx, case.ny, case.nz, case.tau)
    st0, g = W.adjoint_inputs(case)
    g = g * 1e3  # a force large enough that its gradient is not round-off
    L, lam0, dg = oracle.rollout_grad(G, st0, case.steps, g)
    rng = np.random.default_rng(30)

    def loss(s, gf):
        return oracle.ke_seed(G, oracle.run(G, s, case.steps, gf))[0]

    for _ in range(2):
        d = rng.standard_normal(g.shape)
        h = 1e-4 * np.abs(g).max()
        fd = (loss(st0, g + h * d) - loss(st0, g - h * d)) / (2 * h)
        assert (dg * d).sum() == pytest.approx(fd, rel=1e-6)
        du = np.zeros_like(st0)
        du[1:4] = rng.standard_normal((3,) + G.shape)
        h = 1e-4 * np.abs(st0[1:4]).max()
        fd = (loss(st0 + h * du, g) - loss(st0 - h * du, g)) / (2 * h)
        assert (lam0 * du).sum() == pytest.approx(fd, rel=1e-6)


def test_uniform_flow_through_inlet_and_outlets_is_a_fixed_point(oracle):
    """Uniform flow U (any direction) with an inlet disc covering the whole
    inflow face that imposes U (no noise) and zero-gradient ghosts elsewhere:
    every ghost equals the interior, so the state must be reproduced exactly.
    A wrong sign, component or time level in the inlet fill breaks this."""
    U = np.array([0.04, -0.01, 0.015])
    for face in range(6):
        faces = [3] * 6
        faces[face] = 2
        G = oracle.make_grid(7, 6, 5, 0.6, faces=faces, inlet_u=U, inlet_center=(2.5, 2.5), inlet_radius=50.0,
                             inlet_noise=0.0, seed=3)
        st = W.rest_state(G.shape)
        st[0] = 1.01
        st[1:4] = U[:, None, None, None]
        st = oracle.ghost_fill(G, st, 0)
        out = oracle.run(G, st, 3)
        assert np.abs(out - st).max() < 1e-15, face
    # and a non-matching imposed velocity is not a fixed point
    G = oracle.make_grid(7, 6, 5, 0.6, faces=(2, 3, 3, 3, 3, 3), inlet_u=-U, inlet_center=(2.5, 2.5),
                         inlet_radius=50.0)
    st = W.rest_state(G.shape)
    st[1:4] = U[:, None, None, None]
    st = oracle.ghost_fill(G, st, 0)
    assert np.abs(oracle.run(G, st, 1) - st).max() > 1e-4


def test_gaussian_inlet_variates_are_standard_normal(oracle):
    """The Box-Muller variates of the time-varying Gaussian inlet noise
    (Section 3.2) follow N(0, 1): moments, the one-sigma mass, a
    Kolmogorov-Smirnov test, and no correlation between components or
    between consecutive levels."""
    from scipy import stats
    N = 5000
    xs = np.array([[oracle.inlet_gauss(99, t, n, N, a) for n in range(N) for t in range(8)] for a in range(3)])
    x = xs.ravel()
    m = x.size
    assert abs(x.mean()) < 5.0 / np.sqrt(m)
    assert abs(x.var() - 1.0) < 5.0 * np.sqrt(2.0 / m)
    assert abs(stats.kurtosis(x, fisher=False) - 3.0) < 5.0 * np.sqrt(24.0 / m)
    assert abs((np.abs(x) < 1.0).mean() - 0.682689) < 5.0 * np.sqrt(0.2166 / m)
    assert stats.kstest(x, "norm").pvalue > 1e-4
    for a, b in ((0, 1), (0, 2), (1, 2)):
        assert abs(np.corrcoef(xs[a], xs[b])[0, 1]) < 5.0 / np.sqrt(xs.shape[1])
    lag = xs[0].reshape(N, 8)
    assert abs(np.corrcoef(lag[:, :-1].ravel(), lag[:, 1:].ravel())[0, 1]) < 5.0 / np.sqrt(lag[:, 1:].size)


def test_gaussian_inlet_ghost_velocity(oracle):
    """Inlet-disc ghost nodes get u = U + noise |U| xi with the Gaussian xi
    of their (level, node, component); nodes off the disc get none."""
    U = (0.0, 0.0, 0.05)
    G = oracle.make_grid(9, 9, 6, 0.6, faces=(0, 0, 0, 0, 2, 3), inlet_u=U, inlet_center=(4.0, 4.0),
                         inlet_radius=2.5, inlet_noise=0.02, seed=5, noise_kind=1)
    st = oracle.ghost_fill(G, W.rest_state(G.shape), 3)
    kinds = oracle.node_kinds(G)
    hit = 0
    for y in range(9):
        for x in range(9):
            n = x + 9 * y
            if (x - 4) ** 2 + (y - 4) ** 2 <= 2.5 ** 2:
                hit += 1
                for a in range(3):
                    want = U[a] + 0.02 * 0.05 * oracle.inlet_gauss(5, 3, n, G.n, a)
                    assert st[1 + a, 0, y, x] == want
            else:
                assert np.all(st[1:4, 0, y, x] == 0.0)
    assert hit == 21 and kinds[0].max() == 2


def test_wall_shear_objective_of_poiseuille_flow(oracle):
    """Steady Poiseuille flow between half-way walls (y = 1/2, ny - 3/2) has
    sigma_xy = g (y_c - y) with y_c = (ny - 1)/2, so the x force the
    objective measures at the two wall-adjacent layers (y = 1, ny - 2) is
    2 A g (ny - 3) / 2 = g A (ny - 3) for A = nx nz nodes per layer; its
    gradient is -s (1 - omega/2) on Pi_xy of those layers only."""
    ny, g, tau = 12, 1e-6, 0.9
    G = oracle.make_grid(2, ny, 3, tau, faces=(0, 0, 1, 1, 0, 0), force=(g, 0, 0))
    out = oracle.run(G, W.rest_state(G.shape), 6000)
    L, lam = oracle.wall_shear_seed(G, out)
    assert L == pytest.approx(g * 2 * 3 * (ny - 3), rel=1e-9)
    k = 1.0 - 0.5 / tau
    assert np.all(lam[7, :, 1, :] == -k) and np.all(lam[7, :, ny - 2, :] == k)
    lam[7, :, 1, :] = 0.0
    lam[7, :, ny - 2, :] = 0.0
    assert np.all(lam == 0.0)


def test_wall_shear_rollout_gradient_matches_central_differences(oracle):
    """FP64 central differences of the wall shear objective after 8 steps of
    a small channel (walls on y and z) along random directions of the force
    field and of the initial velocity."""
    G = oracle.make_grid(5, 7, 6, 0.7, faces=(0, 0, 1, 1, 1, 1))
    st0 = W.random_state(G.shape, seed=41, u_amp=0.03, pi_amp=1e-3)
    g = W.random_force(G.shape, seed=42, amp=1e-3)
    L, lam0, dg = oracle.rollout_grad(G, st0, 8, g, objective=oracle.OBJ_WALL_SHEAR)
    rng = np.random.default_rng(43)

    def loss(s, gf):
        return oracle.wall_shear_seed(G, oracle.run(G, s, 8, gf))[0]

    assert L == pytest.approx(loss(st0, g), rel=1e-14)
    for _ in range(2):
        d = rng.standard_normal(g.shape)
        h = 1e-4 * np.abs(g).max()
        fd = (loss(st0, g + h * d) - loss(st0, g - h * d)) / (2 * h)
        assert (dg * d).sum() == pytest.approx(fd, rel=1e-6)
        du = np.zeros_like(st0)
        du[1:4] = rng.standard_normal((3,) + G.shape)
        h = 1e-4 * np.abs(st0[1:4]).max()
        fd = (loss(st0 + h * du, g) - loss(st0 - h * du, g)) / (2 * h)
        assert (lam0 * du).sum() == pytest.approx(fd, rel=1e-6)


def _small_jet(oracle, noise_kind=0):
    """7 x 6 x 5 nodes: inlet disc of radius 1.6 on x = 0, outflow ghosts on
    every other face; tau 0.62."""
    return oracle.make_grid(7, 6, 5, 0.62, faces=(2, 3, 3, 3, 3, 3), inlet_u=(0.04, 0.0, 0.0),
                            inlet_center=(2.5, 2.0), inlet_radius=1.6, inlet_noise=0.02, seed=31,
                            noise_kind=noise_kind)


@pytest.mark.parametrize("noise_kind", [0, 1])
def test_adjoint_dot_product_identity_with_ghost_layers(oracle, noise_kind):
    """<lam, J v> = <J^T lam, v> + <dL/dg, dg> through inflow and outflow
    ghost layers (Section 2.3): the tangent is the complex step of the whole
    step (update, then the refill of the new level), the adjoint folds the
    ghosts' sensitivities into the interior nodes they copy and treats the
    ghost values of level t as inputs.  Every node of v and lam is random,
    ghosts included."""
    G = _small_jet(oracle, noise_kind)
    kinds = oracle.node_kinds(G)
    assert (kinds == 2).sum() > 0 and (kinds == 0).sum() > 0
    st = oracle.ghost_fill(G, W.random_state(G.shape, seed=32, u_amp=0.04, pi_amp=1e-3), 3)
    g = W.random_force(G.shape, seed=33, amp=1e-4)
    rng = np.random.default_rng(34)
    v = rng.standard_normal(st.shape)
    dg = rng.standard_normal(g.shape)
    lam1 = rng.standard_normal(st.shape)
    jv = oracle.jvp_step(G, st, v, g, dg, t=3)
    lam0, gg = oracle.adjoint_step(G, st, lam1, g)
    lhs = (lam1 * jv).sum()
    rhs = (lam0 * v).sum() + (gg * dg).sum()
    assert lhs == pytest.approx(rhs, rel=1e-11)
    # the tangent of a ghost node of level t+1 is that of the node it copies
    # (its imposed velocity on the inlet disc has none)
    assert np.abs(jv[:, kinds == 2]).max() > 0
    # a ghost's sensitivity does not stay on it: lam0 at ghosts is what they
    # feed as emitters, and nodes that emit nothing have none
    assert np.abs(lam0[:, kinds == 2]).max() > 0


def test_adjoint_nodes_match_full_adjoint_with_ghost_layers(oracle):
    G = _small_jet(oracle)
    st = oracle.ghost_fill(G, W.random_state(G.shape, seed=35), 0)
    lam1 = np.random.default_rng(36).standard_normal(st.shape)
    lam0, dg = oracle.adjoint_step(G, st, lam1)
    idx = np.arange(0, G.n, 5)
    lam_s, dg_s = oracle.adjoint_nodes(G, st, lam1, idx)
    assert np.allclose(lam_s, lam0.reshape(10, -1)[:, idx], rtol=1e-13, atol=1e-14)
    assert np.allclose(dg_s, dg.reshape(3, -1)[:, idx], rtol=1e-13, atol=1e-14)


def test_rollout_gradient_with_ghost_layers_matches_central_differences(oracle):
    """FP64 central differences of the kinetic energy after 6 steps of the
    small jet (inlet disc with seeded noise, outflow ghosts), along random
    directions of g and of the interior initial velocity; the initial ghost
    layers are refilled from the interior on both sides."""
    G = _small_jet(oracle)
    kinds = oracle.node_kinds(G)
    steps = 6
    st0 = oracle.ghost_fill(G, W.random_state(G.shape, seed=37, u_amp=0.04, pi_amp=1e-3), 0)
    g = W.random_force(G.shape, seed=38, amp=1e-3)
    L, lam0, dgrad = oracle.rollout_grad(G, st0, steps, g)
    assert np.abs(lam0[:, kinds == 2]).max() == 0.0

    def loss(s, gf):
        return oracle.ke_seed(G, oracle.run(G, oracle.ghost_fill(G, s, 0), steps, gf))[0]

    assert L == pytest.approx(loss(st0, g), rel=1e-14)
    rng = np.random.default_rng(39)
    for _ in range(2):
        d = rng.standard_normal(g.shape)
        h = 1e-4 * np.abs(g).max()
        fd = (loss(st0, g + h * d) - loss(st0, g - h * d)) / (2 * h)
        assert (dgrad * d).sum() == pytest.approx(fd, rel=1e-6)
        du = np.zeros_like(st0)
        du[1:4][:, kinds == 0] = rng.standard_normal((3, int((kinds == 0).sum())))
        h = 1e-4 * np.abs(st0[1:4]).max()
        fd = (loss(st0 + h * du, g) - loss(st0 - h * du, g)) / (2 * h)
        assert (lam0 * du).sum() == pytest.approx(fd, rel=1e-6)
