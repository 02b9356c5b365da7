"""GPU parity of the forward update against the FP64 oracle (all through the
C ABI).  Tolerances: the parity bar is max relative error <= 1e-5 in
rho and u after 100 laminar steps (Taylor-Green 32^3); single steps from the
same binary32 state are held to a few binary32 ulps of the largest value
(normwise 2e-6 for u, 1e-7 absolute for rho - 1; Pi^neq is the difference
of sum f c c, rho u u and rho/3 delta, so its bar is 32 binary32 ulps of
the largest of max |u|^2, max |Pi| and max |rho - 1|, the scales of the
terms that cancel (Pi' = (S - J u' - D/3 delta)/216 in the kernels); after n steps
Pi^neq is held to n times that one-step bar, the rounding of every step
added up).  Full-size
workloads are checked at a seeded sample of nodes that the oracle updates
one by one from the GPU's own pre-step state, plus properties (conservation
in FP64 reductions) that hold at any size."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import abs_err, from_device_state, gpu_solver, oracle_grid, rel_err, to_device_state

pytestmark = pytest.mark.gpu

KERNELS = [0, 1, 2]  # tiled, direct, population layout
EPS32 = float(np.finfo(np.float32).eps)
EPS64 = float(np.finfo(np.float64).eps)


def pi_tol(want):
    # plus the oracle's own binary64 rounding of Pi^neq = sum f c c - rho u u
    # - rho/3 delta, a difference of terms of size 1/3 (64 eps64 ~ 1.4e-14)
    return 32 * EPS32 * max(float(np.abs(want[1:4]).max()) ** 2, float(np.abs(want[4:]).max()),
                            float(np.abs(want[0] - 1.0).max())) + 64 * EPS64


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2401_17074_amd  # noqa: F401  (fails loudly if the HIP library is missing)
    torch.cuda.set_device(0)


@pytest.mark.parametrize("order", [3, 2])
@pytest.mark.parametrize("kernel", KERNELS)
def test_taylor_green_100_steps(kernel, order):
    case = W.tgv_case()
    case.order = order
    st0 = W.to_fp32(W.tgv_state(case.nx, case.extra["u0"]))
    G = oracle_grid(case)
    want = oracle.run(G, st0, case.steps)
    s = gpu_solver(case, kernel=kernel)
    s.set_state(to_device_state(st0))
    s.step(case.steps)
    got = from_device_state(s.get_state())
    red, rc = s.reduce()
    s.close()
    e_u = rel_err(got[1:4], want[1:4])
    e_rho = rel_err(got[0], want[0])
    e_pi = abs_err(got[4:], want[4:])
    print("TGV kernel=%d order=%d rel err u %.3e rho %.3e; Pi abs err %.3e (rel %.3e)"
          % (kernel, order, e_u, e_rho, e_pi, rel_err(got[4:], want[4:])))
    assert e_u <= 1e-5 and e_rho <= 1e-5
    assert e_pi < case.steps * pi_tol(want)
    # decay of the Taylor-Green mode at nu = (tau - 1/2)/3
    mode = st0[1]
    amp = (got[1] * mode).sum() / (mode * mode).sum()
    amp_or = (want[1] * mode).sum() / (mode * mode).sum()
    assert amp == pytest.approx(amp_or, rel=1e-5)
    # FP64 reductions of the GPU state: mass and momentum conserved up to the
    # binary32 rounding of the stored u (one ulp of max |u| per node at most)
    r0, _ = oracle.reduce(G, st0)
    assert abs(red[0] - r0[0]) < 1e-9 * r0[0]
    assert np.abs(np.array(red[1:4]) - r0[1:4]).max() < case.nodes * EPS32 * np.abs(st0[1:4]).max()


CASES = [
    ("periodic", (0, 0, 0, 0, 0, 0)),
    ("walls_y", (0, 0, 1, 1, 0, 0)),
    ("walls_xz", (1, 1, 0, 0, 1, 1)),
    ("ghosts", (3, 3, 3, 3, 3, 3)),
]


@pytest.mark.parametrize("order", [3, 2])
@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("name,faces", CASES)
def test_random_state_ragged_grid(kernel, name, faces, order):
    """Odd sizes that span several tiles with ragged tails, random moments,
    per-node force field; 1 and then 6 more steps against the oracle, for the
    third-order update and the regularised second-order one."""
    case = W.Case(name, 71, 37, 23, 0.57, faces=faces, order=order)
    st0 = W.to_fp32(W.random_state(case.shape, seed=101))
    g = W.random_force(case.shape, seed=102, amp=1e-5).astype(np.float32).astype(np.float64)
    G = oracle_grid(case)
    st0 = oracle.ghost_fill(G, st0, 0)
    kinds = oracle.node_kinds(G)
    s = gpu_solver(case, kernel=kernel)
    s.set_force_field(g)
    s.set_state(to_device_state(st0))
    s.step(1)
    got1 = from_device_state(s.get_state())
    want1 = oracle.step(G, st0, g)
    fl = kinds == 0
    assert abs_err(got1[0], want1[0], fl) < 1e-7
    assert rel_err(got1[1:4], want1[1:4], fl) < 2e-6
    assert abs_err(got1[4:], want1[4:], fl) < pi_tol(want1[:, fl])
    # ghosts are refilled from the GPU's own level-1 interior values
    if (kinds == 2).any():
        want_g = oracle.ghost_fill(G, got1, 1)
        assert abs_err(got1, want_g, kinds == 2) < 1e-7
    s.step(6)
    got = from_device_state(s.get_state())
    s.close()
    want = oracle.run(G, st0, 7, g)
    assert rel_err(got[1:4], want[1:4], fl) < 1e-5
    assert abs_err(got[0], want[0], fl) < 1e-6


@pytest.mark.parametrize("kernel", KERNELS)
def test_small_jet_with_inlet_noise(kernel):
    case = W.jet_case(nx=48, ny=30, nz=26, D=8.0, steps=30)
    st0 = W.jet_state(case)
    G = oracle_grid(case)
    st0 = oracle.ghost_fill(G, st0, 0)
    kinds = oracle.node_kinds(G)
    s = gpu_solver(case, kernel=kernel)
    s.set_state(to_device_state(st0))
    got0 = from_device_state(s.get_state())
    # inlet ghosts at level 0 carry the imposed velocity and the seeded noise
    assert abs_err(got0[1:4], st0[1:4], kinds == 2) < 1e-8
    s.step(case.steps)
    got = from_device_state(s.get_state())
    s.close()
    want = oracle.run(G, st0, case.steps)
    assert rel_err(got[1:4], want[1:4]) < 1e-5
    assert abs_err(got[0], want[0]) < 1e-6
    assert abs_err(got[4:], want[4:]) < case.steps * pi_tol(want)


def _sampled_one_step(case, st_pre, got_post, nsamp, seed):
    G = oracle_grid(case)
    kinds = oracle.node_kinds(G)
    idx = W.sample_nodes(case, nsamp, seed, fluid_mask=(kinds == 0))
    want = oracle.update_nodes(G, st_pre, idx)
    got = got_post.reshape(10, -1)[:, idx]
    return got, want, G, kinds


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("dims", [(384, 192, 192), (512, 256, 256)])
def test_channel_full_size_sampled(kernel, dims):
    """The 384x192x192 channel and the 512x256x256 one that the benchmark
    times (walls at y = 0, ny - 1), in the launch configuration the benchmark
    uses: 20 steps, then one more step checked at 4000 sampled fluid nodes."""
    case = W.channel_case(nx=dims[0], ny=dims[1], nz=dims[2])
    st0 = W.to_fp32(W.channel_state(case))
    s = gpu_solver(case, kernel=kernel)
    s.set_state(to_device_state(st0))
    r0, _ = s.reduce()
    s.step(20)
    pre = from_device_state(s.get_state())
    s.step(1)
    post = from_device_state(s.get_state())
    r1, rc = s.reduce()
    s.close()
    got, want, G, kinds = _sampled_one_step(case, pre, post, 4000, 5)
    assert np.abs(got[0] - want[0]).max() < 1e-7
    assert np.abs(got[1:4] - want[1:4]).max() < 2e-6 * np.abs(want[1:4]).max()
    assert np.abs(got[4:] - want[4:]).max() < pi_tol(want)
    # mass with bounce-back walls is conserved; momentum gains sum rho g per step
    assert abs(r1[0] - r0[0]) < 1e-6 * r0[0]


def test_max_size_periodic_sampled():
    """The largest grid the 32-bit field offsets allow, 1024 x 1024 x 1023
    (just under 2^30 nodes, 86 GB of FP32 state), tiled kernel: one step
    from a seeded random state, checked at sampled nodes against the oracle
    run on each node's 3x3x3 neighbourhood (on a 3^3 periodic grid the
    centre node's update reads exactly those 27 nodes), plus FP64
    conservation of mass and momentum over the whole grid."""
    import torch
    case = W.Case("max_periodic", 1024, 1024, 1023, 0.6)
    nz, ny, nx = case.shape
    assert case.nodes < 2 ** 30
    st = W.random_state_device(case.shape, seed=2024)
    s = gpu_solver(case, kernel=0)
    s.set_state(st)
    idx = W.sample_nodes(case, 400, seed=9)
    x, y, z = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    d = np.arange(-1, 2)
    zz = (z[:, None, None, None] + d[None, :, None, None]) % nz
    yy = (y[:, None, None, None] + d[None, None, :, None]) % ny
    xx = (x[:, None, None, None] + d[None, None, None, :]) % nx
    nbr = torch.from_numpy(((zz * ny + yy) * nx + xx).reshape(-1)).cuda()
    pre = st.view(10, -1)[:, nbr].double().cpu().numpy().reshape(10, idx.size, 3, 3, 3)
    del st
    torch.cuda.empty_cache()
    r0, _ = s.reduce()
    s.step(1)
    r1, rc = s.reduce()
    post = s.get_state()
    got = post.view(10, -1)[:, torch.from_numpy(idx).cuda()].double().cpu().numpy()
    del post
    s.close()
    torch.cuda.empty_cache()
    got[0] += 1.0
    G3 = oracle_grid(W.Case("neighbourhood", 3, 3, 3, case.tau))
    want = np.empty_like(got)
    for k in range(idx.size):
        loc = pre[:, k].copy()
        loc[0] += 1.0
        want[:, k] = oracle.update_nodes(G3, loc, np.array([13]))[:, 0]
    assert rc == 0
    assert np.abs(got[0] - want[0]).max() < 1e-7
    assert np.abs(got[1:4] - want[1:4]).max() < 2e-6 * np.abs(want[1:4]).max()
    assert np.abs(got[4:] - want[4:]).max() < pi_tol(want)
    assert abs(r1[0] - r0[0]) < 1e-9 * r0[0]
    assert np.abs(np.asarray(r1[1:4]) - np.asarray(r0[1:4])).max() < 1e-9 * r0[0]


@pytest.mark.parametrize("kernel", KERNELS)
def test_jet_full_size_sampled(kernel):
    """512x256x256 jet (inlet disc, outflow ghosts elsewhere): 10 steps, then
    one step checked at sampled fluid nodes, and the ghost refill checked on
    every ghost node against the rule applied to the GPU's interior."""
    case = W.jet_case()
    s = gpu_solver(case, kernel=kernel)
    s.set_state(to_device_state(W.jet_state(case)))
    s.step(10)
    pre = from_device_state(s.get_state())
    s.step(1)
    post = from_device_state(s.get_state())
    s.close()
    got, want, G, kinds = _sampled_one_step(case, pre, post, 3000, 6)
    assert np.abs(got[0] - want[0]).max() < 1e-7
    assert np.abs(got[1:4] - want[1:4]).max() < 2e-6 * max(np.abs(want[1:4]).max(), 1e-3)
    assert np.abs(got[4:] - want[4:]).max() < pi_tol(want)
    t = 11
    regen = oracle.ghost_fill(G, post, t)
    gh = kinds == 2
    assert np.abs(regen[:, gh] - post[:, gh]).max() < 1e-8


@pytest.mark.parametrize("name,faces,field", [(n, f, False) for n, f in CASES[:2]] + [("periodic_field", CASES[0][1], True)])
def test_work_list_odd_segments(name, faces, field):
    """A grid whose work list hands blocks a column segment of an odd number
    of planes followed by another segment (256 x 60 x 457: 20 tile columns,
    27-plane tiles, the leftover tiles cut in 3; the CPU schedule test checks
    that such transitions occur): with FP32 storage the tiled update loads
    the stored fields two plane-steps ahead into two register sets used in
    turn, and such a segment ends on the other set; a force field is loaded
    one step ahead across the same transitions.  One step from a seeded
    random state, every fluid node against the oracle."""
    case = W.Case(name, 256, 60, 457, 0.57, faces=faces)
    st0 = W.to_fp32(W.random_state(case.shape, seed=457))
    g = W.random_force(case.shape, seed=458, amp=1e-5).astype(np.float32).astype(np.float64) if field else None
    G = oracle_grid(case)
    kinds = oracle.node_kinds(G)
    s = gpu_solver(case, kernel=0)
    if field:
        s.set_force_field(g)
    s.set_state(to_device_state(st0))
    s.step(1)
    got = from_device_state(s.get_state())
    s.close()
    want = oracle.step(G, st0, g)
    fl = kinds == 0
    assert abs_err(got[0], want[0], fl) < 1e-7
    assert rel_err(got[1:4], want[1:4], fl) < 2e-6
    assert abs_err(got[4:], want[4:], fl) < pi_tol(want[:, fl])


@pytest.mark.parametrize("kernel", KERNELS)
def test_determinism(kernel):
    case = W.Case("det", 64, 40, 33, 0.6, faces=(0, 0, 1, 1, 0, 0), force=(1e-6, 0, 0))
    st0 = W.to_fp32(W.random_state(case.shape, seed=103))
    outs = []
    for _ in range(2):
        s = gpu_solver(case, kernel=kernel)
        s.set_state(to_device_state(st0))
        s.step(5)
        outs.append(s.get_state().cpu().numpy())
        s.close()
    assert np.array_equal(outs[0], outs[1])


def test_second_order_update_has_no_adjoint():
    """The adjoint calls reject the regularised second-order update."""
    import torch
    from paper_2401_17074_amd import _binding as C
    case = W.Case("order2", 16, 12, 10, 0.6, order=2)
    s = gpu_solver(case)
    raw = s.save_raw()
    lam = torch.zeros((10,) + case.shape, dtype=torch.float32, device="cuda")
    with pytest.raises(RuntimeError, match="third-order"):
        s.adjoint_step(raw, raw, lam)
    s.close()


@pytest.mark.parametrize("what", ["fp16", "bf16", "d3q19", "d2q9", "alias"])
def test_adjoint_rejects_what_it_does_not_differentiate(what):
    """The adjoint step refuses 16-bit storage, the other lattices
    (TSLB_E_UNSUPPORTED) and an output aliasing its input (TSLB_E_INVALID),
    before touching any buffer."""
    import torch
    from paper_2401_17074_amd import _binding as C
    storage = {"fp16": C.TSLB_FP16, "bf16": C.TSLB_BF16}.get(what, C.TSLB_FP32)
    lattice = {"d3q19": 19, "d2q9": 9}.get(what, 27)
    case = W.Case("adj_" + what, 16, 12, 1 if lattice == 9 else 10, 0.6, lattice=lattice)
    s = gpu_solver(case, storage=storage)
    raw = s.save_raw()
    lam = torch.ones((10,) + case.shape, dtype=torch.float32, device="cuda")
    out = torch.full_like(lam, 7.0)
    with pytest.raises(C.TslbError) as err:
        C.tslb_adjoint_step(s.h, raw, raw, lam, lam if what == "alias" else out, None)
    s.close()
    assert err.value.code == (C.TSLB_E_INVALID if what == "alias" else C.TSLB_E_UNSUPPORTED)
    assert bool((out == 7.0).all()) and bool((lam == 1.0).all())


@pytest.mark.parametrize("kernel", KERNELS)
def test_timed_steps_match_plain_steps(kernel):
    """tslb_step_timed runs the same launches as tslb_step (bit-identical
    state) and reports positive kernel and auxiliary times."""
    case = W.channel_case(nx=40, ny=20, nz=18, re_tau=10)
    st0 = W.to_fp32(W.channel_state(case))
    out = []
    for timed in (False, True):
        s = gpu_solver(case, kernel=kernel)
        s.set_state(to_device_state(st0))
        if timed:
            ms_main, ms_aux = s.step_timed(5)
            assert ms_main > 0.0 and ms_aux >= 0.0
        else:
            s.step(5)
        assert s.t == 5
        out.append(s.get_state().cpu().numpy())
        s.close()
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("kernel", KERNELS)
def test_bound_state_buffers(kernel):
    """After tslb_bind_state the solver runs on caller-owned tensors: the
    bound buffer holds the current level (ghost layers included) and the
    steps that follow match a solver on the library's own buffers bit for
    bit.  Aliasing and misaligned buffers are rejected."""
    import torch
    from paper_2401_17074_amd import _binding as C
    case = W.jet_case(nx=40, ny=22, nz=20, D=6.0, steps=12)
    G = oracle_grid(case)
    st0 = W.to_fp32(oracle.ghost_fill(G, W.jet_state(case), 0))
    out = []
    for bind in (False, True):
        s = gpu_solver(case, kernel=kernel)
        s.set_state(to_device_state(st0))
        s.step(3)
        if bind:
            before = s.save_raw()
            s.bind_state_to_torch()
            assert torch.equal(s.state_buffers[0], before)
            nb = C.tslb_state_bytes(s.h)
            spare = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
            with pytest.raises(RuntimeError):
                C.tslb_bind_state(s.h, spare, spare)
            with pytest.raises(RuntimeError):
                C.tslb_bind_state(s.h, spare[4:], s.state_buffers[1])
        s.step(case.steps - 3)
        out.append(s.get_state().cpu().numpy())
        s.close()
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("name,faces", CASES[:3])
def test_relaxation_profile_ragged_grid(kernel, name, faces):
    """A relaxation time that changes from plane to plane (each population
    relaxes with the tau of its emitting node's plane): 1 and 6 more steps
    against the oracle."""
    case = W.Case(name, 67, 29, 23, 0.57, faces=faces)
    tau_z = [float(np.float32(v)) for v in np.random.default_rng(104).uniform(0.52, 1.6, case.nz)]
    st0 = W.to_fp32(W.random_state(case.shape, seed=105))
    g = W.random_force(case.shape, seed=106, amp=1e-5).astype(np.float32).astype(np.float64)
    G = oracle.make_grid(case.nx, case.ny, case.nz, float(np.float32(case.tau)), faces=faces, tau_z=tau_z)
    kinds = oracle.node_kinds(G)
    fl = kinds == 0
    s = gpu_solver(case, kernel=kernel)
    s.set_relaxation_profile(tau_z)
    s.set_force_field(g)
    s.set_state(to_device_state(st0))
    s.step(1)
    got1 = from_device_state(s.get_state())
    want1 = oracle.step(G, st0, g)
    assert abs_err(got1[0], want1[0], fl) < 1e-7
    assert rel_err(got1[1:4], want1[1:4], fl) < 2e-6
    assert abs_err(got1[4:], want1[4:], fl) < pi_tol(want1[:, fl])
    s.step(6)
    got = from_device_state(s.get_state())
    # back to the uniform tau: the next step matches the scalar-tau oracle
    s.set_relaxation_profile(None)
    s.step(1)
    got8 = from_device_state(s.get_state())
    s.close()
    want = oracle.run(G, st0, 7, g)
    assert rel_err(got[1:4], want[1:4], fl) < 1e-5
    assert abs_err(got[0], want[0], fl) < 1e-6
    G0 = oracle.make_grid(case.nx, case.ny, case.nz, float(np.float32(case.tau)), faces=faces)
    want8 = oracle.step(G0, got, g, t=7)
    assert rel_err(got8[1:4], want8[1:4], fl) < 2e-6


@pytest.mark.parametrize("kernel", KERNELS)
def test_small_paper_jet(kernel):
    """The jet as the paper sets it up, scaled down: inlet disc on z = 0 with
    time-varying Gaussian noise, periodic crossflow faces, outflow on top and
    an outlet sponge; 30 steps against the oracle."""
    case = W.paper_jet_case(nx=30, ny=28, nz=40, D=8.0, steps=30, sponge=(1000.0, 3.0, 10))
    st0 = W.jet_state(case)
    G = oracle_grid(case)
    st0 = oracle.ghost_fill(G, st0, 0)
    kinds = oracle.node_kinds(G)
    s = gpu_solver(case, kernel=kernel)
    s.set_state(to_device_state(st0))
    got0 = from_device_state(s.get_state())
    # inlet ghosts at level 0 carry the imposed velocity and the Gaussian noise
    assert abs_err(got0[1:4], st0[1:4], kinds == 2) < 1e-8
    s.step(case.steps)
    got = from_device_state(s.get_state())
    s.close()
    want = oracle.run(G, st0, case.steps)
    assert rel_err(got[1:4], want[1:4]) < 1e-5
    assert abs_err(got[0], want[0]) < 1e-6
    assert abs_err(got[4:], want[4:]) < case.steps * pi_tol(want)


def test_paper_jet_full_size_sampled():
    """440x440x600 jet of the paper's set-up in the benchmark launch (tiled
    kernel): 10 steps, then one step checked at sampled fluid nodes (several
    inside the sponge), and the Gaussian inlet refill on the whole inlet face."""
    case = W.paper_jet_case()
    s = gpu_solver(case)
    s.set_state(to_device_state(W.jet_state(case)))
    s.step(10)
    pre = from_device_state(s.get_state())
    s.step(1)
    post = from_device_state(s.get_state())
    s.close()
    G = oracle_grid(case)
    kinds = oracle.node_kinds(G)
    idx = W.sample_nodes(case, 3000, 7, fluid_mask=(kinds == 0))
    top = np.flatnonzero((kinds == 0).ravel()[-60 * case.nx * case.ny:]) + (case.nz - 60) * case.nx * case.ny
    idx = np.concatenate([idx, np.random.default_rng(8).choice(top, 500, replace=False)])
    want = oracle.update_nodes(G, pre, idx)
    got = post.reshape(10, -1)[:, idx]
    assert np.abs(got[0] - want[0]).max() < 1e-7
    assert np.abs(got[1:4] - want[1:4]).max() < 2e-6 * max(np.abs(want[1:4]).max(), 1e-3)
    assert np.abs(got[4:] - want[4:]).max() < pi_tol(want)
    inlet = post[:, 0]
    regen = oracle.ghost_fill(G, post, 11)[:, 0]
    assert np.abs(regen - inlet).max() < 1e-8


DEGENERATE = [
    ("one_node", (1, 1, 1), (0,) * 6),
    ("one_fluid_node", (3, 3, 3), (1,) * 6),
    ("thin_periodic", (2, 1, 5), (0,) * 6),
    ("one_tile_plus_one", (65, 3, 4), (0, 0, 1, 1, 0, 0)),
    ("single_column", (1, 64, 3), (0, 0, 1, 1, 0, 0)),
    ("long_thin_ghosts", (200, 3, 3), (3, 3, 1, 1, 0, 0)),
]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("name,dims,faces", DEGENERATE)
def test_degenerate_grids(kernel, name, dims, faces):
    """Axes of one node (every neighbour is the node itself), a single fluid
    node between six walls, one column past a tile, one-column grids, and
    zero steps; 1 and 4 steps against the oracle."""
    nx, ny, nz = dims
    case = W.Case(name, nx, ny, nz, 0.62, faces=faces, force=(2e-6, -1e-6, 0.0))
    st0 = W.to_fp32(W.random_state(case.shape, seed=106))
    G = oracle_grid(case)
    st0 = oracle.ghost_fill(G, st0, 0)
    kinds = oracle.node_kinds(G)
    fl = kinds == 0
    s = gpu_solver(case, kernel=kernel)
    s.set_state(to_device_state(st0))
    s.step(0)
    assert s.t == 0
    s.step(1)
    got1 = from_device_state(s.get_state())
    s.step(3)
    got4 = from_device_state(s.get_state())
    s.close()
    want1 = oracle.step(G, st0)
    want4 = oracle.run(G, st0, 4)
    assert abs_err(got1[0], want1[0], fl) < 1e-7
    assert rel_err(got1[1:4], want1[1:4], fl) < 2e-6
    assert abs_err(got1[4:], want1[4:], fl) < pi_tol(want1[:, fl])
    assert rel_err(got4[1:4], want4[1:4], fl) < 1e-5
