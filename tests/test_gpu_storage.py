"""FP16 / BF16 moment storage and FP64 reductions on the GPU.

Pinned: one step from a state that is exactly representable in the storage
format must match the oracle (FP64 step, then the same storage rounding,
emulated from the IEEE definition) to within one storage ulp plus the
binary32 error of the computed value, everywhere, and exactly on at least
99 % of the stored values.  The binary32 error is absolute, at the scale of
the terms that cancel: each new moment is formed from sums of 27 scaled
populations (rho - 1 = D/216, Pi' = (S - J u' - D/3)/216), so a near-zero
value carries the rounding error of the largest terms, which can exceed one
storage ulp of that small value.  The bar is 16 eps32 times the largest
magnitude of the field, for rho - 1 also of |u| (the size of the c.u terms
of the populations summed into D) and for Pi also of |u|^2.  Reported, not pinned: the error of multi-step FP16/BF16
runs against the pure FP64 oracle on the 64^3 channel subcase."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import from_device_state, gpu_solver, oracle_grid, to_device_state

pytestmark = pytest.mark.gpu

DEFAULT_SCALES = {1: (2.0 ** 12, 2.0 ** 12, 2.0 ** 16), 2: (1.0, 1.0, 1.0)}
FRAC_BITS = {1: 10, 2: 7}
EMIN = {1: -14, 2: -126}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2401_17074_amd  # noqa: F401
    torch.cuda.set_device(0)


def _ulp(x, kind):
    """Spacing of the storage format at |x| (x already scaled)."""
    ax = np.abs(x)
    e = np.floor(np.log2(np.where(ax > 0, ax, 1.0)))
    e = np.maximum(e, EMIN[kind])
    return 2.0 ** (e - FRAC_BITS[kind])


EPS32 = float(np.finfo(np.float32).eps)


def _bar(want_s, want, sc, kind):
    """Allowed |got - want| in scaled storage units: one storage ulp of the
    expected value plus the binary32 error of the field (see module doc)."""
    u2 = float((want[1:4] ** 2).sum(axis=0).max())
    fp32 = np.empty(10)
    # rho - 1 = D/216 sums 27 scaled populations whose sizes are set by c.u:
    # its binary32 error scales with the larger of |rho - 1| and |u|
    fp32[0] = 16 * EPS32 * max(np.abs(want[0] - 1.0).max(), np.abs(want[1:4]).max()) * sc[0]
    fp32[1:4] = 16 * EPS32 * np.abs(want[1:4]).max() * sc[1]
    fp32[4:] = 16 * EPS32 * max(np.abs(want[4:]).max(), u2) * sc[2]
    shape = (10,) + (1,) * (want_s.ndim - 1)
    return _ulp(want_s, kind) * 1.0000001 + fp32.reshape(shape)


def _worst(diff, bar, want_s, got_s, extra=None, nodes=None):
    """Field, node, expected and obtained scaled values of the largest
    violation of the bar (for the failure message)."""
    over = diff - bar
    q, k = np.unravel_index(np.argmax(over), over.shape)
    msg = "field %d node %d: want %r got %r diff %r bar %r" % (q, k, want_s[q, k], got_s[q, k], diff[q, k], bar[q, k])
    if extra is not None:
        msg += " exact %r" % (extra[q, k],)
    if nodes is not None:
        idx, nx, ny = nodes
        n = int(idx[k])
        msg += " at (x, y, z) = (%d, %d, %d)" % (n % nx, (n // nx) % ny, n // (nx * ny))
    return msg


def _scaled(st, sc):
    out = np.empty_like(st)
    out[0] = (st[0] - 1.0) * sc[0]
    out[1:4] = st[1:4] * sc[1]
    out[4:] = st[4:] * sc[2]
    return out


def _one_step_ulp(kind, kernel, faces, field, lattice=27, order=3):
    nz = 1 if lattice == 9 else 21
    case = W.Case("store", 67, 29, nz, 0.61, faces=faces, force=(2e-6, 0.0, 0.0), lattice=lattice, order=order)
    sc = DEFAULT_SCALES[kind]
    G = oracle_grid(case)
    st = W.random_state(case.shape, seed=301, u_amp=0.05, pi_amp=2e-3)
    if lattice == 9:
        st[[3, 6, 8, 9]] = 0.0  # no z components in two dimensions
    st0 = oracle.round_storage(G, st, kind, sc)
    kinds = oracle.node_kinds(G)
    st0[:, kinds == 1] = W.rest_state((1,))[:, 0:1]  # wall nodes hold the rest state
    g = W.random_force(case.shape, seed=302, amp=2e-6).astype(np.float32).astype(np.float64) if field else None
    if g is not None and lattice == 9:
        g[2] = 0.0
    s = gpu_solver(case, storage=kind, kernel=kernel)
    if field:
        s.set_force_field(g)
    s.set_state(to_device_state(st0))
    back = from_device_state(s.get_state())
    fl = kinds == 0
    assert np.array_equal(back[:, fl], st0[:, fl])  # representable input is stored exactly
    s.step(1)
    got = from_device_state(s.get_state())
    s.close()
    exact = oracle.step(G, st0, g)
    want = oracle.round_storage(G, exact, kind, sc)
    g_s, w_s = _scaled(got, sc)[:, fl], _scaled(want, sc)[:, fl]
    diff = np.abs(g_s - w_s)
    bar = _bar(w_s, exact[:, fl], sc, kind)
    assert np.all(diff <= bar), _worst(diff, bar, w_s, g_s, _scaled(exact, sc)[:, fl])
    assert (diff == 0).mean() >= 0.99


@pytest.mark.parametrize("field", [False, True])
@pytest.mark.parametrize("kind", [1, 2])
@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("faces", [(0,) * 6, (0, 0, 1, 1, 0, 0), (1, 1, 0, 0, 1, 1)])
def test_one_step_within_one_storage_ulp(kind, kernel, faces, field):
    """One step from a state representable in the 16-bit storage, against
    the oracle's exact step rounded the same way: periodic, walls on y, walls
    on x and z, with a uniform force or a per-node force field."""
    _one_step_ulp(kind, kernel, faces, field)


@pytest.mark.parametrize("field", [False, True])
@pytest.mark.parametrize("kind", [1, 2])
@pytest.mark.parametrize("faces", [(0,) * 6, (0, 0, 1, 1, 0, 0)])
def test_d3q19_one_step_within_one_storage_ulp(kind, faces, field):
    """The same for the D3Q19 update (tiled kernel)."""
    _one_step_ulp(kind, 0, faces, field, lattice=19)


def test_fp64_reductions_match_oracle_sums():
    case = W.Case("red", 50, 31, 17, 0.7, faces=(0, 0, 1, 1, 0, 0))
    st0 = W.to_fp32(W.random_state(case.shape, seed=302))
    G = oracle_grid(case)
    s = gpu_solver(case)
    s.set_state(to_device_state(st0))
    got = from_device_state(s.get_state())
    red, rc = s.reduce()
    s.close()
    want, bad = oracle.reduce(G, got)
    assert rc == 0 and bad == 0
    assert np.allclose(red, want, rtol=1e-12, atol=1e-15)


def test_reduce_flags_non_finite_state():
    from paper_2401_17074_amd import capi
    case = W.Case("nan", 16, 12, 10, 0.7)
    st0 = W.to_fp32(W.random_state(case.shape, seed=303))
    st0[2, 5, 6, 7] = np.nan
    s = gpu_solver(case)
    s.set_state(to_device_state(st0))
    _, rc = s.reduce(check=False)
    s.close()
    assert rc == capi.TSLB_E_UNSTABLE


def test_precision_error_report_channel_64():
    """64^3 channel subcase of the precision workload (h = 31, tau = 0.5045,
    laminar centreline 0.05): FP32 / FP16 / BF16 storage after 10 and 40
    steps against the pure FP64 oracle.  Printed for the record; the bounds
    are loose sanity checks, not parity claims."""
    case = W.channel_case(nx=64, ny=64, nz=64, tau=0.5045)
    nu = (case.tau - 0.5) / 3
    h = case.extra["h"]
    case.force = (0.05 * 2 * nu / h ** 2, 0.0, 0.0)
    case.extra["uc"] = 0.05
    st0 = W.to_fp32(W.channel_state(case))
    G = oracle_grid(case)
    kinds = oracle.node_kinds(G)
    fl = kinds == 0
    ref = {0: st0}
    cur = st0
    for t0, t1 in ((0, 10), (10, 40)):
        cur = oracle.run(G, cur, t1 - t0, t0=t0)
        ref[t1] = cur
    report = {}
    for kind, name in ((0, "fp32"), (1, "fp16"), (2, "bf16")):
        s = gpu_solver(case, storage=kind)
        s.set_state(to_device_state(st0))
        done = 0
        for t in (10, 40):
            s.step(t - done)
            done = t
            got = from_device_state(s.get_state())
            want = ref[t]
            du = (got[1:4] - want[1:4])[:, fl]
            dp = (got[4:] - want[4:])[:, fl]
            report[(name, t)] = (float(np.abs(du).max() / np.abs(want[1:4][:, fl]).max()),
                                 float(np.sqrt((du ** 2).mean() / (want[1:4][:, fl] ** 2).mean())),
                                 float(np.abs(dp).max() / np.abs(want[4:][:, fl]).max()),
                                 float(np.sqrt((dp ** 2).mean() / (want[4:][:, fl] ** 2).mean())))
        s.close()
    for k, v in sorted(report.items()):
        print("precision %s step %3d: u max %.3e rms %.3e | Pi max %.3e rms %.3e" % (k + v))
    assert report[("fp32", 40)][0] < 1e-5
    assert report[("fp16", 40)][0] < 1e-2
    assert report[("bf16", 40)][0] < 5e-2


@pytest.mark.parametrize("kind", [1, 2])
def test_precision_workload_full_size_sampled(kind):
    """512x256x256 channel with FP16 / BF16 moments (the launch the benchmark
    times): 5 steps, then one step checked at sampled fluid nodes against the
    oracle's FP64 update of the GPU's own stored state, rounded to storage."""
    case = W.channel_case(nx=512, ny=256, nz=256)
    sc = DEFAULT_SCALES[kind]
    s = gpu_solver(case, storage=kind)
    s.set_state(to_device_state(W.to_fp32(W.channel_state(case))))
    s.step(5)
    pre = from_device_state(s.get_state())
    s.step(1)
    post = from_device_state(s.get_state())
    s.close()
    G = oracle_grid(case)
    kinds = oracle.node_kinds(G)
    idx = W.sample_nodes(case, 2000, 305, fluid_mask=(kinds == 0))
    want = oracle.update_nodes(G, pre, idx)
    rnd = oracle.round_fp16 if kind == 1 else oracle.round_bf16
    want_s = np.empty_like(want)
    want_s[0] = [rnd((v - 1.0) * sc[0]) for v in want[0]]
    for q in range(1, 10):
        k = 1 if q < 4 else 2
        want_s[q] = [rnd(v * sc[k]) for v in want[q]]
    got_s = _scaled(post.reshape(10, -1)[:, idx], sc)
    diff = np.abs(got_s - want_s)
    bar = _bar(want_s, want, sc, kind)
    assert np.all(diff <= bar), _worst(diff, bar, want_s, got_s, _scaled(want, sc), (idx, case.nx, case.ny))
    assert (diff == 0).mean() >= 0.99


def test_precision_error_report_horizons():
    """The precision workload's 64^3 laminar channel subcase at the horizons
    it names (10, 100 and 2000 steps): FP32, FP16 and BF16 storage against
    the pure FP64 oracle at 2048 seeded fluid nodes, whose oracle values
    tests/golden/make_precision_ref.py wrote (the oracle alone needs minutes
    for 2000 steps).  Max (normwise) and RMS relative errors of u and Pi are
    printed for the record.  Bars: FP32 storage holds the 1e-5 parity bar in
    u up to 100 steps; everything stays finite and within loose sanity
    bounds (the 16-bit errors are reported, not pinned)."""
    import os
    ref = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                               "precision_ref_channel_64.npz"), allow_pickle=False)
    idx = ref["idx"]
    case = W.precision_subcase()
    st0 = W.to_fp32(W.channel_state(case))
    report = {}
    for kind, name in ((0, "fp32"), (1, "fp16"), (2, "bf16")):
        s = gpu_solver(case, storage=kind)
        s.set_state(to_device_state(st0))
        done = 0
        for t in ref["horizons"]:
            s.step(int(t) - done)
            done = int(t)
            got = from_device_state(s.get_state()).reshape(10, -1)[:, idx]
            want = ref["moments_%d" % t]
            du, dp = got[1:4] - want[1:4], got[4:] - want[4:]
            report[(name, done)] = (float(np.abs(du).max() / np.abs(want[1:4]).max()),
                                    float(np.sqrt((du ** 2).mean() / (want[1:4] ** 2).mean())),
                                    float(np.abs(dp).max() / np.abs(want[4:]).max()),
                                    float(np.sqrt((dp ** 2).mean() / (want[4:] ** 2).mean())))
            assert np.all(np.isfinite(got))
        s.close()
    for k, v in sorted(report.items(), key=lambda kv: (kv[0][0], kv[0][1])):
        print("precision %s step %4d: u max %.3e rms %.3e | Pi max %.3e rms %.3e" % (k + v))
    assert report[("fp32", 10)][0] < 1e-5 and report[("fp32", 100)][0] < 1e-5
    for t in (10, 100, 2000):
        assert report[("fp32", t)][0] < 1e-3
        assert report[("fp16", t)][0] < 5e-2
        assert report[("bf16", t)][0] < 2e-1


@pytest.mark.parametrize("field", [False, True])
@pytest.mark.parametrize("kind", [1, 2])
@pytest.mark.parametrize("faces", [(0,) * 6, (0, 0, 1, 1, 0, 0), (1, 1, 1, 1, 0, 0)])
def test_d2q9_one_step_within_one_storage_ulp(kind, faces, field):
    """The same for the D2Q9 update."""
    _one_step_ulp(kind, 0, faces, field, lattice=9)


@pytest.mark.parametrize("kind", [1, 2])
@pytest.mark.parametrize("faces", [(0,) * 6, (0, 0, 1, 1, 0, 0)])
def test_second_order_one_step_within_one_storage_ulp(kind, faces):
    """The same for the regularised second-order update (tiled kernel)."""
    _one_step_ulp(kind, 0, faces, True, order=2)
