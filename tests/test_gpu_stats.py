"""On-device velocity statistics (Section 3.1 channel moments, Section 3.2
jet centreline and half-width) against the statistics oracle applied to the
GPU's own states, downloaded at every sample.  The GPU sums in FP64 in a
different order than numpy, so sums agree to ~1e-12 relative; derived
float32 outputs to a few float32 ulps."""
import numpy as np
import pytest

import workloads as W
from helpers import from_device_state, gpu_solver, oracle_grid, to_device_state
from oracle import stats as OS
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2401_17074_amd  # noqa: F401
    torch.cuda.set_device(0)


def _run_and_sample(s, nsamples, every):
    states = []
    for _ in range(nsamples):
        s.step(every)
        s.stats_sample()
        states.append(from_device_state(s.get_state()))
    return states


@pytest.mark.parametrize("storage", [0, 1])
@pytest.mark.parametrize("axis", [1, 0, 2])
def test_profile_sums_match_oracle(axis, storage):
    case = W.channel_case(nx=40, ny=22, nz=18, re_tau=10)
    st0 = W.to_fp32(W.channel_state(case))
    kinds = oracle.node_kinds(oracle_grid(case))
    s = gpu_solver(case, storage=storage)
    s.set_state(to_device_state(st0))
    s.stats_begin(profile_axis=axis)
    states = _run_and_sample(s, 4, 3)
    sums, ns = s.stats_profile()
    s.close()
    want = OS.profile_sums([st[1:4] for st in states], axis, kinds == 0)
    assert ns == 4
    got = sums.numpy()
    assert got.shape == want.shape
    assert np.array_equal(got[:, 0], want[:, 0])
    scale = np.abs(want).max(axis=0) + 1e-300
    assert np.all(np.abs(got - want) <= 1e-12 * scale)
    U, c2, c3 = OS.profile_moments(got[want[:, 0] > 0])
    if axis == 1:
        assert np.all(U[:, 0] > 0) and np.all(c2[:, 0] >= -1e-15)


def test_field_moments_match_oracle():
    import torch
    case = W.channel_case(nx=36, ny=20, nz=16, re_tau=10)
    st0 = W.to_fp32(W.channel_state(case))
    s = gpu_solver(case)
    s.set_state(to_device_state(st0))
    s.stats_begin(profile_axis=1, field=True)
    states = _run_and_sample(s, 5, 2)
    mean, cov = s.stats_field()
    torch.cuda.synchronize()
    s.close()
    s1, s2 = OS.field_sums([st[1:4] for st in states])
    m = s1 / 5
    c = np.stack([s2[k] / 5 - m[a] * m[b] for k, (a, b) in enumerate(OS.PAIRS)])
    assert np.abs(mean.double().cpu().numpy() - m).max() <= 2 * np.finfo(np.float32).eps * np.abs(m).max()
    umax2 = float((m ** 2).max())
    assert np.abs(cov.double().cpu().numpy() - c).max() <= 4 * np.finfo(np.float32).eps * max(umax2, 1e-30)


@pytest.mark.parametrize("center", [(30.0, 30.0), (29.5, 31.5)])
def test_jet_diagnostics_of_a_cone(center):
    """A state whose axial velocity is the cone U (1 - r / 2R): one sample,
    then U_c and r_1/2 of every cross-section against the oracle's binning
    (which is exact for a cone)."""
    import torch
    case = W.Case("cone", 61, 61, 7, 0.6, faces=(0, 0, 0, 0, 0, 0))
    ny, nx = 61, 61
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((xx - center[0]) ** 2 + (yy - center[1]) ** 2)
    st = W.rest_state(case.shape)
    st[3] = (0.05 * (1.0 - r / 34.0))[None]
    st = W.to_fp32(st)
    s = gpu_solver(case)
    s.set_state(to_device_state(st))
    s.stats_begin(field=True)
    s.stats_sample()
    uc, rh = s.stats_jet(2, center)
    torch.cuda.synchronize()
    uc, rh = uc.double().cpu().numpy(), rh.double().cpu().numpy()
    s.close()
    want_uc, want_rh = OS.jet_axis(st[3], center, axis=2)
    assert np.allclose(uc, want_uc, rtol=2e-7)
    assert np.allclose(rh, want_rh, rtol=2e-7)


def test_jet_diagnostics_of_a_running_jet():
    """The scaled-down paper jet: field statistics over 20 samples, then U_c
    and r_1/2 against the oracle's rule applied to the mean of the
    downloaded states."""
    import torch
    case = W.paper_jet_case(nx=40, ny=40, nz=48, D=12.0, steps=60, sponge=(1000.0, 3.0, 10))
    s = gpu_solver(case)
    s.set_state(to_device_state(W.jet_state(case)))
    s.step(40)
    s.stats_begin(profile_axis=2, field=True)
    states = _run_and_sample(s, 20, 1)
    uc, rh = s.stats_jet(2, case.inlet_center)
    torch.cuda.synchronize()
    uc, rh = uc.double().cpu().numpy(), rh.double().cpu().numpy()
    s.close()
    s1, _ = OS.field_sums([st[1:4] for st in states])
    want_uc, want_rh = OS.jet_axis(s1[2] / 20, case.inlet_center, axis=2)
    assert np.allclose(uc, want_uc, rtol=1e-6, atol=1e-9)
    ok = want_rh > 0
    assert ok[1:8].all()  # the jet has a half-width near the inlet
    assert np.array_equal(rh > 0, ok)
    assert np.allclose(rh[ok], want_rh[ok], rtol=1e-5)


def test_statistics_argument_errors():
    from paper_2401_17074_amd import TslbError
    case = W.Case("err", 16, 12, 10, 0.7)
    s = gpu_solver(case)
    with pytest.raises(TslbError):
        s.stats_sample()  # no begin
    s.stats_begin(profile_axis=2)
    with pytest.raises(TslbError):
        s.stats_field()  # field sums not enabled
    s.stats_begin(field=True)
    s.stats_sample()
    with pytest.raises(TslbError):
        s.stats_jet(2, (20.0, 3.0))  # centre outside the cross-section
    s.close()
