"""GPU discrete adjoint against the FP64 oracle adjoint (which is itself
pinned by the dot-product identity and by FP64 central differences in the
CPU suite).  All calls go through the C ABI."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import gpu_solver, oracle_grid, to_device_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2401_17074_amd  # noqa: F401
    torch.cuda.set_device(0)


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("faces", [(0,) * 6, (0, 0, 1, 1, 0, 0), (1, 1, 0, 0, 1, 1)])
def test_one_adjoint_step_matches_oracle(faces, kernel):
    import torch
    case = W.Case("adj1", 71, 26, 19, 0.62, faces=faces)
    st0 = W.to_fp32(W.random_state(case.shape, seed=201, u_amp=0.05, pi_amp=2e-3))
    g = W.random_force(case.shape, seed=202, amp=1e-4).astype(np.float32).astype(np.float64)
    lam1 = np.random.default_rng(203).standard_normal(st0.shape).astype(np.float32).astype(np.float64)
    G = oracle_grid(case)
    kinds = oracle.node_kinds(G)
    lam1[:, kinds != 0] = 0.0
    s = gpu_solver(case, kernel=kernel)
    s.set_force_field(g)
    s.set_state(to_device_state(st0))
    raw0 = s.save_raw()
    s.step(1)
    raw1 = s.save_raw()
    lam1_t = torch.tensor(lam1, dtype=torch.float32, device="cuda")
    dg = torch.zeros((3,) + case.shape, dtype=torch.float32, device="cuda")
    lam0 = s.adjoint_step(raw0, raw1, lam1_t, dg).double().cpu().numpy()
    dg = dg.double().cpu().numpy()
    s.close()
    want_lam, want_dg = oracle.adjoint_step(G, st0, lam1, g)
    assert _rel(lam0, want_lam) < 1e-5
    assert _rel(dg, want_dg) < 1e-5


@pytest.mark.parametrize("kernel", [0, 1])
def test_checkpointed_rollout_gradient_matches_oracle(kernel):
    """TslbRollout (checkpoint every 7 of 30 steps) on a 16^3 forced periodic
    box: dL/dg and dL/du0 against the oracle's stored-trajectory adjoint."""
    import torch
    from paper_2401_17074_amd import TslbRollout
    case = W.adjoint_case(n=16, steps=30, ckpt=7)
    st0, g = W.adjoint_inputs(case)
    st0 = W.to_fp32(st0)
    g = g.astype(np.float32).astype(np.float64)
    G = oracle_grid(case)
    L_or, lam0_or, dg_or = oracle.rollout_grad(G, st0, case.steps, g)
    s = gpu_solver(case, kernel=kernel)
    gt = torch.tensor(g, dtype=torch.float32, device="cuda", requires_grad=True)
    ut = torch.tensor(st0[1:4], dtype=torch.float32, device="cuda", requires_grad=True)
    L = TslbRollout.apply(gt, ut, s, case.steps, case.extra["ckpt"])
    L.backward()
    s.close()
    assert float(L.detach()) == pytest.approx(L_or, rel=1e-5)
    assert _rel(gt.grad.double().cpu().numpy(), dg_or) < 1e-4
    assert _rel(ut.grad.double().cpu().numpy(), lam0_or[1:4]) < 1e-4


@pytest.mark.parametrize("kernel", [0, 1])
def test_full_size_adjoint_step_sampled(kernel):
    """64^3 forced periodic box of the differentiable workload: one adjoint
    step at the step the rollout uses, checked at sampled nodes."""
    import torch
    case = W.adjoint_case()
    st0, g = W.adjoint_inputs(case)
    st0 = W.to_fp32(st0)
    g = g.astype(np.float32).astype(np.float64)
    G = oracle_grid(case)
    s = gpu_solver(case, kernel=kernel)
    s.set_force_field(g)
    s.set_state(to_device_state(st0))
    s.step(3)
    raw0 = s.save_raw()
    pre = s.get_state().double().cpu().numpy()
    pre[0] += 1.0
    s.step(1)
    raw1 = s.save_raw()
    lam1 = s.adjoint_seed(raw1)
    lam0 = s.adjoint_step(raw0, raw1, lam1).double().cpu().numpy()
    lam1 = lam1.double().cpu().numpy()
    s.close()
    idx = W.sample_nodes(case, 600, 204)
    want, _ = oracle.adjoint_nodes(G, pre, lam1, idx, g)
    got = lam0.reshape(10, -1)[:, idx]
    assert _rel(got, want) < 1e-5


@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("faces", [(0,) * 6, (0, 0, 1, 1, 0, 0)])
def test_adjoint_step_with_relaxation_profile(faces, kernel):
    """One adjoint step when tau changes from plane to plane: each emitted
    population is differentiated with the tau of its emitter's plane."""
    import torch
    case = W.Case("adj_sponge", 69, 21, 17, 0.62, faces=faces)
    tau_z = [float(np.float32(v)) for v in np.random.default_rng(210).uniform(0.55, 1.5, case.nz)]
    st0 = W.to_fp32(W.random_state(case.shape, seed=211, u_amp=0.05, pi_amp=2e-3))
    g = W.random_force(case.shape, seed=212, amp=1e-4).astype(np.float32).astype(np.float64)
    lam1 = np.random.default_rng(213).standard_normal(st0.shape).astype(np.float32).astype(np.float64)
    G = oracle.make_grid(case.nx, case.ny, case.nz, float(np.float32(case.tau)), faces=faces, tau_z=tau_z)
    lam1[:, oracle.node_kinds(G) != 0] = 0.0
    s = gpu_solver(case, kernel=kernel)
    s.set_relaxation_profile(tau_z)
    s.set_force_field(g)
    s.set_state(to_device_state(st0))
    raw0 = s.save_raw()
    s.step(1)
    raw1 = s.save_raw()
    lam1_t = torch.tensor(lam1, dtype=torch.float32, device="cuda")
    dg = torch.zeros((3,) + case.shape, dtype=torch.float32, device="cuda")
    lam0 = s.adjoint_step(raw0, raw1, lam1_t, dg).double().cpu().numpy()
    dg = dg.double().cpu().numpy()
    s.close()
    want_lam, want_dg = oracle.adjoint_step(G, st0, lam1, g)
    assert _rel(lam0, want_lam) < 1e-5
    assert _rel(dg, want_dg) < 1e-5


@pytest.mark.parametrize("kernel", [0, 1])
def test_wall_shear_objective_rollout_matches_oracle(kernel):
    """The wall shear force on the y and z walls of a small forced channel:
    its value, its seed, and TslbRollout's gradients (20 steps, checkpoint
    every 6) against the oracle's stored-trajectory adjoint."""
    import torch
    from paper_2401_17074_amd import TslbRollout
    from paper_2401_17074_amd import capi as C
    case = W.Case("ws", 24, 18, 14, 0.7, faces=(0, 0, 1, 1, 1, 1))
    g = W.random_force(case.shape, seed=221, amp=1e-4).astype(np.float32).astype(np.float64)
    u0 = W.random_state(case.shape, seed=222, u_amp=0.02, pi_amp=0.0)[1:4].astype(np.float32).astype(np.float64)
    G = oracle_grid(case)
    kinds = oracle.node_kinds(G)
    u0[:, kinds != 0] = 0.0
    st0 = W.rest_state(case.shape)
    st0[1:4] = u0
    L_or, lam0_or, dg_or = oracle.rollout_grad(G, st0, 20, g, objective=oracle.OBJ_WALL_SHEAR)
    s = gpu_solver(case, kernel=kernel)
    # value and seed of the objective at the initial state
    s.set_state(to_device_state(st0))
    assert s.objective(C.TSLB_OBJ_WALL_SHEAR) == pytest.approx(oracle.wall_shear_seed(G, st0)[0], abs=1e-12)
    lam = s.adjoint_seed(s.save_raw(), C.TSLB_OBJ_WALL_SHEAR).double().cpu().numpy()
    assert np.abs(lam - oracle.wall_shear_seed(G, st0)[1]).max() < 1e-7
    gt = torch.tensor(g, dtype=torch.float32, device="cuda", requires_grad=True)
    ut = torch.tensor(u0, dtype=torch.float32, device="cuda", requires_grad=True)
    L = TslbRollout.apply(gt, ut, s, 20, 6, C.TSLB_OBJ_WALL_SHEAR)
    L.backward()
    s.close()
    assert float(L.detach()) == pytest.approx(L_or, rel=1e-4)
    assert _rel(gt.grad.double().cpu().numpy(), dg_or) < 1e-4
    fl = kinds == 0
    assert _rel(ut.grad.double().cpu().numpy()[:, fl], lam0_or[1:4][:, fl]) < 1e-4


def test_differentiable_workload_full_size_vs_central_differences():
    """The differentiable workload at its own size: 64^3 forced periodic box,
    400 steps, checkpoint every 20 steps, through TslbRollout.  Directional
    derivatives of the kinetic energy along two seeded directions of the
    force field and two of the initial velocity against the oracle's FP64
    central differences at a relative step of 1e-4
    (tests/golden/rollout_fd_forced_periodic_64.json, written by
    tests/golden/make_rollout_fd.py from the oracle alone): within 1e-3
    relative.  The loss itself, after 400 binary32 steps, within 1e-4: four
    times the 1e-5 bar on u after 100 laminar steps, doubled for the
    quadratic objective."""
    import json
    import os
    import torch
    from paper_2401_17074_amd import TslbRollout
    rec = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                      "rollout_fd_forced_periodic_64.json")))
    case = W.adjoint_case()
    assert rec["workload"] == case.name and rec["steps"] == case.steps
    st0, g = W.adjoint_inputs(case)
    st0 = W.to_fp32(st0)
    g = g.astype(np.float32).astype(np.float64)
    s = gpu_solver(case)
    gt = torch.tensor(g, dtype=torch.float32, device="cuda", requires_grad=True)
    ut = torch.tensor(st0[1:4], dtype=torch.float32, device="cuda", requires_grad=True)
    L = TslbRollout.apply(gt, ut, s, case.steps, case.extra["ckpt"])
    L.backward()
    s.close()
    grad_g = gt.grad.double().cpu().numpy()
    grad_u = ut.grad.double().cpu().numpy()
    dgs, dus = W.gradient_directions(case, rec["direction_seed"])
    print("loss GPU %.10g oracle %.10g" % (float(L.detach()), rec["loss"]))
    assert float(L.detach()) == pytest.approx(rec["loss"], rel=1e-4)
    for name, grad, dirs, fds in (("g", grad_g, dgs, rec["fd_g"]), ("u0", grad_u, dus, rec["fd_u0"])):
        for k, (d, fd) in enumerate(zip(dirs, fds)):
            got = float((grad * d).sum())
            print("d/d%s along direction %d: adjoint %.10g central differences %.10g (rel %.2e)"
                  % (name, k, got, fd, abs(got - fd) / abs(fd)))
            assert abs(got - fd) <= 1e-3 * abs(fd)


@pytest.mark.parametrize("kernel", [0, 1])
def test_adjoint_step_through_ghost_layers(kernel):
    """One adjoint step on a small jet (inlet disc with seeded noise, outflow
    ghosts on the other faces) against the oracle's: the ghost refill of the
    new level transposed first (in place on lam_t1), then the update with
    ghost nodes as ordinary emitters (Section 2.3)."""
    import torch
    case = W.jet_case(nx=30, ny=17, nz=14, D=6.0, steps=1)
    G = oracle_grid(case)
    kinds = oracle.node_kinds(G)
    st0 = W.to_fp32(oracle.ghost_fill(G, W.random_state(case.shape, seed=401, u_amp=0.04, pi_amp=1e-3), 0))
    g = W.random_force(case.shape, seed=402, amp=1e-4).astype(np.float32).astype(np.float64)
    lam1 = np.random.default_rng(403).standard_normal(st0.shape).astype(np.float32).astype(np.float64)
    s = gpu_solver(case, kernel=kernel)
    s.set_force_field(g)
    s.set_state(to_device_state(st0))
    raw0 = s.save_raw()
    s.step(1)
    raw1 = s.save_raw()
    lam1_t = torch.tensor(lam1, dtype=torch.float32, device="cuda")
    dg = torch.zeros((3,) + case.shape, dtype=torch.float32, device="cuda")
    lam0 = s.adjoint_step(raw0, raw1, lam1_t, dg).double().cpu().numpy()
    folded = lam1_t.double().cpu().numpy()
    dg = dg.double().cpu().numpy()
    s.close()
    want_lam, want_dg = oracle.adjoint_step(G, st0, lam1, g)
    assert np.abs(lam0[:, kinds == 2]).max() > 0  # ghost nodes emit
    assert np.abs(folded[:, kinds == 2]).max() == 0.0  # cleared by the fold
    assert _rel(lam0, want_lam) < 1e-5
    assert _rel(dg, want_dg) < 1e-5


def test_rollout_gradient_through_ghost_layers():
    """TslbRollout on a small jet (12 steps, checkpoint every 5) against the
    oracle's FP64 stored-trajectory gradient, both with the initial ghosts
    refilled from the interior: dL/dg and dL/du0 (zero on ghost nodes)."""
    import torch
    from paper_2401_17074_amd import TslbRollout
    case = W.jet_case(nx=30, ny=17, nz=14, D=6.0, steps=12)
    G = oracle_grid(case)
    kinds = oracle.node_kinds(G)
    st0 = W.to_fp32(W.random_state(case.shape, seed=404, u_amp=0.04, pi_amp=0.0, rho_amp=0.0))
    g = W.random_force(case.shape, seed=405, amp=1e-4).astype(np.float32).astype(np.float64)
    L_or, lam0_or, dg_or = oracle.rollout_grad(G, st0, case.steps, g)
    s = gpu_solver(case)
    gt = torch.tensor(g, dtype=torch.float32, device="cuda", requires_grad=True)
    ut = torch.tensor(st0[1:4], dtype=torch.float32, device="cuda", requires_grad=True)
    L = TslbRollout.apply(gt, ut, s, case.steps, 5)
    L.backward()
    s.close()
    du = ut.grad.double().cpu().numpy()
    assert float(L.detach()) == pytest.approx(L_or, rel=1e-5)
    assert np.abs(du[:, kinds == 2]).max() == 0.0
    assert _rel(gt.grad.double().cpu().numpy(), dg_or) < 1e-4
    assert _rel(du, lam0_or[1:4]) < 1e-4
