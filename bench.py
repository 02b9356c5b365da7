"""Benchmark of the moment-only high-order TSLB update on one MI355X.

Workload (the timed `value`): the precision workload's channel, D3Q27,
512 x 256 x 256 nodes (x, z periodic; bounce-back walls at y = 0 and
y = ny - 1), friction Reynolds number 180 forcing, tau = 0.5045, FP32
moments, seeded synthetic initial state (parabolic profile + 5 % uniform
perturbations).  One step is one full update of every node (the paper's
lattice-update count, Section 4).

Printed: ONE JSON line with MLUPS, the HBM roofline of the update kernel
(algorithmic bytes per launch / measured average launch time, against the
8 TB/s peak and against the library's streaming copy measured in the same
run), the FP64 CPU oracle timed on the host cores on bounded samples, and
the side measurements the metric names: FP16/BF16-moment storage on the same
channel (each with its own kernel roofline), and the adjoint-to-forward time
ratio with checkpoints every 20 steps, on the 64^3 differentiable box and on
a 256^3 box where bytes rather than launches dominate.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# VALU issue ceiling for FP32 arithmetic that is not packed: 256 CUs x 4 SIMDs
# x 16 lanes x 2.4 GHz, one lane operation per lane and clock (a wave64
# instruction takes four clocks); the published 157.3 TFLOP/s counts packed
# FP32 fused multiply-adds, four FLOP per lane and clock
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
BYTES_PER_FIELD = {0: 4, 1: 2, 2: 2}


# the sources the tiled update kernel is compiled from: HBM counters taken
# with other sources are not reported as this kernel's traffic
KERNEL_SOURCES = ("update_tiled.hip", "tslb_tiles.h", "tslb_device.h", "tslb_params.h")


def _source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2401_17074_amd", "csrc")
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(d, name), "rb").read())
    return h.hexdigest()[:16]


def _fluid_nodes(case):
    n = [case.nx, case.ny, case.nz]
    for d in range(3):
        lo, hi = case.faces[2 * d], case.faces[2 * d + 1]
        n[d] -= (lo != 0) + (hi != 0)
    return n[0] * n[1] * n[2]


def algorithmic_bytes(case, storage):
    """Bytes one update launch must move: read the stored fields of every
    node once, write those of every fluid node once (ten fields for D3Q27,
    six for D2Q9)."""
    b = BYTES_PER_FIELD[storage]
    nf = 6 if case.lattice == 9 else 10
    return nf * b * case.nodes + nf * b * _fluid_nodes(case)


def time_steps(solver, steps, warmup):
    import torch
    solver.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    solver.step(steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1), wall


def _solver(case, storage=0, kernel=0, order=3):
    import numpy as np
    import workloads as W
    from paper_2401_17074_amd import Solver
    f32 = lambda v: float(np.float32(v))  # noqa: E731
    s = Solver(case.nx, case.ny, case.nz, f32(case.tau), force=[f32(v) for v in case.force], faces=case.faces,
               storage=storage, inlet_u=case.inlet_u, inlet_center=case.inlet_center,
               inlet_radius=case.inlet_radius, inlet_noise=case.inlet_noise, seed=case.seed, kernel=kernel,
               order=order, inlet_noise_kind=case.noise_kind, lattice=case.lattice)
    prof = W.tau_profile(case)
    if prof is not None:
        s.set_relaxation_profile([f32(v) for v in prof])
    return s


def _device_state(st64):
    import numpy as np
    dev = st64.astype(np.float32)
    dev[0] = (st64[0] - 1.0).astype(np.float32)
    return dev


def kernel_roofline(case, storage, kms_per_launch, kname, copy_gbs):
    """Roofline figures of one update launch: algorithmic bytes / launch time
    against the 8 TB/s peak and the same-run streaming copy, and the counted
    HBM bytes per launch when a counter summary of these sources exists."""
    algo = algorithmic_bytes(case, storage)
    achieved = algo / (kms_per_launch * 1e-3) / 1e9
    rec = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": load_traffic(kname, case.name, storage),
           "algorithmic_bytes_per_launch": algo, "avg_launch_ms": round(kms_per_launch, 5), "kernel": kname}
    if copy_gbs:
        rec["copy_gbs"] = round(copy_gbs, 1)
        rec["frac_of_copy"] = round(achieved / copy_gbs, 4)
    if rec["traffic"]:
        rec["traffic_over_algorithmic"] = round(rec["traffic"] / algo, 4)
    insts = load_valu(kname, case.name, storage)
    if insts:
        # the same launch against the VALU issue ceiling: thread-level VALU
        # instructions (wave instructions x 64 lanes) per second
        lane_ops = insts * 64 / (kms_per_launch * 1e-3)
        rec["valu"] = {"bound": "alu", "achieved": round(lane_ops / 1e12, 2), "peak": round(VALU_PEAK_LANE_OPS / 1e12, 2),
                       "unit": "T VALU lane-instructions/s", "frac": round(lane_ops / VALU_PEAK_LANE_OPS, 4),
                       "insts_per_node": round(insts * 64 / case.nodes, 1)}
    return rec


def measure_storage_variants(case, st, steps, warmup, kernel, copy_gbs, timed=None):
    """FP32 / FP16 / BF16 moment storage on the same workload: whole-step
    MLUPS and each storage's own update-kernel roofline.  `timed` reuses an
    already measured (mlups, kernel ms) pair for one storage."""
    kname = ("update_tiled", "update_direct", "push")[kernel]
    out = {}
    for storage, name in ((0, "fp32"), (1, "fp16"), (2, "bf16")):
        if timed and storage in timed:
            mlups, kms = timed[storage]
        else:
            s = _solver(case, storage, kernel)
            s.set_state(st)
            n_timed = min(max(steps, 50), 200)
            s.step(max(warmup, 20))
            kms, _ = s.step_timed(n_timed)
            kms /= n_timed
            ms, _ = time_steps(s, steps, warmup)
            s.close()
            mlups = case.nodes * steps / (ms * 1e-3) / 1e6
        out[name] = {"mlups": round(mlups, 1), "kernel_ms": round(kms, 5),
                     "roofline": kernel_roofline(case, storage, kms, kname, copy_gbs)}
    for name in ("fp16", "bf16"):
        out[name]["mlups_over_fp32"] = round(out[name]["mlups"] / out["fp32"]["mlups"], 3)
    return {"workload": case.name, "steps": steps, **out}


def measure_adjoint(kernel, n=64, nsteps=None):
    """Checkpointed rollout (every 20 steps) on an n^3 forced periodic box:
    forward and backward-with-recompute wall time, and one adjoint step
    against one update step (kernel only, event timed)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2401_17074_amd import capi as C
    case = W.adjoint_case(n=n) if nsteps is None else W.adjoint_case(n=n, steps=nsteps)
    st, g = W.adjoint_inputs(case)
    s = _solver(case, 0, kernel)
    s.set_force_field(g.astype(np.float32))
    s.set_state(_device_state(st))
    del st, g
    nsteps, every = case.steps, case.extra["ckpt"]
    ws = torch.empty(C.tslb_rollout_workspace_bytes(s.h, nsteps, every), dtype=torch.uint8, device="cuda")
    init = s.save_raw()
    # warm up both directions once
    C.tslb_rollout_forward(s.h, nsteps, every, ws)
    lam = s.adjoint_seed(s.save_raw())
    dg = torch.zeros((3,) + case.shape, dtype=torch.float32, device="cuda")
    C.tslb_rollout_backward(s.h, nsteps, every, ws, lam, dg)
    s.load_raw(init)
    s.t = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    C.tslb_rollout_forward(s.h, nsteps, every, ws)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    lam = s.adjoint_seed(s.save_raw())
    dg.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    C.tslb_rollout_backward(s.h, nsteps, every, ws, lam, dg)
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    del ws
    # kernel-only: one adjoint step vs one forward step, event timed
    raw0 = s.save_raw()
    s.step(1)
    raw1 = s.save_raw()
    lam_out = torch.empty_like(lam)
    reps = 50
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e[0].record()
    for _ in range(reps):
        C.tslb_adjoint_step(s.h, raw0, raw1, lam, lam_out, dg)
    e[1].record()
    e[2].record()
    s.step(reps)
    e[3].record()
    torch.cuda.synchronize()
    s.close()
    k_adj = e[0].elapsed_time(e[1]) / reps
    k_fwd = e[2].elapsed_time(e[3]) / reps
    del raw0, raw1, lam, lam_out, dg, init
    torch.cuda.empty_cache()
    return {"workload": case.name, "steps": nsteps, "checkpoint_every": every,
            "forward_ms_per_step": round(t_fwd * 1e3 / nsteps, 4),
            "backward_ms_per_step": round(t_bwd * 1e3 / nsteps, 4),
            "adjoint_over_forward": round(t_bwd / t_fwd, 3),
            "adjoint_kernel_ms": round(k_adj, 5), "update_kernel_ms": round(k_fwd, 5),
            "adjoint_kernel_over_update_kernel": round(k_adj / k_fwd, 3)}


def copy_rates_gbs(mib=1024, reps=20):
    """Bytes moved per second (read + write) by two plain device copies of
    `mib` MiB: the library's streaming copy kernel and the runtime's own
    device-to-device copy.  The faster is the practical ceiling of a
    read+write stream that the update's rate is compared with."""
    import torch
    from paper_2401_17074_amd import capi as C
    n = mib * (1 << 20) // 4
    a = torch.rand(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)

    def rate(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return 2.0 * n * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9

    lib = rate(lambda: C.tslb_stream_copy(b, a))
    ok = bool(torch.equal(a, b))
    rt = rate(lambda: b.copy_(a))
    del a, b
    torch.cuda.empty_cache()
    if not ok:
        raise RuntimeError("streaming copy produced a wrong result")
    return {"library_stream_copy": round(lib, 1), "runtime_copy": round(rt, 1)}


def fluid_nodes(case):
    """Nodes that are neither wall nor ghost (x fastest, product of the
    per-axis counts)."""
    count = 1
    for d, n in enumerate((case.nx, case.ny, case.nz)):
        lo, hi = case.faces[2 * d], case.faces[2 * d + 1]
        count *= n - (lo in (1, 2, 3)) - (hi in (1, 2, 3))
    return count


def _oracle_block_rate(case, st64, seconds_budget):
    """The FP64 oracle as it stands: single-step updates of a contiguous block
    of z-planes of the state, repeated until about seconds_budget of wall
    time; returns (MLUPS, description)."""
    import numpy as np
    import oracle
    G = oracle.make_grid(case.nx, case.ny, case.nz, case.tau, faces=case.faces, force=case.force)
    plane = case.nx * case.ny
    kinds = oracle.node_kinds(G).reshape(-1)
    # calibrate on one plane, then size the sample to the time budget
    idx = np.arange(plane, 2 * plane)
    idx = idx[kinds[idx] == 0]
    t0 = time.perf_counter()
    oracle.update_nodes(G, st64, idx)
    dt = time.perf_counter() - t0
    nplanes = int(max(1, min(case.nz - 2, seconds_budget / max(dt, 1e-6))))
    idx = np.arange(plane, (1 + nplanes) * plane)
    idx = idx[kinds[idx] == 0]
    reps = 0
    t0 = time.perf_counter()
    while True:
        oracle.update_nodes(G, st64, idx)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= 0.8 * seconds_budget or reps >= 100:
            break
    return reps * idx.size / dt / 1e6, ("%d x one FP64 update of %d fluid nodes (%d z-planes) of the %s initial state, "
                                         "%.1f s" % (reps, idx.size, nplanes, case.name, dt))


def oracle_sample(kind):
    """One bounded oracle timing, run in a child process (no GPU use) so that
    its OpenMP thread count can be set through the environment."""
    import numpy as np
    import oracle
    import workloads as W
    if kind == "single_core":
        case = W.channel_case(nx=512, ny=256, nz=6)
        rate, desc = _oracle_block_rate(case, W.channel_state(case), 5.0)
        return {"value": round(rate, 4), "unit": "MLUPS", "threads": oracle.num_threads(), "sample": desc}
    if kind == "tgv32":
        case = W.tgv_case()
        G = oracle.make_grid(case.nx, case.ny, case.nz, case.tau)
        st = W.tgv_state(case.nx, case.extra["u0"])
        t0 = time.perf_counter()
        oracle.run(G, st, case.steps)
        dt = time.perf_counter() - t0
        return {"value": round(case.nodes * case.steps / dt / 1e6, 4), "unit": "MLUPS", "seconds": round(dt, 2),
                "threads": oracle.num_threads(), "sample": "the whole run: 32^3 Taylor-Green, 100 FP64 steps"}
    if kind == "adjoint64":
        case = W.adjoint_case()
        st, g = W.adjoint_inputs(case)
        G = oracle.make_grid(case.nx, case.ny, case.nz, case.tau)
        t0 = time.perf_counter()
        st1 = oracle.step(G, st, g)
        t_f = time.perf_counter() - t0
        lam = oracle.ke_seed(G, st1)[1]
        t0 = time.perf_counter()
        oracle.adjoint_step(G, st, lam, g)
        t_a = time.perf_counter() - t0
        n, k = case.steps, case.extra["ckpt"]
        return {"forward_s_per_step": round(t_f, 3), "adjoint_s_per_step": round(t_a, 3),
                "rollout_s_extrapolated": round(n * t_f + n * (t_f + t_a), 1), "threads": oracle.num_threads(),
                "sample": "one FP64 step and one FP64 adjoint step of the 64^3 differentiable box; the %d-step "
                          "rollout with checkpoints every %d (forward, recompute, adjoint) extrapolated from them"
                          % (n, k)}
    raise ValueError(kind)


def _child_sample(kind, threads=None):
    import subprocess
    env = dict(os.environ)
    if threads:
        env["OMP_NUM_THREADS"] = str(threads)
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-sample", kind], capture_output=True,
                       text=True, env=env, timeout=300)
    if r.returncode != 0:
        return {"error": r.stderr.strip().splitlines()[-1:] or ["failed"]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(case, st64, seconds_budget=12.0):
    """The FP64 oracle as it stands, on the host cores: the headline value is
    single-step updates of a block of z-planes of the timed workload's own
    initial state on all threads; beside it the same on one thread, the
    32^3 Taylor-Green run, and one forward and one adjoint step of the 64^3
    differentiable box."""
    import oracle
    rate, desc = _oracle_block_rate(case, st64, seconds_budget)
    return {"value": round(rate, 4), "unit": "MLUPS", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": desc, "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS"),
            "single_core": _child_sample("single_core", threads=1),
            "taylor_green_32_100_steps": _child_sample("tgv32"),
            "adjoint_64": _child_sample("adjoint64")}


STORAGE_NAMES = ("fp32", "fp16", "bf16")


def _pmc_path(kernel_name, case_name, storage):
    suffix = "" if storage == 0 else "_" + STORAGE_NAMES[storage]
    return os.path.join(ROOT, "profiles", "pmc_%s_%s%s.json" % (kernel_name, case_name, suffix))


def load_traffic(kernel_name, case_name, storage):
    """HBM bytes per launch from a committed rocprofv3 counter summary, only
    if it was taken on the current kernel sources."""
    path = _pmc_path(kernel_name, case_name, storage)
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except ValueError:
        return None
    if rec.get("source_hash") != _source_hash() or rec.get("storage") != storage:
        return None
    return rec.get("hbm_bytes_per_launch")


def load_valu(kernel_name, case_name, storage):
    """VALU wave instructions per launch (SQ_INSTS_VALU) from the same
    counter summary, only if it was taken on the current kernel sources."""
    path = _pmc_path(kernel_name, case_name, storage)
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except ValueError:
        return None
    if rec.get("source_hash") != _source_hash() or rec.get("storage") != storage:
        return None
    return rec.get("valu_insts_per_dispatch")


def summarize_valu(args):
    """Add SQ_INSTS_VALU per update launch (a rocprofv3 --pmc run of its own)
    to the counter summary of the same workload and storage."""
    kname = ("update_tiled", "update_direct", "push")[args.kernel]
    insts, n = _counter_mean(args.summarize_valu, "SQ_INSTS_VALU", kname + "_kernel")
    import workloads as W
    case, _ = WORKLOADS[args.workload](W)
    path = _pmc_path(kname, case.name, args.storage)
    rec = json.load(open(path))
    if rec.get("source_hash") != _source_hash():
        raise SystemExit("%s was taken on other kernel sources" % path)
    rec["valu_insts_per_dispatch"] = insts
    rec["valu_dispatches"] = n
    json.dump(rec, open(path, "w"), indent=1)
    print(json.dumps(rec))


def _counter_mean(folder, counter, name_part):
    import csv
    import glob
    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    vals = []
    for f in files:
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] == counter and name_part in r["Kernel_Name"]:
                vals.append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit("no %s samples for %s in %s" % (counter, name_part, folder))
    return sum(vals) / len(vals), len(vals)


def summarize_pmc(args):
    """HBM bytes per launch of the update kernel from FETCH_SIZE / WRITE_SIZE
    (KiB per dispatch), each scaled by what the same counter reads for a plain
    copy of known size (bench.py --copy-calibration 1024: the library's streaming
    copy kernel, 1 GiB read + 1 GiB written per launch)."""
    fdir, wdir, cfdir, cwdir = args.summarize_pmc
    kname = ("update_tiled", "update_direct", "push")[args.kernel]
    fetch, nf = _counter_mean(fdir, "FETCH_SIZE", kname + "_kernel")
    write, nw = _counter_mean(wdir, "WRITE_SIZE", kname + "_kernel")
    cfetch, _ = _counter_mean(cfdir, "FETCH_SIZE", "stream_copy_kernel")
    cwrite, _ = _counter_mean(cwdir, "WRITE_SIZE", "stream_copy_kernel")
    copy_kib = 1024.0 * 1024.0  # 1 GiB each way
    ffac, wfac = copy_kib / cfetch, copy_kib / cwrite
    import workloads as W
    case, _ = WORKLOADS[args.workload](W)
    algo = algorithmic_bytes(case, args.storage)
    rec = {"kernel": kname, "workload": case.name, "storage": args.storage, "source_hash": _source_hash(),
           "fetch_kib_per_dispatch": fetch, "write_kib_per_dispatch": write, "dispatches": [nf, nw],
           "copy_fetch_factor": ffac, "copy_write_factor": wfac,
           "hbm_bytes_per_launch": (fetch * ffac + write * wfac) * 1024.0,
           "algorithmic_bytes_per_launch": algo}
    rec["traffic_over_algorithmic"] = rec["hbm_bytes_per_launch"] / algo
    path = _pmc_path(kname, case.name, args.storage)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    json.dump(rec, open(path, "w"), indent=1)
    print(json.dumps(rec))


WORKLOADS = {
    "channel": lambda W: (lambda c: (c, W.channel_state(c)))(W.channel_case()),
    "channel512": lambda W: (lambda c: (c, W.channel_state(c)))(W.channel_case(nx=512, ny=256, nz=256)),
    "jet": lambda W: (lambda c: (c, W.jet_state(c)))(W.jet_case()),
    "paper_jet": lambda W: (lambda c: (c, W.jet_state(c)))(W.paper_jet_case()),
    "channel2d": lambda W: (lambda c: (c, W.channel2d_state(c)))(W.channel2d_case()),
    "channel_d3q19": lambda W: (lambda c: (c, W.channel_state(c)))(W.channel_case(lattice=19)),
    "cube512": lambda W: (lambda c: (c, W.tgv_state(c.nx, 0.01)))(W.tgv_case(n=512)),
    "tgv32": lambda W: (lambda c: (c, W.tgv_state(c.nx, 0.01)))(W.tgv_case()),
}


def measure_workloads(names, steps, warmup, kernel):
    """MLUPS and HBM roofline fraction of the update kernel on the other
    synthetic workloads (same bytes-per-node accounting as the headline)."""
    import workloads as W
    out = {}
    for name in names:
        case, st64 = WORKLOADS[name](W)
        s = _solver(case, 0, kernel)
        s.set_state(_device_state(st64))
        ms, _ = time_steps(s, steps, warmup)
        kms, _ = s.step_timed(steps)
        s.close()
        gbs = algorithmic_bytes(case, 0) / (kms * 1e-3 / steps) / 1e9
        out[case.name] = {"mlups": round(case.nodes * steps / (ms * 1e-3) / 1e6, 1),
                          "kernel_ms": round(kms / steps, 5), "hbm_gbs": round(gbs, 1),
                          "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    return {"steps": steps, **out}


def measure_stats_cost(case, st, samples):
    """Cost of one statistics sample on the device (profile sums along y and
    per-node FP64 sums), event-timed over `samples` samples of the state."""
    import torch
    s = _solver(case, 0, 0)
    s.set_state(st)
    out = {}
    for name, kw in (("profile", {"profile_axis": 1}), ("field", {"field": True})):
        s.stats_begin(**kw)
        s.stats_sample()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(samples):
            s.stats_sample()
        e1.record()
        torch.cuda.synchronize()
        out[name + "_ms_per_sample"] = round(e0.elapsed_time(e1) / samples, 5)
    s.close()
    return {"workload": case.name, "samples": samples, **out}


def measure_order_variants(case, st, steps, warmup, kernel):
    """Third-order update against the regularised second-order one
    (Eq. (fullstrcoll)) on the same workload: the cost of the high-order
    reconstruction."""
    out = {}
    for order in (3, 2):
        s = _solver(case, 0, kernel, order)
        s.set_state(st)
        ms, _ = time_steps(s, steps, warmup)
        kms, _ = s.step_timed(steps)
        s.close()
        out["order%d" % order] = {"mlups": round(case.nodes * steps / (ms * 1e-3) / 1e6, 1),
                                  "kernel_ms": round(kms / steps, 5)}
    return {"workload": case.name, "steps": steps, **out}


def measure_layout_variants(case, st, steps, warmup):
    """The moment-only layout (tiled kernel) against the paper's own layout,
    one population set plus the moments (push pass + moment pass), on the
    same workload.  Algorithmic bytes per node: 10 + 10 stored values against
    10 + 27 + 27 + 10."""
    out = {}
    fl = _fluid_nodes(case)
    for kernel, name, vals in ((0, "moments_only", 10 * case.nodes + 10 * fl),
                               (2, "populations_plus_moments", 37 * case.nodes + 37 * fl)):
        s = _solver(case, 0, kernel)
        s.set_state(st)
        ms, _ = time_steps(s, steps, warmup)
        kms, _ = s.step_timed(steps)
        s.close()
        out[name] = {"mlups": round(case.nodes * steps / (ms * 1e-3) / 1e6, 1),
                     "update_ms": round(kms / steps, 5),
                     "algorithmic_bytes_per_step": 4 * vals,
                     "hbm_gbs": round(4 * vals / (kms * 1e-3 / steps) / 1e9, 1)}
    return {"workload": case.name, "steps": steps, **out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--kernel", type=int, default=0, help="0 tiled (default), 1 direct, 2 population layout")
    ap.add_argument("--workload", default="channel512", choices=sorted(WORKLOADS),
                    help="timed workload (default: the 512x256x256 channel of the precision workload)")
    ap.add_argument("--quick", action="store_true", help="only the timed workload (for profiling)")
    ap.add_argument("--order", type=int, default=3, choices=(2, 3),
                    help="Hermite order of the timed workload (2: the regularised collision, for profiling)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--storage", type=int, default=0, choices=(0, 1, 2),
                    help="moment storage of the timed workload: 0 FP32 (default), 1 FP16, 2 BF16")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run the library's streaming copy of MIB MiB 20 times (HBM counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="turn four rocprofv3 --pmc output folders into profiles/pmc_<kernel>_<workload>.json")
    ap.add_argument("--summarize-valu", metavar="VALU_DIR",
                    help="add SQ_INSTS_VALU per launch from a rocprofv3 --pmc output folder to the counter summary")
    ap.add_argument("--adjoint", type=int, default=0, metavar="N",
                    help="only the checkpointed-rollout and adjoint-kernel timing on the N^3 forced box (for profiling)")
    ap.add_argument("--oracle-sample", choices=("single_core", "tgv32", "adjoint64"),
                    help="(internal) time one bounded oracle sample on the host and print it as JSON")
    args = ap.parse_args()
    if args.oracle_sample:
        print(json.dumps(oracle_sample(args.oracle_sample)))
        return
    if args.summarize_pmc:
        summarize_pmc(args)
        return
    if args.summarize_valu:
        summarize_valu(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs the update on a single MI355X and has no "
              "multi-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.adjoint:
        import torch
        torch.cuda.set_device(0)
        rec = measure_adjoint(args.kernel, n=args.adjoint, nsteps=None if args.adjoint <= 64 else 100)
        # per node: M_t 40 B, rho' and u' 16 B, lambda_{t+1} 40 B, the force
        # field 12 B, lambda_t 40 B written, dg read and written 24 B
        algo = 172 * args.adjoint ** 3
        rec["adjoint_algorithmic_bytes_per_launch"] = algo
        rec["adjoint_kernel_gbs"] = round(algo / (rec["adjoint_kernel_ms"] * 1e-3) / 1e9, 1)
        print(json.dumps(rec))
        return
    if args.copy_calibration:
        import torch
        from paper_2401_17074_amd import capi as C
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(20):
            C.tslb_stream_copy(b, a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 2 * n * 4, "launches": 20}))
        return

    import torch
    import workloads as W
    torch.cuda.set_device(0)

    case, st64 = WORKLOADS[args.workload](W)
    st_dev = _device_state(st64)
    s = _solver(case, args.storage, args.kernel, args.order)
    s.set_state(st_dev)
    # the dominant kernel alone: HIP events around each of its launches, on
    # the stream it runs on (the library's; the default stream here).  Taken
    # after untimed steps and before the whole-step timing, so that neither
    # measurement starts on a GPU still at its idle clocks (short runs would
    # otherwise carry the ramp-up)
    n_timed = min(max(args.steps, 50), 200)
    s.step(max(args.warmup, 20))
    kms, aux_ms = s.step_timed(n_timed)
    ms, wall = time_steps(s, args.steps, args.warmup)
    _, rc = s.reduce(check=False)
    s.close()
    mlups = case.nodes * args.steps / (ms * 1e-3) / 1e6
    copies = copy_rates_gbs()
    copy_gbs = max(copies.values())
    kname = "update_d2q9" if case.lattice == 9 else ("update_tiled", "update_direct", "push")[args.kernel]
    roof = kernel_roofline(case, args.storage, kms / n_timed, kname, copy_gbs)
    roof["aux_ms_per_step"] = round(aux_ms / n_timed, 5)
    roof["copy_rates_gbs"] = copies
    rec = {
        "metric": "MLUPS and % of HBM roofline (FP32 vs FP16-moment); adjoint step time / forward",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": case.name, "nodes": case.nodes, "lattice": {9: "D2Q9", 19: "D3Q19"}.get(case.lattice, "D3Q27"),
                   "tau": case.tau,
                   "storage": STORAGE_NAMES[args.storage], "faces": list(case.faces), "kernel": kname, "order": args.order,
                   "stable": rc == 0},
        "fluid_mlups": round(fluid_nodes(case) * args.steps / (ms * 1e-3) / 1e6, 1),
        "roofline": roof,
        "wall_s": round(wall, 3),
    }
    if not args.quick:
        timed = {args.storage: (mlups, kms / n_timed)} if args.order == 3 and case.lattice == 27 else None
        rec["storage_variants"] = measure_storage_variants(case, st_dev, 200, 10, args.kernel, copy_gbs, timed)
        del st_dev
        ch, ch_st = WORKLOADS["channel"](W)
        rec["order_variants"] = measure_order_variants(ch, _device_state(ch_st), 200, 10, args.kernel)
        rec["layout_variants"] = measure_layout_variants(ch, _device_state(ch_st), 200, 10)
        rec["statistics"] = measure_stats_cost(ch, _device_state(ch_st), 50)
        del ch_st
        rec["other_workloads"] = measure_workloads(["channel", "cube512", "jet", "paper_jet", "channel2d",
                                                    "channel_d3q19"], 100, 5, args.kernel)
        rec["adjoint"] = measure_adjoint(args.kernel)
        rec["adjoint_256"] = measure_adjoint(args.kernel, n=256, nsteps=100)
        if not args.no_cpu:
            rec["cpu_baseline"] = cpu_baseline(case, st64)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
