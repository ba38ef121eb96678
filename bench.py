"""Benchmark of the SPG reconstruction on one MI355X.

One step = one whole solve of the precision-512 workload: set the data (fold and
checks), 3 reweighting rounds x 100 SPG iterations from x = 0 (two reweights in
between), fetch the map and run the fp64 objective / KKT check.  Inputs are resident
in HBM before the timed region starts.  The JSON line reports SPG iterations per
second, the per-kernel device time from HIP events recorded on the solver's stream
during the timed steps, the roofline of the dominant kernel, and the FP64 oracle
timed on the host cores on a bounded sample (three iterations of the same workload).

Other workloads (one JSON line each):
  --config 1   32^3 plain, 50 iterations: eager launches against one replayed HIP graph
  --config 2   256^3 reweighting workload, 3 x 100 (the same step as the default)
  --config 4   8-volume batch {128..256}^3 in one HIP graph, 200 iterations each
  --config 5   128^3 differentiation: forward + reverse (adjoint) against the plain forward
  --storage    fp32 | bf16 | compensated (default) iterate / map storage

  python bench.py [--steps K] [--warmup W] [--config 3] [--no-cpu-baseline]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SPG iterations/sec and HBM GB/s at 512^3 FP32 (rel. L2 ≤1e-5 vs FP64 oracle)"
# measured HBM bytes per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE, copy-calibrated)
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "hbm_traffic_solve_512.txt")
HBM_PEAK_GBPS = 8000.0


def kernel_bytes(shape, storage="compensated"):
    """Algorithmic HBM bytes per launch of each kernel class (each array read or written once).

    Returned as functions of the launch kind where the traffic depends on it (the stencil
    kernel reads x_{k-1} only when the momentum is non-zero and u, v only when explicit).
    Storage: 'compensated' (fp32 + bf16 iterate words), 'fp32', or 'bf16' (fp32 iterate,
    bf16 penalty weights and gradient / extrapolated map).
    """
    nz, ny, nx = shape
    n = nx * ny * nz
    spec = 4 * n           # packed half spectrum, complex64: nz*ny*(nx/2)*8
    xb = 6 if storage == "compensated" else 4
    rb = 2 if storage == "bf16" else 4    # map buffer and penalty weights
    col = ny * nz
    return {
        "fft_y_fwd": 2 * spec,
        "fft_z_weight": 2 * spec + spec // 2 + spec,          # S in/out, w~ (fp32), c (complex64)
        "dc_nyquist": col * (8 + 4 + 4 + 8 + 8 + 8),           # the packed kx=0 column in/out + its weights
        "fft_y_inv": 2 * spec,
        "c2r_x": spec + rb * n,
        "r2c_x": rb * n + spec,
        # gradient map in, y' out, x_k in, x_{k+1} out, [x_{k-1} in], [u, v in]
        "prox_tv": lambda momentum, explicit_uv: (rb + rb + xb + xb + (xb if momentum else 0)
                                                  + (2 * rb if explicit_uv else 0)) * n,
        # fused x transforms: gradient spectrum rows in, spectrum of y' out, x_k in,
        # x_{k+1} out, [x_{k-1} in], [u, v in]
        "prox_fft": lambda momentum, explicit_uv: 2 * spec + (xb + xb + (xb if momentum else 0)
                                                              + (2 * rb if explicit_uv else 0)) * n,
        # check mode: fp32 gradient in, x in, [u, v in]
        "prox_tv_check": lambda explicit_uv: (4 + xb + (2 * rb if explicit_uv else 0)) * n,
        "r2c_x_check": 4 * n + spec,
        "c2r_x_check": spec + 4 * n,
    }


def schedule_bytes(shape, rounds, iters, steps, storage="compensated", fused=False):
    """Total algorithmic bytes per kernel class over `steps` solves of the schedule (fused:
    the x-axis transforms of each iteration run inside the stencil/prox kernel)."""
    kb = kernel_bytes(shape, storage)
    sweeps = ["fft_y_fwd", "fft_z_weight", "dc_nyquist", "fft_y_inv"] + ([] if fused else ["c2r_x", "r2c_x"])
    tot = {k: 0 for k in ["fft_y_fwd", "fft_z_weight", "dc_nyquist", "fft_y_inv", "c2r_x", "prox_tv", "r2c_x"]}
    launches = {k: 0 for k in tot}
    for _ in range(steps):
        for r in range(rounds):
            explicit = r > 0
            for j in range(1, iters + 1):
                for k in sweeps:
                    tot[k] += kb[k]
                    launches[k] += 1
                tot["prox_tv"] += kb["prox_fft" if fused else "prox_tv"](j >= 3, explicit)
                launches["prox_tv"] += 1
            tot["r2c_x"] += kb["r2c_x"]      # priming transform at the start of each round
            launches["r2c_x"] += 1
        # final check: one more forward/inverse pipeline (fp32 map in, fp32 gradient out) and
        # the stencil in check mode
        for k in ["fft_y_fwd", "fft_z_weight", "dc_nyquist", "fft_y_inv"]:
            tot[k] += kb[k]
            launches[k] += 1
        for k in ["c2r_x", "r2c_x"]:
            tot[k] += kb[k + "_check"]
            launches[k] += 1
        tot["prox_tv"] += kb["prox_tv_check"](rounds > 1)
        launches["prox_tv"] += 1
    return tot, launches


def schedule_iteration_bytes(shape, rounds, iters, storage="compensated", fused=False):
    """Mean algorithmic bytes of one SPG iteration over the schedule: round 1 has uniform
    penalty weights (u, v not read), later rounds explicit ones; the first two iterations of
    a round have no momentum term (x_{k-1} not read).  Priming and the final check are not
    iterations and are left out."""
    kb = kernel_bytes(shape, storage)
    sweeps = ["fft_y_fwd", "fft_z_weight", "dc_nyquist", "fft_y_inv"] + ([] if fused else ["c2r_x", "r2c_x"])
    per_sweep = sum(kb[k] for k in sweeps)
    tot = 0
    for r in range(rounds):
        for j in range(1, iters + 1):
            tot += per_sweep + kb["prox_fft" if fused else "prox_tv"](j >= 3, r > 0)
    return tot / (rounds * iters)


def iteration_bytes(shape, explicit_uv=True, storage="compensated", fused=False):
    kb = kernel_bytes(shape, storage)
    if fused:
        return sum(kb[k] for k in ["fft_y_fwd", "fft_z_weight", "dc_nyquist", "fft_y_inv"]) + \
            kb["prox_fft"](True, explicit_uv)
    return sum(kb[k] for k in ["fft_y_fwd", "fft_z_weight", "dc_nyquist", "fft_y_inv", "c2r_x", "r2c_x"]) + \
        kb["prox_tv"](True, explicit_uv)


def plain_iteration_bytes(shape, explicit_uv):
    """A byte model of the path with a plain fp32 iterate and four HBM sweeps per iteration,
    independent of this implementation's storage choices: the fused real-space kernel reads x_k, x_{k-1}, [u, v] and the gradient
    spectrum and writes x_{k+1} and the spectrum of y_{k+1} (5R + 2H with explicit u, v, else
    3R + 2H), the y passes 2H each and the z pass 3.5H, with R = 4 n and H = 8 nz ny (nx/2 + 1)
    (the unpacked half spectrum).  Returns (stencil kernel bytes, whole iteration bytes)."""
    nz, ny, nx = shape
    n = nx * ny * nz
    R = 4 * n
    H = 8 * nz * ny * (nx // 2 + 1)
    prox = (5 * R if explicit_uv else 3 * R) + 2 * H
    return prox, prox + 2 * H + 3.5 * H + 2 * H


def plain_schedule_mean(shape, rounds):
    """Mean of plain_iteration_bytes over a schedule whose first round has uniform u, v."""
    vals = [plain_iteration_bytes(shape, r > 0) for r in range(rounds)]
    return sum(v[0] for v in vals) / rounds, sum(v[1] for v in vals) / rounds


def cpu_baseline(vol, c):
    """The FP64 oracle, as it stands, timed for three SPG iterations of the same workload."""
    import numpy as np

    from oracle import spg_ref as O

    p = O.Problem(w=vol.w.astype(np.float64), b=vol.b.astype(np.complex128), lam=c["lam"], mu=c["mu"], eps=c["eps"])
    lr = 1.0 / O.lipschitz(p)
    x = np.zeros(c["shape"])
    t0 = time.perf_counter()
    n_it = 3
    O.spg_solve(p, n_it, x0=x, lr=lr)
    dt = time.perf_counter() - t0
    cores = O.fft_workers()
    return {"value": n_it / dt, "unit": "iterations/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_it} SPG iterations of the {c['shape'][0]}^3 workload (float64 NumPy, scipy.fft with "
                      f"{cores} workers), {dt:.1f} s wall"}


def copy_ceiling(gib: float = 1.0, reps: int = 5, how=("copy", "scale")) -> dict:
    """Plain device copies of known size: read + write bytes per second of the best of `reps`
    runs (HIP events) of the runtime's device copy and of a vectorised elementwise kernel
    (b = 1 * a); the faster is the practical HBM ceiling beside the 8 TB/s peak."""
    import torch

    n = int(gib * (1 << 30)) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    ops = {"copy": lambda: b.copy_(a), "scale": lambda: torch.mul(a, 1.0, out=b)}
    res = {}
    for name in how:
        ops[name]()
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ops[name]()
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        res[name] = 2 * n * 4 / (best * 1e-3) / 1e9
    del a, b
    top = max(res, key=res.get)
    return {"copy_bytes_each_way": n * 4, "reps": reps, "GBps_read_plus_write": res[top], "by": top,
            "GBps_each": res}


def copy_calibration(gib: float = 1.0, reps: int = 5):
    """A plain device copy of known size, for scaling HBM counters (FETCH_SIZE / WRITE_SIZE)."""
    print(json.dumps(copy_ceiling(gib, reps, how=("copy",))))


BATCH_SIZES = [128, 160, 192, 256, 256, 192, 160, 128]


def batch_members(seed=0):
    """The batching workload: two half-maps and six class volumes of uneven boxes, each with
    its own blob truth (0.003 blobs per voxel on chains of 250), SNR ~ U[0.3, 1] and lambda,
    mu = (0.01, 0.05) x U[0.5, 2] each."""
    import numpy as np

    from paper_1905_13408_amd import synth

    rng = np.random.default_rng(np.random.SeedSequence([seed, 4, 999]))
    out = []
    for i, n in enumerate(BATCH_SIZES):
        nb = int(0.003 * n ** 3)
        snr = float(rng.uniform(0.3, 1.0))
        lam = 0.01 * float(rng.uniform(0.5, 2.0))
        mu = 0.05 * float(rng.uniform(0.5, 2.0))
        vol = synth.make_volume((n, n, n), nb, max(1, nb // 250), 1.2, 0.39 * n, snr, seed=seed, config_id=4,
                                volume_id=i)
        out.append(((n, n, n), vol, lam, mu))
    return out


def batch_roofline(members, shapes_tuned, iters, storage, sec_per_step):
    tot = sum(schedule_iteration_bytes(tuple(int(v) for v in shape), 1, iters, storage, bool(tuned[3])) * iters
              for (shape, _, _, _), tuned in zip(members, shapes_tuned))
    ach = tot / sec_per_step / 1e9
    return {"scope": "whole batch step (all members)", "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBPS,
            "unit": "GB/s", "frac": ach / HBM_PEAK_GBPS, "traffic": None, "bytes_per_step": tot}


def bench_batch(args):
    """8 volumes x `iters` SPG iterations: one HIP graph per step versus eager launches."""
    import torch

    from paper_1905_13408_amd import spg

    iters = args.iters or 200
    t_gen = time.perf_counter()
    members = batch_members()
    print(f"# batch inputs generated in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    solvers = []
    shapes_tuned = []
    for shape, vol, lam, mu in members:
        sv = spg.SPGSolver(shape, lam, mu, 1e-3, storage=args.storage)
        sv.set_data(torch.from_numpy(vol.w).cuda(), torch.from_numpy(vol.b).cuda())
        shapes_tuned.append(list(sv.autotune(8) if not args.no_autotune else sv.launch_shape()) + [sv.fusion])
        solvers.append(sv)
    batch = spg.SPGBatch(solvers)
    vox_it = sum(int(sh[0]) ** 3 for sh, _, _, _ in members) * iters

    def graph_step():
        for sv in solvers:
            sv.set_map(None)
        batch.run(iters)

    def eager_step():
        for sv in solvers:
            sv.set_map(None)
            sv.run(iters)

    res = {}
    for name, fn in [("graph", graph_step), ("eager", eager_step)]:
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0) / args.steps
    line = {
        "metric": "SPG volume-iterations/s, 8-volume batch {128,160,192,256,256,192,160,128}^3 in one HIP graph",
        "value": len(solvers) * iters / res["graph"],
        "unit": "volume-iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * res["graph"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch-8: boxes {BATCH_SIZES}, 0.003 blobs/voxel, SNR U[0.3,1], lambda/mu x U[0.5,2], "
                               f"{iters} SPG iterations each", "storage": args.storage},
        "voxel_iterations_per_s": vox_it / res["graph"],
        "eager_ms_per_step": 1e3 * res["eager"],
        # the whole batch step against 8 TB/s: every member's algorithmic bytes (one round from
        # a zero map: uniform penalty weights, momentum from the third iteration); maps of
        # 128^3-256^3 are partly served by the last-level cache, so this is an effective rate
        "roofline": batch_roofline(members, shapes_tuned, iters, args.storage, res["graph"]),
        "graph_speedup_vs_eager": res["eager"] / res["graph"],
        "launch_shapes_nt_y_nt_z_zc_fused": shapes_tuned,
    }
    print(json.dumps(line))
    batch.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--iters", type=int, default=None, help="override SPG iterations per round")
    ap.add_argument("--storage", choices=["compensated", "fp32", "bf16"], default="compensated",
                    help="iterate / map storage mode")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="time without per-kernel HIP events")
    ap.add_argument("--copy-calib", action="store_true", help="only run the copy kernel used to scale HBM counters")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--launch-shape", type=int, nargs=3, metavar=("NT_Y", "NT_Z", "ZC"), default=None,
                    help="fix the launch shape instead of autotuning it")
    ap.add_argument("--no-fusion", action="store_true", help="run the x-axis transforms as separate sweeps")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build runs a single SPG problem per device and has no "
              "multi-GPU path; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calib:
        copy_calibration()
        return
    if args.config == 4:
        bench_batch(args)
        return
    if args.config == 1:
        bench_small(args)
        return
    if args.config == 5:
        bench_diff(args)
        return

    from paper_1905_13408_amd import profiling, spg, synth

    t_gen = time.perf_counter()
    vol, c = synth.make_config(args.config)
    if args.iters:
        c["iters"] = args.iters
    print(f"# inputs generated in {time.perf_counter() - t_gen:.1f} s: {c['name']} {c['shape']}", file=sys.stderr,
          flush=True)
    shape = c["shape"]
    storage = args.storage
    w = torch.from_numpy(vol.w).cuda()
    b = torch.from_numpy(vol.b).cuda()
    out = torch.empty(shape, dtype=torch.float32, device="cuda")
    solver = spg.SPGSolver(shape, c["lam"], c["mu"], c["eps"], storage=storage)
    if args.no_fusion:
        solver.set_fusion(False)
    rounds, iters = c["rounds"], c["iters"]
    solver.set_data(w, b)
    # tune in the state of the reweighted rounds: explicit penalty weights are read (their
    # values do not change the timing); every step below starts from uniform weights again
    ones = torch.ones(shape, dtype=torch.float32, device="cuda")
    solver.set_penalty_weights(ones, ones)
    if args.launch_shape:
        solver.set_launch_shape(*args.launch_shape)
        launch_shape = solver.launch_shape()
    else:
        launch_shape = solver.launch_shape() if args.no_autotune else solver.autotune(8)
    del ones
    if args.no_fusion:
        solver.set_fusion(False)
    fused = solver.fusion
    print(f"# launch shape (nt_y, nt_z, zc) = {launch_shape}, fused x transforms: {fused}", file=sys.stderr,
          flush=True)

    result = {}

    def step():
        solver.set_data(w, b)
        solver.set_penalty_weights(None, None)
        solver.set_map(None)
        for r in range(rounds):
            if r > 0:
                solver.reweight(c["eps1"], c["eps2"])
            solver.run(iters)
        solver.get_map(out)
        result["check"] = solver.final_check()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("# warmup done", file=sys.stderr, flush=True)

    # One untimed step with HIP events around every kernel gives the per-kernel table and
    # names the dominant kernel; the timed steps record events around that kernel only
    # (events around all seven classes cost about 2% of the step time).
    # (large maps run the y, z, y passes on four column ranges: four launches per pass)
    cap = 4 * (rounds * (iters + 1) + 2)
    prof_all, dom = None, None
    if not args.no_profile:
        solver.profile_begin(None, cap)
        step()
        prof_all = solver.profile_end()
        # a class that filled its event capacity would be undercounted
        assert all(n < cap for _, n in prof_all.values()), prof_all
        dom = max(prof_all, key=lambda k: prof_all[k][0])
        solver.profile_begin(dom, args.steps * cap)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof_dom = solver.profile_end()[dom] if not args.no_profile else None
    print("# timed steps done", file=sys.stderr, flush=True)

    elapsed = t1 - t0
    total_iters = rounds * iters * args.steps
    value = total_iters / elapsed
    it_bytes = schedule_iteration_bytes(shape, rounds, iters, storage, fused)
    _, plain_it = plain_schedule_mean(shape, rounds)
    line = {
        "metric": METRIC if args.config == 3 else METRIC.replace("512^3", f"{shape[0]}^3"),
        "value": value,
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{c['name']}: {shape[0]}x{shape[1]}x{shape[2]}, {c['n_blobs']} Gaussian blobs on "
                               f"{c['n_chains']} chains, SNR {c['snr']}, lambda {c['lam']}, mu {c['mu']}, eps "
                               f"{c['eps']}, {rounds} rounds x {iters} SPG iterations, reweight floors "
                               f"{c['eps1']}/{c['eps2']}",
                   "iterate_storage": {"compensated": "fp32 hi + bf16 lo iterate, fp64 prox",
                                       "fp32": "fp32 iterate",
                                       "bf16": "fp32 iterate, bf16 weights and map buffer"}[storage],
                   "step": "set data + solve + fetch map + fp64 objective/KKT check",
                   "x_transforms": "fused into the stencil/prox kernel" if fused else "separate sweeps",
                   "launch_shape_nt_y_nt_z_zc": list(launch_shape)},
        "ms_per_iteration": 1e3 * elapsed / total_iters,
        "model_bytes_per_iteration": it_bytes,
        "model_GBps": it_bytes * value / 1e9,
        "plain_fp32_model_bytes_per_iteration": plain_it,
        "plain_fp32_model_GBps": plain_it * value / 1e9,
        "plain_fp32_model_frac_of_peak": plain_it * value / 1e9 / HBM_PEAK_GBPS,
        "final_objective": result["check"][0],
        "final_kkt_rel": result["check"][2],
    }
    if prof_all is not None:
        # per-kernel table: the untimed profiled step (one solve)
        tot1, launches1 = schedule_bytes(shape, rounds, iters, 1, storage, fused)
        kern = {}
        for k, (ms, n) in prof_all.items():
            if n:
                # us_avg per launch; us_per_pass per pass over the map (a pass may be
                # launched as several column ranges)
                kern[k] = {"ms_total": ms, "launches": n, "us_avg": 1e3 * ms / n,
                           "us_per_pass": 1e3 * ms / launches1[k] if launches1[k] else None,
                           "GBps": tot1[k] / (ms * 1e-3) / 1e9 if ms > 0 else None,
                           "model_launches": launches1[k]}
        line["kernels_profiled_step"] = kern
        line["kernel_ms_per_iteration"] = sum(v["ms_total"] for v in kern.values()) / (rounds * iters)
        # roofline of the dominant kernel: its events in the timed steps
        tot_bytes, launches = schedule_bytes(shape, rounds, iters, args.steps, storage, fused)
        ms_dom, n_dom = prof_dom
        assert n_dom == launches[dom], (n_dom, launches[dom])
        bytes_per_launch = tot_bytes[dom] / n_dom
        t_avg = ms_dom * 1e-3 / n_dom
        ach = bytes_per_launch / t_avg / 1e9
        traffic = None
        rec = profiling.load(TRAFFIC_RECORD) if (args.config == 3 and storage == "compensated" and
                                                   not args.iters and fused == profiling.record_fused(TRAFFIC_RECORD)) \
            else None
        if rec and dom in rec["per_launch"]:
            e = rec["per_launch"][dom]
            traffic = e["fetch_bytes"] + e["write_bytes"]
        line["roofline"] = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                            "frac": ach / HBM_PEAK_GBPS, "traffic": traffic,
                            "bytes_per_launch": bytes_per_launch, "us_per_launch": t_avg * 1e6}
        if dom == "prox_tv" and fused:
            # the same launches priced with the plain fp32 byte model (unpacked half spectrum):
            # what the method must move, whatever the storage
            sp, _ = plain_schedule_mean(shape, rounds)
            line["roofline"]["plain_fp32_model"] = {"bytes_per_launch": sp, "achieved": sp / t_avg / 1e9,
                                                "frac": sp / t_avg / 1e9 / HBM_PEAK_GBPS}
    # the practical HBM ceiling (a 1 GiB device copy, outside the timed steps) and the whole
    # iteration's algorithmic bytes against it
    cc = copy_ceiling()
    line["copy_ceiling_GBps"] = cc["GBps_read_plus_write"]
    line["copy_ceiling_by"] = cc["by"]
    line["model_frac_of_copy_ceiling"] = line["model_GBps"] / cc["GBps_read_plus_write"]
    if args.config == 2:
        line["hbm_note"] = ("256^3: about 1 GB per iteration against the 256 MiB last-level (Infinity) cache, "
                            "so part of the traffic is served from it: GB/s figures are effective, not HBM")
    if not args.no_cpu_baseline:
        print("# cpu baseline (FP64 oracle, three iterations)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(vol, c)
    print(json.dumps(line))


def bench_small(args):
    """The 32^3 plain workload (50 SPG iterations from x = 0, uniform weights): launch-bound, so
    iterations per second are given for eager launches (5 kernels per iteration; the value) and
    for the 50 iterations captured once as a HIP graph and replayed."""
    import torch

    from paper_1905_13408_amd import spg, synth

    vol, c = synth.make_config(1)
    iters = args.iters or c["iters"]
    s = spg.SPGSolver(c["shape"], c["lam"], c["mu"], c["eps"], storage=args.storage)
    s.set_data(torch.from_numpy(vol.w).cuda(), torch.from_numpy(vol.b).cuda())
    launch_shape = s.launch_shape() if args.no_autotune else s.autotune(8)
    batch = spg.SPGBatch([s])
    res = {}
    for name, run in [("eager", lambda: s.run(iters)), ("graph", lambda: batch.run(iters))]:
        for _ in range(args.warmup + 1):
            s.set_map(None)
            run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            s.set_map(None)
            run()
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0) / args.steps
    batch.close()
    line = {
        "metric": "SPG iterations/sec at 32^3 (launch-bound)",
        "value": iters / res["eager"], "unit": "iterations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * res["eager"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.storage != "bf16" else "f32/bf16", "data": "synthetic",
        "config": {"workload": f"plain-32: 32x32x32, 60 Gaussian blobs on 1 chain, SNR 1, lambda {c['lam']}, "
                               f"mu {c['mu']}, eps {c['eps']}, {iters} SPG iterations from x = 0",
                   "storage": args.storage},
        "graph_iterations_per_s": iters / res["graph"],
        "graph_speedup_vs_eager": res["eager"] / res["graph"],
        "launch_shape_nt_y_nt_z_zc": list(launch_shape), "x_transforms": "fused" if s.fusion else "separate",
        "step": "set_map + the iterations, launched eagerly (graph: one HIP graph of all of them, replayed)",
    }
    print(json.dumps(line))


def bench_diff(args):
    """The differentiation workload (128^3, 50 unrolled iterations, checkpoint every 10): the
    plain forward solve against the checkpointed forward and the reverse pass (spg_vjp) that
    gives d loss / d (lambda, mu, b) for loss = |x_50 - x_true|^2."""
    import torch

    from paper_1905_13408_amd import spg, synth

    vol, c = synth.make_config(5)
    K, C = c["iters"], 10
    w = torch.from_numpy(vol.w).cuda()
    s = spg.SPGSolver(c["shape"], c["lam"], c["mu"], c["eps"])
    s.set_data(w, torch.from_numpy(vol.b).cuda())
    xt = torch.from_numpy(vol.x_true).cuda()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    def plain():
        s.set_map(None)
        s.run(K)

    def fwd_rev():
        s.set_map(None)
        s.run_checkpointed(K, C)
        x = s.get_map()
        s.vjp(w, 2.0 * (x - xt))

    reps = max(1, args.steps)
    t_plain = timed(plain, reps)
    t_both = timed(fwd_rev, reps)
    line = {
        "metric": "SPG forward + reverse (adjoint) time at 128^3, 50 unrolled iterations",
        "value": 1e3 * t_both, "unit": "ms", "n_gpus": 1, "steps": reps, "warmup": 1,
        "ms_per_step": 1e3 * t_both, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "diff-128: 128^3, 1000 Gaussian blobs on 4 chains, SNR 0.5, 50 SPG iterations, "
                               "checkpoint every 10, loss |x_50 - x_true|^2"},
        "plain_forward_ms": 1e3 * t_plain,
        "forward_plus_reverse_over_plain_forward": t_both / t_plain,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
