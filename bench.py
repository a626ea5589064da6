"""Benchmark of the pFFT loop-analysis hot path on one MI355X.

Workload (default): the package-trace configuration -- 32 seeded Manhattan
meander traces (20 x 15 um section, 3-8 turns, 2-6 mm long) on a 5 x 5 mm
area, 200,196 triangles, 32 ports x 16 log-spaced frequencies 0.1-10 GHz =
512 right-hand sides, FP32 complex grid convolution on a 256 x 256 x 32 grid,
FP64 near field.

One step = one application of the preconditioned loop operator P^-1 Z_l to
all 512 right-hand sides (tree scan A^T, projection, three-axis FFT
convolution, interpolation, near-field + Gram combine, tree scan A,
preconditioner), inputs resident on the device.  value = right-hand-side
matvecs per second.  After the steps: per-stage HIP-event times, the
roofline of the dominant kernel, the branch-space product against exact
dense-kernel rows of the oracle (sampled edges), the bond-wire array (39,936
triangles, 80 RHS) as a second measured workload, the sweep solve (all ports
x frequencies to a 1e-6 true relative residual, plain and learned
preconditioner) and the oracle's stored-kernel matvec timed on the host.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
# MI355X vector FP32: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz = 78.6
# TFLOP/s per instruction stream; packed FP32 doubles it to the published
# 157.3 TFLOP/s (the library's kernels are compiled without packed FP32)
FP32_PEAK_TFLOPS = 157.3
FP32_NOPACK_TFLOPS = 78.6


def traces_workload():
    import workloads as W
    s = W.config3_traces()
    freqs = np.logspace(8, 10, 16)
    return s, freqs, (256, 256, 32)


def wires_workload():
    import workloads as W
    s = W.config2_wires()
    freqs = 10.0 ** (6 + 4 * np.arange(10) / 9.0)
    return s, freqs, (256, 64, 32)


WORKLOADS = {
    "traces": (traces_workload, "package traces: 32 meander traces, 200,196 triangles, 32 ports x 16 freqs "
                                "(0.1-10 GHz) = 512 RHS, grid 256x256x32, O_s=4, kappa=1.5"),
    "wires": (wires_workload, "bond-wire array: 8 wires, 39,936 triangles, 8 ports x 10 freqs = 80 RHS, "
                              "grid 256x64x32, O_s=4, kappa=1.5"),
}


def stage_bytes(sz, R, vbytes=8):
    """Algorithmic HBM bytes of one launch of each stage for R right-hand
    sides (each input and output touched once; matrix data read once).  The
    fused plane kernel ("fft_y") reads and writes the 2 N_g points of each
    channel's x-transformed grid once."""
    N, n, b, l, nn = sz["Ng"], sz["n"], sz["b"], sz["l"], sz["nprime"]
    ch = 3 * R
    return {
        "loop_to_branch": R * (16 * l + 16 * b + 32 * (nn + 1)),
        "tri_current": R * (16 * b + 4 * vbytes * n) + 12 * n,
        "project": ch * N * vbytes + R * 4 * vbytes * n + 64 * n * (4 + 4 * (vbytes // 2)),
        "fft_x": ch * N * vbytes * 3,          # read N, write 2N
        "fft_y": ch * N * vbytes * 4,          # fused plane: read 2N, write 2N
        "ifft_x": ch * N * vbytes * 3,         # read 2N, write N
        "interp": ch * N * vbytes + R * 64 * n + 64 * n * 4 * (vbytes // 2),
        "combine": R * (16 * b * 2 + 64 * n) + 12 * sz["nnz_near"] + 60 * b,
        "branch_to_loop": R * (16 * b + 16 * l + 32 * nn),
    }


def _fft(n):
    """5 N log2 N flops of an N-point complex FFT."""
    return 5 * n * int(np.log2(n)) if n > 1 else 0


def yz_plane_flops(ny, nz):
    """FFT flops of the register plane kernel (planes up to 64 x 32) for one
    (channel, k_x) plane: the z and y transforms of both zero-padding halves,
    their split twiddles, the real spectrum product and the half sums."""
    ly, lz = int(np.log2(ny)), int(np.log2(nz))
    z_fwd = ny * (2 * 5 * nz * lz + 6 * nz)
    y_fwd = 2 * nz * (2 * 5 * ny * ly + 6 * ny)
    mult = 2 * ny * 2 * nz * 2
    y_inv = 2 * nz * (2 * 5 * ny * ly + 6 * ny + 2 * ny)
    z_inv = ny * (2 * 5 * nz * lz + 6 * nz + 2 * nz)
    return z_fwd + y_fwd + mult + y_inv + z_inv


def big_plane_flops(ny, nz):
    """Flops of the big-plane kernel (256 x 32, 512 x 16 planes) for one
    (channel, k_x) plane, per y half e_y: the forward and inverse N_y-point y
    transforms of the N_z columns (four-step: 5 N log2 N plus 6 flops per
    cross twiddle), the modulation and demodulation of the odd half, and per
    row both z halves (forward and inverse N_z-point transforms, the odd
    half's twiddles, the real spectrum product, the half sum); then the sum
    of the two y halves and the scale."""
    tot = 0
    for ey in (0, 1):
        y = nz * (2 * (_fft(ny) + 6 * ny) + (2 * 6 * ny if ey else 0))
        z = ny * (2 * 2 * _fft(nz) + 2 * 6 * nz + 2 * 2 * nz + 2 * nz)
        tot += y + z
    return tot + 4 * ny * nz


def traffic_table(table):
    """A committed counter table (profiles/<table>.json: rocprofv3
    FETCH_SIZE and WRITE_SIZE per kernel, each scaled by a 1 GiB copy), or
    None when it is absent or the kernel sources changed since the counters
    were taken."""
    import hashlib
    path = os.path.join(HERE, "profiles", table + ".json")
    try:
        tab = json.load(open(path))
    except (OSError, ValueError):
        return None
    for rel, sha in tab.get("sources_sha256", {}).items():
        try:
            if hashlib.sha256(open(os.path.join(HERE, rel), "rb").read()).hexdigest() != sha:
                return None
        except OSError:
            return None
    return tab


def measured_traffic(stage, table):
    """HBM bytes per launch of a stage from the counter table, or None."""
    tab = traffic_table(table)
    ent = None if tab is None else tab.get("stages", {}).get(stage)
    return None if ent is None else int(ent["read_bytes"] + ent["write_bytes"])


def measured_step_bytes(table):
    """HBM bytes of one whole step (every kernel of the product) from the
    counter table, or None."""
    tab = traffic_table(table)
    if tab is None or "step_read_bytes" not in tab:
        return None
    return int(tab["step_read_bytes"] + tab["step_write_bytes"])


def exact_rows_check(ctx, structure, nrow=24, nrhs=4, seed=0):
    """The branch-space product K alpha on the GPU against exact dense-kernel
    rows of the oracle (both surfaces integrated numerically) at nrow sampled
    edges, for nrhs seeded right-hand sides: relative 2-norm error over the
    sampled entries and the largest entry error relative to the largest
    entry.  Returns (dict, rows, alpha, seconds spent on the rows)."""
    import torch
    import workloads as W
    from oracle.mesh import RWGMesh
    from oracle import integrals as I
    m = RWGMesh(structure.V, structure.T)
    rows = np.sort(np.random.default_rng(seed).choice(m.nedge, nrow, replace=False))
    t0 = time.perf_counter()
    Krows = I.kernel_rows(m, rows)
    t_rows = time.perf_counter() - t0
    X = W.complex_normal(seed + 1, (nrhs, m.nedge))
    y = ctx.matvec(torch.from_numpy(X).cuda(), space=0).cpu().numpy()[:, rows]
    ref = X @ Krows.T
    return ({"rows": int(nrow), "rhs": int(nrhs),
             "rel_err_2norm": float(np.linalg.norm(y - ref) / np.linalg.norm(ref)),
             "max_abs_err_rel_to_max": float(np.abs(y - ref).max() / np.abs(ref).max())},
            Krows, X, t_rows)


def cpu_oracle_baseline(Krows, X, nrhs_full, b, t_rows):
    """The oracle's matvec with a stored dense kernel (numpy BLAS on the host
    cores): a block of stored rows (the exact sampled rows repeated to 512)
    times the right-hand sides as a real matrix times complex columns, timed
    and scaled to the b rows of one full product of nrhs_full right-hand
    sides.  Extrapolated: the full K (b x b doubles) does not fit in memory."""
    reps = max(1, 512 // Krows.shape[0])
    Kb = np.ascontiguousarray(np.tile(Krows, (reps, 1)))
    Xr = np.ascontiguousarray(np.tile(X.T, (1, max(1, nrhs_full // X.shape[0])))[:, :nrhs_full])
    Xre, Xim = np.ascontiguousarray(Xr.real), np.ascontiguousarray(Xr.imag)
    _ = Kb[:8] @ Xre[:, :8]
    # repeated until about 10 s of host work has been timed (3 passes at least)
    t0 = time.perf_counter()
    reps_done = 0
    while reps_done < 3 or time.perf_counter() - t0 < 10.0:
        _ = Kb @ Xre
        _ = Kb @ Xim
        reps_done += 1
    total = time.perf_counter() - t0
    dt = total / reps_done
    per_row = dt / Kb.shape[0]
    full = per_row * b
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": nrhs_full / full, "unit": "RHS-matvecs/s", "cores": threads, "kind": "oracle",
            "sample": "stored-kernel K.alpha: %d stored rows (%d exact oracle rows, repeated) x %d right-hand "
                      "sides with numpy BLAS, %d passes in %.1f s (%.3f s each), scaled to the %d rows of a "
                      "full product (extrapolated; exact rows took %.1f s to integrate)"
                      % (Kb.shape[0], Krows.shape[0], nrhs_full, reps_done, total, dt, b, t_rows)}


def roofline(stages, sz, R, grid):
    """Roofline of the dominant kernel (largest share of the step)."""
    nbytes = stage_bytes(sz, R)
    dom = max((k for k in stages if stages[k][1] > 0), key=lambda k: stages[k][0])
    ms, calls = stages[dom]
    avg_s = ms / 1e3 / calls
    gx, gy, gz = grid
    big = (gy, gz) in ((256, 32), (512, 16))
    reg = (gy, gz) in ((64, 32), (32, 16), (16, 8))
    if dom == "fft_y" and (big or reg):
        # the fused plane kernels issue vector ALU work at their limit (packed
        # FP32 is not used): FFT flops against the FP32 vector peak, with the
        # HBM figure beside
        per_plane = big_plane_flops(gy, gz) if big else yz_plane_flops(gy, gz)
        flops = 3 * R * 2 * gx * per_plane
        achieved = flops / avg_s / 1e12
        return {"kernel": "k_fft_yz_big" if big else "k_fft_yz_reg", "stage": dom, "bound": "alu",
                "achieved": round(achieved, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_PEAK_TFLOPS, 4), "avg_launch_ms": round(ms / calls, 4),
                "flops_per_launch": int(flops), "peak_without_packed_fp32": FP32_NOPACK_TFLOPS,
                "frac_without_packed_fp32": round(achieved / FP32_NOPACK_TFLOPS, 4),
                "hbm_GBs": round(nbytes[dom] / avg_s / 1e9, 1), "bytes_per_launch": int(nbytes[dom])}
    if dom in nbytes:
        achieved = nbytes[dom] / avg_s / 1e9
        return {"stage": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "avg_launch_ms": round(ms / calls, 4),
                "bytes_per_launch": int(nbytes[dom])}
    return {"stage": dom, "bound": "latency", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": None, "avg_launch_ms": round(ms / calls, 4)}


def run_steps(ctx, R, omega, steps, warmup, flags):
    import torch
    sz = ctx.sizes
    rng = np.random.default_rng(0)
    x = torch.from_numpy(rng.standard_normal((R, sz["l"])) + 1j * rng.standard_normal((R, sz["l"]))).cuda()
    y = torch.empty_like(x)
    for _ in range(warmup):
        ctx.matvec(x, omega, space=1, flags=flags, out=y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.matvec(x, omega, space=1, flags=flags, out=y)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # per-stage HIP-event timing on the library's stream
    psteps = max(1, min(steps, 3))
    ctx.profile(True)
    for _ in range(psteps):
        ctx.matvec(x, omega, space=1, flags=flags, out=y)
    torch.cuda.synchronize()
    stages = ctx.stage_times()
    ctx.profile(False)
    del x, y
    return dt, stages, psteps


def protocol_layout(seed):
    """A layout of the package-trace generator for the learned-correction
    protocol: 32 meander traces on 5 x 5 mm, triangle count drawn (seeded)
    from 20k-100k, grid 128 x 128 x 16 (39 um cells, about the mesh step of
    a 100k-triangle layout; the package-trace configuration's 256 x 256 x 32
    grid matches its 200k triangles)."""
    import workloads as W
    target = int(np.random.default_rng(7919 + seed).integers(20_000, 100_001))
    s = W.traces(seed=seed, target_tris=target, name="traces_s%d" % seed)
    return s, (128, 128, 16)


def learned_protocol(train_seeds, eval_seeds, freqs_eval=(1e8, 4.6e8, 2.2e9, 1e10), steps_per_layout=300,
                     log=None):
    """Train the correction network over seeded layouts (weights carried from
    one layout's context to the next), then compare plain and learned FGMRES
    sweeps (all ports x freqs_eval, 1e-6 true relative residual) on unseen
    layouts, the learned sweep with the convergence judge measured on the
    last training layout.  Returns a dict with per-layout records and the
    medians."""
    import torch
    import paper_2210_04891_amd as P
    fe = np.asarray(freqs_eval, np.float64)
    f_train = np.sqrt(fe[:-1] * fe[1:])
    blob, judge, rows_total, t_train = None, 0, 0, 0.0
    for k, sd in enumerate(train_seeds):
        s, grid = protocol_layout(sd)
        ctx = P.Context(s, grid, stencil=4, near_kappa=1.5, grid_fp64=False)
        t0 = time.perf_counter()
        if blob is not None:
            ctx.precond_load(blob)
        rows = ctx.learned_collect(f_train, tol=1e-8, maxit=40)
        ctx.learned_train(steps_per_layout, batch=8192, hidden=256, lr=1e-3, seed=sd)
        blob = ctx.precond_save()
        judge = ctx.get_option("learned_judge_ppm")   # plain per-step factor x 1.1, from this collection
        torch.cuda.synchronize()
        t_train += time.perf_counter() - t0
        rows_total += rows
        if log:
            log("protocol: train layout %d (seed %d, %d triangles): %d rows, loss %.4f"
                % (k, sd, ctx.sizes["n"], rows, ctx.learned_eval()))
        ctx.close()
    recs = []
    for sd in eval_seeds:
        s, grid = protocol_layout(sd)
        ctx = P.Context(s, grid, stencil=4, near_kappa=1.5, grid_fp64=False)
        p = len(s.ports)
        om = np.repeat(2 * np.pi * fe, p)
        # factor P and size the workspaces before either timed sweep
        ctx.matvec(torch.zeros((om.size, ctx.sizes["l"]), dtype=torch.complex128, device="cuda"),
                   omega=om, space=1, flags=P.PFFT_PRECOND)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Y1, it1, rr1, c1 = ctx.solve_ports(fe, tol=1e-6, maxit=600, restart=60, precond=1)
        t1 = time.perf_counter()
        ctx.precond_load(blob)
        ctx.set_option("learned_judge_ppm", judge)
        Y2, it2, rr2, c2 = ctx.solve_ports(fe, tol=1e-6, maxit=600, restart=60, precond=2)
        t2 = time.perf_counter()
        n_apply, n_fall, n_off = ctx.learned_stats()
        rec = {"seed": int(sd), "triangles": int(ctx.sizes["n"]), "rhs": int(om.size),
               "plain_s": round(t1 - t0, 3), "learned_s": round(t2 - t1, 3),
               "plain_iters_median": float(np.median(it1)), "learned_iters_median": float(np.median(it2)),
               "plain_status": int(c1), "learned_status": int(c2),
               "learned_max_relres": float(rr2.max()), "learned_rhs_switched_to_plain": int(n_off),
               "Y_rel_diff": float(np.abs(Y2 - Y1).max() / np.abs(Y1).max())}
        recs.append(rec)
        if log:
            log("protocol: eval seed %d: %s" % (sd, json.dumps(rec)))
        ctx.close()
    med = lambda key: float(np.median([r[key] for r in recs]))
    return {"train_layouts": len(train_seeds), "train_rows": int(rows_total), "train_s": round(t_train, 1),
            "judge_factor": judge * 1e-6,
            "eval_layouts": len(eval_seeds), "median_plain_s": med("plain_s"),
            "median_learned_s": med("learned_s"), "median_plain_iters": med("plain_iters_median"),
            "median_learned_iters": med("learned_iters_median"), "layouts": recs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="traces")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-correction sweep arm")
    ap.add_argument("--no-second", action="store_true", help="skip the second (bond-wire) workload")
    ap.add_argument("--no-check", action="store_true", help="skip the exact-row check and the CPU baseline")
    ap.add_argument("--learned-protocol", default="",
                    help="TRAIN,EVAL: train the correction network on TRAIN seeded trace layouts (seeds 0..) and "
                         "compare plain and learned sweeps on EVAL unseen ones (seeds 10000..); prints its own "
                         "JSON line and exits")
    ap.add_argument("--plan", action="append", default=[], metavar="NAME=VALUE",
                    help="set a plan option instead of running the autotuner (repeatable; e.g. for profiler runs "
                         "that should not include the autotuner's trial products)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="before the steps, copy a buffer of this size three times (device to device) so that "
                         "hardware byte counters can be scaled against a transfer of known size")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs the whole hot path on a single "
              "MI355X (sharding over right-hand sides is described, not built); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2210_04891_amd as P

    if args.learned_protocol:
        ntr, nev = (int(x) for x in args.learned_protocol.split(","))
        res = learned_protocol(list(range(ntr)), list(range(10_000, 10_000 + nev)),
                               log=lambda m: print(m, file=sys.stderr, flush=True))
        print(json.dumps({"learned_protocol": res}), flush=True)
        return
    make, label = WORKLOADS[args.workload]
    s, freqs, grid = make()
    p = len(s.ports)
    R = p * len(freqs)
    t_setup = time.perf_counter()
    ctx = P.Context(s, grid, stencil=4, near_kappa=1.5, grid_fp64=False)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    print("bench: setup %.1f s" % t_setup, file=sys.stderr, flush=True)
    sz = ctx.sizes
    omega = np.repeat(2 * np.pi * freqs, p)
    if args.copy_probe_mb > 0:
        a = torch.ones(args.copy_probe_mb * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    # the autotuner picks each plan (FFT passes, band solve, projection tile
    # shape, near-field kernel, stream split) on this workload's product
    t_tune = time.perf_counter()
    if args.plan:
        for kv in args.plan:
            name, val = kv.split("=")
            ctx.set_option(name, int(val))
        tune = {name: {"chosen": ctx.get_option(name)} for name in (kv.split("=")[0] for kv in args.plan)}
    else:
        tune = ctx.autotune(omega, reps=3)
    t_tune = time.perf_counter() - t_tune
    print("bench: plans (%.1f s): %s" % (t_tune, {k: v["chosen"] for k, v in tune.items()}), file=sys.stderr,
          flush=True)
    dt, stages, psteps = run_steps(ctx, R, omega, args.steps, args.warmup, P.PFFT_PRECOND)
    value = R * args.steps / dt
    print("bench: %d steps, %.1f ms/step" % (args.steps, dt / args.steps * 1e3), file=sys.stderr, flush=True)
    roof = roofline(stages, sz, R, grid)
    table = {"traces": "package_traces512_traffic", "wires": "bond_wires80_traffic"}[args.workload]
    roof["traffic"] = measured_traffic(roof["stage"], table)
    out = {
        "metric": "pFFT matvecs/s (% HBM peak); sweep solve time learned vs plain @1e-6 resid",
        "value": round(value, 2),
        "unit": "RHS-matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32 grid / fp64 near field, scans, preconditioner",
        "data": "synthetic",
        "config": {"workload": label, "triangles": sz["n"], "loops": sz["l"], "rhs": R, "grid": list(grid),
                   "near_nnz": sz["nnz_near"], "setup_s": round(t_setup, 2),
                   "setup_phases_ms": dict(zip(("topology", "circuit", "gram", "grid", "near_lists",
                                                "near_pair_blocks_device", "near_csr", "device_build"),
                                               np.round(ctx.model_array("setup_ms", np.float64), 1).tolist())),
                   "plans": {k: v["chosen"] for k, v in tune.items()}, "autotune_s": round(t_tune, 2)},
        "roofline": roof,
        "stages_ms_per_step": {k: round(v[0] / psteps, 4) for k, v in stages.items() if v[1]},
        "stage_sum_ms": round(sum(v[0] for v in stages.values()) / psteps, 3),
        "device": {"name": torch.cuda.get_device_name(0),
                   "lds_per_block": getattr(torch.cuda.get_device_properties(0), "shared_memory_per_block", None)},
    }
    # whole-product model bytes per step (the algorithmic bytes of every
    # stage) over the step time, against the HBM peak
    model = sum(stage_bytes(sz, R).values())
    out["model_bytes_per_step"] = int(model)
    out["model_GBs_frac"] = round(model / (dt / args.steps) / 1e9 / HBM_PEAK_GBS, 4)
    # the same ratio with the bytes the HBM counters saw over a whole step
    sb = measured_step_bytes(table)
    out["counter_bytes_per_step"] = sb
    out["counter_GBs_frac"] = None if sb is None else round(sb / (dt / args.steps) / 1e9 / HBM_PEAK_GBS, 4)
    Krows = X = None
    t_rows = 0.0
    if not args.no_check:
        chk, Krows, X, t_rows = exact_rows_check(ctx, s)
        out["matvec_vs_oracle"] = chk
    if not args.no_sweep:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        Y, it, rr, code = ctx.solve_ports(freqs, tol=1e-6, maxit=400, restart=60, precond=1)
        t_sweep = time.perf_counter() - t1
        out["sweep"] = {"rhs": R, "plain_s": round(t_sweep, 3), "status": int(code), "iters_max": int(it.max()),
                        "iters_mean": round(float(it.mean()), 2), "max_relres": float(rr.max()), "learned_s": None}
        if not args.no_learned:
            # learned correction: pairs from plain solves at frequencies between
            # the sweep's, device training, then the same sweep
            f_train = np.sqrt(freqs[:-1] * freqs[1:])[::2]
            t3 = time.perf_counter()
            rows = ctx.learned_collect(f_train, tol=1e-8, maxit=40)
            t_collect = time.perf_counter() - t3
            t4 = time.perf_counter()
            ctx.learned_train(600, batch=8192, hidden=256, lr=1e-3, seed=0)
            ctx.learned_clear()      # the training set (tens of GB here) is not needed by the sweep
            torch.cuda.synchronize()
            t_train = time.perf_counter() - t4
            t5 = time.perf_counter()
            Y2, it2, rr2, code2 = ctx.solve_ports(freqs, tol=1e-6, maxit=400, restart=60, precond=2)
            t_learned = time.perf_counter() - t5
            n_apply, n_fall, n_off = ctx.learned_stats()
            out["sweep"].update({"learned_s": round(t_learned, 3), "learned_status": int(code2),
                                 "learned_iters_mean": round(float(it2.mean()), 2),
                                 "learned_iters_max": int(it2.max()),
                                 "learned_rhs_switched_to_plain": n_off, "learned_rhs_applications": n_apply,
                                 "learned_collect_s": round(t_collect, 2), "learned_train_s": round(t_train, 2),
                                 "learned_training_rows": int(rows)})
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    if not args.no_second and args.workload == "traces":
        # the bond-wire array, same step definition, as a second workload
        s2, f2, g2 = wires_workload()
        ctx2 = P.Context(s2, g2, stencil=4, near_kappa=1.5, grid_fp64=False)
        R2 = len(s2.ports) * len(f2)
        om2 = np.repeat(2 * np.pi * f2, len(s2.ports))
        tune2 = ctx2.autotune(om2, reps=3)
        dt2, st2, ps2 = run_steps(ctx2, R2, om2, 20, 3, P.PFFT_PRECOND)
        out["second_workload"] = {"workload": WORKLOADS["wires"][1], "value": round(R2 * 20 / dt2, 2),
                                  "unit": "RHS-matvecs/s", "ms_per_step": round(dt2 / 20 * 1e3, 3),
                                  "plans": {k: v["chosen"] for k, v in tune2.items()},
                                  "stages_ms_per_step": {k: round(v[0] / ps2, 4) for k, v in st2.items() if v[1]}}
        ctx2.close()
    if not args.no_cpu_baseline and Krows is not None:
        out["cpu_baseline"] = cpu_oracle_baseline(Krows, X, R, sz["b"], t_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
