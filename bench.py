"""Benchmark: time per density matrix D and effective TFLOP/s on one MI355X.

Workload (default): 1024 water-like molecules (23,552 basis functions, 6 A
cutoff, one submatrix per molecule, n_g ~ 600-1060), synthetic and seeded.
A step is one full evaluation of the hot path with K already resident in
HBM: gather + shift + Gershgorin bound, batched Newton-Schulz to
max|X^2 - I| <= 1e-12, scatter of D, and the N / E reductions.

Effective TFLOP/s = sum_g 4 n_g^3 k_g / time per D, with k_g the Newton-Schulz
steps the FP64 path takes (two dense products per step); the same numerator
is used for every precision mode.

Prints one JSON line (see the "roofline" and "cpu_baseline" objects).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time per density matrix D + effective TFLOP/s at max|dD|<=1e-6 vs FP64 GPU"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2516.6}

WORKLOADS = {
    "water1024": "1024 water-like molecules (23552 basis functions, O 13 / H 5 per atom), "
                 "periodic 31.3 A box, 6 A cutoff, one submatrix per molecule",
    "water256": "256 water-like molecules (5888 basis functions), periodic 19.7 A box, 6 A cutoff, "
                "one submatrix per molecule",
    "water16": "16 water-like molecules (368 basis functions), periodic 7.8 A box, 4 A cutoff, "
               "one submatrix per molecule",
    "water6912": "6912 water-like molecules (158976 basis functions), periodic 59.6 A box, 7 A cutoff, "
                 "one submatrix per molecule, processed in memory-bounded waves",
}


def progress(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(system, gpu_d, stats_iters, n_g, nthreads, n_sample, seed=2024, kT=0.0):
    """Time the CPU oracle on a seeded sample of groups and compare with the GPU D there."""
    import oracle
    rng = np.random.default_rng(seed)
    pick = np.sort(rng.choice(system.ngroups, size=min(n_sample, system.ngroups), replace=False))
    t0 = time.perf_counter()
    ref = oracle.submatrix(system, which=pick, nthreads=nthreads, kT=kT)
    dt = time.perf_counter() - t0
    ok = ~np.isnan(ref.d_values)
    err = float(np.abs(gpu_d[ok] - ref.d_values[ok]).max())
    n3k = 4.0 * n_g.astype(np.float64) ** 3 * stats_iters
    frac = float(n3k[pick].sum() / n3k.sum())
    t_full = dt / frac
    return {
        "value": float(n3k[pick].sum() / dt / 1e12),
        "unit": "TFLOP/s",
        "cores": int(nthreads),
        "kind": "oracle",
        "sample": f"{len(pick)} of {system.ngroups} submatrices (seeded), cyclic Jacobi FP64, "
                  f"{nthreads} threads, {dt:.1f} s wall; time per D extrapolated by sum 4 n_g^3 k_g",
        "seconds_sample": dt,
        "time_per_D_s_extrapolated": t_full,
    }, err, pick


def full_sign_report(system, d_values, n_gpu, e_gpu):
    """Error of the submatrix D against the exact D of the whole K (dense
    symmetric eigendecomposition, numpy/LAPACK), at K's stored blocks.  The
    submatrix method is an approximation (Sec. III-A); this is reported, not
    gated."""
    t0 = time.perf_counter()
    kd = system.to_dense()
    kd -= system.mu * np.eye(system.n)
    lam, q = np.linalg.eigh(kd)
    occ = lam < 0
    d_exact = (q[:, occ] @ q[:, occ].T)
    boff = np.concatenate([[0], np.cumsum(system.blk_size)])
    voff = system.val_off()
    err = 0.0
    for j in range(system.nblk):
        for p in range(int(system.col_ptr[j]), int(system.col_ptr[j + 1])):
            i = int(system.row_idx[p])
            blk = d_exact[boff[i]:boff[i + 1], boff[j]:boff[j + 1]].T.reshape(-1)
            err = max(err, float(np.abs(d_values[voff[p]:voff[p + 1]] - blk).max()))
    n_exact = float(occ.sum())
    e_exact = float((lam[occ] + system.mu).sum())
    return {"max_abs_dD": err, "N_exact": n_exact, "dN": n_gpu - n_exact, "E_exact": e_exact, "dE": e_gpu - e_exact,
            "method": "numpy.linalg.eigh of the dense K - mu I", "seconds": time.perf_counter() - t0}


def literal_bf16_report(smx, stream_handle, reps=20):
    """The paper's plain-BF16 mode on water16 (one BF16 word per value, FP32
    accumulation, then the FP64 own-column polish): device time per D against
    the FP64 path, and its D against the FP64 GPU D.  Returns (report, D)."""
    from waterbox import water_config
    s = water_config("water16")
    out, dvals = {"workload": "water16: " + WORKLOADS["water16"]}, {}
    for prec in ("fp64", "bf16"):
        ctx = smx.Context(0, stream=stream_handle).load(s).configure(precision=prec)
        ms = []
        for _ in range(reps + 3):
            res = ctx.evaluate(allow_not_converged=True)
            ms.append(ctx.stats()["time_total_ms"])
        dvals[prec] = res
        out[f"{prec}_ms_per_D"] = float(np.median(ms[3:]))
        out[f"{prec}_status"] = int(res.status)
        ctx.close()
    out["speedup_over_fp64"] = out["fp64_ms_per_D"] / out["bf16_ms_per_D"]
    out["max_abs_dD_vs_fp64_gpu"] = float(np.abs(dvals["bf16"].d_values - dvals["fp64"].d_values).max())
    out["dN_vs_fp64_gpu"] = dvals["bf16"].n_elec - dvals["fp64"].n_elec
    return out, s, dvals["bf16"]


def kernel_name(kind, precision):
    """Product kernel of a launch kind (smx_get_launch_profile)."""
    if kind in (0, 1, 4, 5, 6, 11):
        return "ns_f64_kernel"
    if kind in (7, 8, 10):
        return "ns_words256_kernel"
    if kind == 12:
        return "tridiag_kernel"
    return "ns_f32_kernel" if precision == "fp32" else "ns_words_kernel"


def run_path(smx, ctx, precision, steps, warmup, d_out, graph_steps=0):
    """Warm up, then time exactly `steps` evaluations; returns timings and stats.

    With graph_steps > 0 the step launches are replayed from HIP graphs, which
    record no per-launch events; the per-launch profile then comes from one
    direct evaluation after the timed region."""
    import torch
    ctx.configure(precision=precision, graph_steps=graph_steps)

    def step():
        smx.smx_evaluate(ctx.handle)
        smx.smx_wait(ctx.handle)

    def record(prof):
        # per kernel: [device ms, algorithmic flops, launches, issued matrix-core flops]
        ms, fl, kd = ctx.launch_profile()
        iss = smx.smx_get_launch_issued(ctx.handle)
        for m, f, k, q in zip(ms, fl, kd, iss):
            e = prof.setdefault(kernel_name(k, precision), [0.0, 0.0, 0, 0.0])
            e[0] += m
            e[1] += f
            e[2] += 1
            e[3] += q

    for w in range(warmup):
        step()
        progress(f"{precision}: warm-up step {w + 1}/{warmup} done")
    torch.cuda.synchronize()
    prof = {}
    dev_ms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        record(prof)
        dev_ms.append(ctx.stats()["time_total_ms"])
        if dev_ms[-1] > 2000:
            progress(f"{precision}: timed step {len(dev_ms)}/{steps} done ({dev_ms[-1]:.0f} ms)")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stats = ctx.stats()
    info = ctx.group_info()
    smx.smx_get_d(ctx.handle, d_out)
    if graph_steps:
        ctx.configure(precision=precision, graph_steps=0)
        step()
        record(prof)
    return dict(ms_per_step=wall / steps * 1e3, dev_ms=dev_ms, prof=prof, stats=stats, info=info,
                n_elec=smx.smx_trace(ctx.handle), energy=smx.smx_energy(ctx.handle))


DTYPES = {"fp64": "f64", "fp16x2": "f16x2 words, f32 accumulation; f64 polish",
          "bf16x3": "bf16x3 words, f32 accumulation; f64 polish",
          "bf16": "bf16 words, f32 accumulation; f64 polish",
          "fp32": "f32, f32 accumulation; f64 polish"}
PEAK_BY_KERNEL = {"ns_f64_kernel": ("fp64", 78.6), "ns_words_kernel": ("fp16/bf16", 2516.6),
                  "ns_words256_kernel": ("fp16/bf16", 2516.6), "ns_f32_kernel": ("fp32", 157.3),
                  "tridiag_kernel": ("HBM", 8000.0)}

# HBM bytes per launch of the dominant kernel on water1024, from two rocprofv3
# counter runs (FETCH_SIZE, WRITE_SIZE) scaled by a plain-copy calibration; the
# figure is valid only while the kernel's sources hash to the recorded value.
# The same runs give the matrix-core busy fraction (SQ_VALU_MFMA_BUSY_CYCLES
# over 1024 SIMDs x 2.4 GHz x kernel time).
TRAFFIC = {
    ("water1024", "ns_words_kernel"): (8.164e9, ("smx_ns_words.hip", "smx_internal.h"), "9cfd87bdfd482aeb",
                                       "profiles/ns_words_kernel_water1024_fp16x2.md", 0.300),
    ("water1024", "ns_f64_kernel"): (19.29e9, ("smx_ns_f64.hip", "smx_internal.h"), "7739624ee052bcd3",
                                     "profiles/ns_f64_kernel_water1024_fp64.md", 0.684),
}


def measured_traffic(workload, kernel):
    """Counter-measured (HBM bytes per launch, source, MFMA busy fraction), or Nones if
    absent or the kernel changed since the counters were taken."""
    import hashlib
    ent = TRAFFIC.get((workload, kernel))
    if ent is None:
        return None, None, None
    nbytes, files, digest, src, busy = ent
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2004_10811_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return (nbytes, src, busy) if h.hexdigest()[:16] == digest else (None, None, None)


def d_asymmetry(system, d_values):
    """max |D_IJ - D_JI^T| over the stored blocks (D is not symmetrised)."""
    bs = system.blk_size.astype(np.int64)
    cols = np.repeat(np.arange(system.nblk), np.diff(system.col_ptr))
    rows = system.row_idx.astype(np.int64)
    voff = system.val_off()
    key = rows * system.nblk + cols
    order = np.argsort(key)
    mirror = order[np.searchsorted(key[order], cols * system.nblk + rows)]
    worst = 0.0
    for bi in np.unique(bs):
        for bj in np.unique(bs):
            sel = np.nonzero((bs[rows] == bi) & (bs[cols] == bj))[0]
            if sel.size == 0:
                continue
            a = d_values[voff[sel][:, None] + np.arange(bi * bj)[None, :]].reshape(-1, bj, bi)
            m = d_values[voff[mirror[sel]][:, None] + np.arange(bi * bj)[None, :]].reshape(-1, bi, bj)
            worst = max(worst, float(np.abs(a - m.transpose(0, 2, 1)).max()))
    return worst


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="water1024", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp16x2", choices=sorted(DTYPES))
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="groups in the CPU oracle sample (default: two per thread, about 15 s on 16 host threads "
                         "for water1024)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--full-sign", action="store_true",
                    help="also report the error against the exact sign of the whole K (dense eigendecomposition; "
                         "done by default up to 8000 basis functions)")
    ap.add_argument("--backward", action="store_true",
                    help="also time the adjoint (dE/dK through the frozen map of the timed evaluation)")
    ap.add_argument("--kernel-variant", type=int, default=0, choices=[0, 1, 2],
                    help="operand stream of the word products (0: global_load_lds per K step, 1: register prefetch, 2: persistent launch over per-XCD work lists)")
    ap.add_argument("--kT", type=float, default=0.0,
                    help="electronic temperature in Hartree; kT > 0 times the diagonalisation path (Fermi D, FP64)")
    ap.add_argument("--iteration", default="ns2", choices=["ns2", "pade3"],
                    help="sign iteration of the timed path: second-order Newton-Schulz (two products per step) or "
                         "third-order Pade (three products per step); the FP64 reference that fixes the flop "
                         "numerator is always Newton-Schulz")
    ap.add_argument("--tile-shape", type=int, default=None, metavar="NPAD",
                    help="size bucket boundary of the word products: groups with n_pad >= NPAD on 256 x 256 "
                         "tiles (0: 128 x 128 only; default: the library's)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the timed precision in the given launch configuration instead of the autotuner's "
                         "choice (launch order x step graphs x size bucket boundary)")
    ap.add_argument("--graph-steps", type=int, default=0,
                    help="replay the Newton-Schulz steps from HIP graphs of this many steps (0: direct launches)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (to scale "
                         "the FETCH_SIZE / WRITE_SIZE counters of a profiler run) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.rand(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": n * 8, "launches": 3}), flush=True)
        return

    if args.kT > 0 and args.precision != "fp64":
        ap.error("--kT > 0 runs the diagonalisation path, which is FP64 (use --precision fp64)")
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the submatrix groups are independent and would shard by contiguous group chunks, "
              "but no multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2004_10811_amd as smx
    from waterbox import water_config

    system = water_config(args.workload)
    progress(f"{args.workload}: {system.n} basis functions, {system.ngroups} submatrices generated")
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = smx.Context(0, stream=stream.cuda_stream).load(system)
    smx.smx_set_kernel_variant(ctx.handle, args.kernel_variant)
    if args.tile_shape is not None:
        smx.smx_set_tile_shape(ctx.handle, args.tile_shape)
    d64 = torch.empty(ctx.nvalues, dtype=torch.float64, device="cuda")
    d_mix = torch.empty_like(d64)

    graph_steps = args.graph_steps
    tuned = None

    def autotune():
        # the autotuner times whole evaluations of every candidate launch
        # configuration (launch order x step graphs x size bucket boundary) for
        # the timed precision and applies the fastest
        ctx.configure(precision=args.precision, graph_steps=0, iteration=args.iteration)
        g, o, tms = smx.smx_autotune(ctx.handle, reps=2, use_cache=True)
        cfg = {"best_ms": tms, **smx.smx_get_launch_config(ctx.handle)}
        progress(f"autotune {args.precision}: {cfg}")
        return g, cfg

    # FP64 path first: the reference D and the iteration counts k_g of the
    # effective-TFLOP/s numerator (the same numerator for every precision)
    timed_ref = args.precision == "fp64" and args.iteration == "ns2" and args.kT == 0.0
    if timed_ref and not args.no_autotune:
        graph_steps, tuned = autotune()
    smx.smx_set_iteration(ctx.handle, "ns2")
    r64 = run_path(smx, ctx, "fp64", args.steps if timed_ref else 2, 1, d64, graph_steps if timed_ref else 0)
    algo = r64["stats"]["algo_flops"]
    run = r64
    d_out = d64
    if not timed_ref:
        smx.smx_set_iteration(ctx.handle, args.iteration)
        if args.kT > 0:
            smx.smx_set_temperature(ctx.handle, args.kT)
        elif not args.no_autotune:
            graph_steps, tuned = autotune()
        run = run_path(smx, ctx, args.precision, args.steps, args.warmup, d_mix, graph_steps)
        d_out = d_mix
    backward = None
    if args.backward:
        # dE/dK through the frozen map of one evaluation in the timed precision
        # (the adjoint differentiates the Newton-Schulz map)
        ctx.configure(precision=args.precision, graph_steps=0, iteration="ns2")
        smx.smx_evaluate(ctx.handle)
        smx.smx_wait(ctx.handle)
        dk = torch.empty(ctx.nvalues, dtype=torch.float64, device="cuda")
        smx.smx_backward(ctx.handle, 1.0, 0.0, None, dk)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            smx.smx_backward(ctx.handle, 1.0, 0.0, None, dk)
        torch.cuda.synchronize()
        bms = (time.perf_counter() - t0) / args.steps * 1e3
        backward = {"what": "dE/dK and dE/dmu, FP64 adjoint through the frozen map (checkpoints every 8 steps)",
                    "ms_per_backward": bms, "backward_over_forward": bms / run["ms_per_step"],
                    "max_abs_dK": float(dk.abs().max().item())}
        progress(f"backward: {bms:.1f} ms per call")
    launch_config = smx.smx_get_launch_config(ctx.handle)
    ctx.close()

    stats = run["stats"]
    ms_per_step = run["ms_per_step"]
    value = algo / (ms_per_step * 1e-3) / 1e12
    # dominant product kernel by device time
    kname, (kms, kfl, kn, kiss) = max(run["prof"].items(), key=lambda kv: kv[1][0])
    pdt, peak = PEAK_BY_KERNEL[kname]
    achieved = kfl / (kms * 1e-3) / 1e12
    bound, unit = "mfma", "TFLOP/s"
    if kname == "tridiag_kernel":
        # BLAS2-bound: each reduction step reads the trailing block at least once
        # (p = tau A22 v), 8 n^3 / 3 bytes per group = 2 bytes per counted flop (4/3 n^3)
        bound, unit = "hbm", "GB/s"
        achieved = 2.0 * kfl / (kms * 1e-3) / 1e9
    traffic, traffic_src, busy = measured_traffic(args.workload, kname)
    roofline = {
        "bound": bound,
        "achieved": achieved,
        "peak": peak,
        "unit": unit,
        "frac": achieved / peak,
        "traffic": traffic,
        "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x 2 + WRITE_SIZE x 1, copy-calibrated)",
        "traffic_source": traffic_src,
        "mfma_busy_counter": busy,
        "kernel": kname,
        "peak_dtype": pdt,
        "launches": kn,
        "avg_launch_ms": kms / max(kn, 1),
        "time_share": kms / sum(v[0] for v in run["prof"].values()),
        # issued matrix-core flops (word products, padding and half tiles included)
        # over the launch time and the same peak: the matrix-core utilisation proper
        "issued_frac": (kiss / (kms * 1e-3) / 1e12 / peak) if bound == "mfma" else None,
        "issued_per_algorithmic": kiss / kfl if kfl > 0 else None,
        "issued_mfma_tflops_all_products": (stats["exec_flops"] / (stats["time_iterate_ms"] * 1e-3) / 1e12
                                            if stats["time_iterate_ms"] > 0 else None),
    }
    diff_vs_fp64 = float((d_out - d64).abs().max().item()) if not timed_ref and args.kT == 0.0 else None

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[args.precision],
        "data": "synthetic",
        "config": {
            "workload": args.workload + ": " + WORKLOADS[args.workload],
            "precision": args.precision,
            "iteration": args.iteration,
            "kT_hartree": args.kT,
            "solver": "diagonalisation (Householder + bisection + twisted factorisations)" if args.kT > 0
                      else "matrix sign by products",
            "basis_functions": int(system.n),
            "submatrices": int(system.ngroups),
            "n_g_min_mean_max": [int(stats["n_min"]), round(stats["n_mean"], 1), int(stats["n_max"])],
            "ns_steps_min_mean_max": [int(stats["iters_min"]), round(stats["iters_mean"], 2),
                                      int(stats["iters_max"])],
            "fp64_ns_steps_mean": round(r64["stats"]["iters_mean"], 2),
            "tol": 1e-12,
            "waves": int(stats["nwaves"]),
            "graph_steps": graph_steps,
            "tile_order": launch_config["tile_order"],
            "kernel_variant": args.kernel_variant,
            "big_tile_min_npad": launch_config["big_min_npad"],
            "autotuned": tuned is not None,
        },
        "device_ms_per_D_median": float(np.median(run["dev_ms"])),
        "phase_ms": {"gather": stats["time_gather_ms"], "iterate": stats["time_iterate_ms"],
                     "scatter_reduce": stats["time_scatter_ms"]},
        "algo_flops_per_D": algo,
        "fp64_path": {"ms_per_D": r64["ms_per_step"], "tflops": algo / (r64["ms_per_step"] * 1e-3) / 1e12},
        "speedup_vs_fp64": r64["ms_per_step"] / ms_per_step,
        "max_abs_dD_vs_fp64_gpu": diff_vs_fp64,
        "N_trace_D": run["n_elec"],
        "E_band": run["energy"],
        "roofline": roofline,
    }
    if backward is not None:
        out["backward"] = backward

    d_host = d_out.cpu().numpy()
    out["max_abs_D_minus_DT"] = d_asymmetry(system, d_host)
    if args.kT > 0:
        out["vs_full_matrix_sign"] = "not computed: the exact reference is the sign (T = 0)"
    elif args.full_sign or system.n <= 8000:
        progress(f"exact sign of the whole K ({system.n} x {system.n})")
        out["vs_full_matrix_sign"] = full_sign_report(system, d_host, run["n_elec"], run["energy"])
    else:
        out["vs_full_matrix_sign"] = f"not computed: dense eigendecomposition of a {system.n} x {system.n} matrix " \
                                     "(use --full-sign)"
    if args.workload == "water1024" and args.kT == 0.0:
        progress("plain BF16 on water16")
        import torch as _t
        lit, lit_sys, lit_res = literal_bf16_report(smx, _t.cuda.current_stream().cuda_stream)
        out["literal_bf16_water16"] = lit
    if not args.no_cpu_baseline:
        nth = min(16, os.cpu_count() or 1)
        nsamp = args.cpu_sample or 2 * nth
        progress(f"CPU oracle on a sample of {nsamp} submatrices, {nth} threads")
        base, err, pick = cpu_baseline(system, d_out.cpu().numpy(), r64["info"]["iters"], r64["info"]["n"],
                                       nth, nsamp, kT=args.kT)
        out["cpu_baseline"] = base
        out["max_abs_dD_vs_oracle_on_sample"] = err
        if "literal_bf16_water16" in out:
            import oracle
            ref = oracle.submatrix(lit_sys)
            out["literal_bf16_water16"]["max_abs_dD_vs_oracle"] = float(np.abs(lit_res.d_values - ref.d_values).max())
            out["literal_bf16_water16"]["dN_vs_oracle"] = lit_res.n_elec - ref.n_elec
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
