#!/usr/bin/env python3
"""Benchmark of the field-dependent PSF operator on one MI355X.

Headline: simulated images per second for the 128 x 128 single-scene workload
(64 sampled PSFs of 128 x 128, a 16384 x 16384 float32 library of 1 GiB built
on the device), S = A Z with the library resident in HBM -- the paper's
"matrix-multiplication" simulation (Sec. 3, Table 4).  One step is one
simulated scene.  The same run also times every other part of the hot path
(library build in each storage form, the 16-bit scaled products, the
adjoint, the batched matrix-core products) and prints them under "rows".

Prints ONE JSON line.  ``--gpus`` above 1 is refused: the operator has no
multi-GPU path, so the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E datasheet
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2516.6, "fp16": 2516.6}  # dense matrix-core peaks


def _timed(torch, fn, iters, warmup):
    """Average milliseconds per call of fn() over `iters` back-to-back calls on
    the current stream, bracketed by HIP events on that stream."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(iters):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / iters


def _timed_cold(torch, fn, iters, warmup):
    """Median milliseconds of fn() with the 256 MB last-level cache (MALL)
    flushed before each call: 1 GiB is written between calls, outside the
    timed region, so no library starts out cache-resident."""
    flush = torch.empty(2**28, dtype=torch.float32, device="cuda")
    for _ in range(warmup):
        fn()
    s = torch.cuda.current_stream()
    times = []
    for _ in range(iters):
        flush.zero_()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        fn()
        e1.record(s)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    del flush
    times.sort()
    return times[len(times) // 2]


def _profiled_traffic():
    """HBM bytes per matvec launch from the committed counter summary, if the
    kernel source is unchanged since the counters were taken (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "matvec_f32_128_hbm_counters.md")
    try:
        kv = {}
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith(("|", "*", "#", " ")):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        src = os.path.join(ROOT, kv["source"])
        with open(src, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != kv["source_sha256"]:
                return None
        return int(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def _lscpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return platform.processor() or "unknown"


def _time_build(torch, psflib, desc, cube, radii, buf, nbytes, reps=3):
    """Milliseconds of one library build (events on the current stream; the
    handle's small workspace allocation is included), best of `reps`."""
    best = None
    for r in range(reps + 1):
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        h = psflib.build(desc, cube.data_ptr(), radii, buf.data_ptr(), nbytes, s.cuda_stream)
        e1.record(s)
        torch.cuda.synchronize()
        psflib.destroy(h)
        if r > 0:
            t = e0.elapsed_time(e1)
            best = t if best is None else min(best, t)
    return best


def probes(torch, psflib, dev):
    """Ceilings measured on this part (the library's probe kernels): the best
    16-byte-load read rate over a sweep of launch shapes on a 2 GiB buffer,
    and the matrix cores' issue rate (FP32, BF16, FP16) on register operands.
    Each is timed with HIP events on the stream the probe runs on."""
    st = torch.cuda.current_stream().cuda_stream
    sink = torch.zeros(65536, dtype=torch.float32, device=dev)
    nbytes = 2 << 30
    buf = torch.zeros(nbytes // 4, dtype=torch.float32, device=dev)
    sweep = {}
    for slice_ in (False, True):
        for wg in (1024, 2048, 4096, 8192, 16384):
            for un in (4, 8, 16):
                ms = _timed(torch, lambda: psflib.probe_hbm_read(buf.data_ptr(), nbytes, wg, un, slice_,
                                                                 sink.data_ptr(), st), 10, 2)
                sweep[f"{'slice' if slice_ else 'stride'}_wg{wg}_u{un}"] = nbytes / (ms * 1e-3) / 1e9
    del buf
    best = max(sweep, key=sweep.get)
    out = {"hbm_read_GB_per_s": sweep[best], "hbm_read_shape": best,
           "hbm_read_sweep_GB_per_s": {k: round(v, 1) for k, v in sweep.items()}}
    wgs = 1024  # 4 workgroups of 4 waves per CU: four waves on every SIMD
    for kind, name, flop, iters in ((0, "fp32", 4096, 8000), (1, "bf16", 32768, 16000),
                                    (2, "fp16", 32768, 16000)):
        ms = _timed(torch, lambda: psflib.probe_mfma(kind, iters, wgs, sink.data_ptr(), st), 10, 3)
        out[f"mfma_{name}_TFLOP_per_s"] = wgs * 4 * iters * 4 * flop / (ms * 1e-3) / 1e12
    return out


def cpu_baseline(d, ref_scenes):
    """The FP64 oracle, as it stands, on the host.  It builds the library
    columns on which the reference scenes are non-zero (their common support:
    the field inside the last sampled offset), times S = A Z over them and
    scales to the full library (the product is linear in the number of
    columns).  The same columns give the exact FP64 images of every scene in
    `ref_scenes` (columns outside the support multiply zeros), which the
    reduced-precision rows are measured against."""
    import numpy as np

    import oracle

    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        threads = max((i.get("num_threads", 1) for i in info if i.get("user_api") == "blas"), default=1)
    except Exception:
        threads = os.cpu_count() or 1
    N = d["N"]
    ncols = N * N
    Zs = np.stack([np.asarray(z, dtype=np.float32).reshape(-1) for z in ref_scenes])
    cols = np.nonzero(np.any(Zs != 0, axis=0))[0]
    t0 = time.perf_counter()
    A = oracle.build_library(d["cube"], d["radii"], N, d["S"], columns=cols)
    t_build = time.perf_counter() - t0
    Z = d["scene"][cols].astype(np.float64)
    reps = []
    for _ in range(10):
        t0 = time.perf_counter()
        oracle.apply(A, Z)
        reps.append(time.perf_counter() - t0)
    t_apply = float(np.median(reps)) * (ncols / cols.size)
    refs = oracle.apply_batched(A, Zs[:, cols])
    del A
    return {
        "value": 1.0 / t_apply, "unit": "scenes/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"FP64 oracle: the {cols.size} library columns inside the last sampled offset "
                   f"built ({cols.size / t_build:.1f} columns/s, one core), then S = A Z over them "
                   f"with numpy BLAS, median of 10, scaled by {ncols}/{cols.size} to the full "
                   f"16384-column library"),
        "build_columns_per_s": cols.size / t_build,
        "host_cpu": _lscpu_model(), "host_cpu_count": os.cpu_count(),
    }, refs


def image_errors(got, ref):
    """Errors of a float32 image against its FP64 reference: peak-normalised
    max |dS| / max S, the largest per-pixel relative error over pixels above
    1e-6 of the peak, and the relative L2 error."""
    import numpy as np
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.abs(got - ref)
    peak = np.abs(ref).max()
    big = np.abs(ref) > 1e-6 * peak
    return {"peak_normalised": float(d.max() / peak),
            "max_rel_above_1e-6_of_peak": float(np.max(d[big] / np.abs(ref[big]))),
            "l2_rel": float(np.linalg.norm(got - ref) / np.linalg.norm(ref))}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probes", action="store_true", help="skip the measured-ceiling probes")
    ap.add_argument("--no-rows", action="store_true", help="time only the headline matvec")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates profiler byte counters)")
    ap.add_argument("--storage", choices=("fp32", "bf16", "fp16"), default="fp32",
                    help="storage form of the headline library (profiling runs of the 16-bit "
                         "matvec and adjoint; the reported metric is defined for fp32)")
    ap.add_argument("--with-adjoint", action="store_true",
                    help="also run --steps adjoint products after the headline (profiling runs)")
    args = ap.parse_args()
    if args.storage != "fp32" and not (args.no_rows and args.no_cpu_baseline):
        print("--storage bf16/fp16 is a profiling mode: give it with --no-rows --no-cpu-baseline",
              file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the operator "
              "has no multi-GPU path (sharding is described, not implemented).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2106_09122_amd import psflib

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    d = synth.config_inputs(2)
    n, N, S, K = d["n"], d["N"], d["S"], d["radii"].size
    M, ncols = n * n, N * N
    cube = torch.from_numpy(d["cube"]).to(dev)
    scene = torch.from_numpy(d["scene"]).to(dev)
    image = torch.empty(M, dtype=torch.float32, device=dev)
    print(f"[bench] workload n={n} N={N} K={K}: building {args.storage} library", file=sys.stderr, flush=True)

    rows = {}
    ref_scenes = [d["scene"]]   # scenes whose FP64 oracle images the CPU leg computes
    gpu_images = {}             # name -> (index into ref_scenes, float32 image on the host)
    lib = psflib.Library(cube, d["radii"], N, S, storage=args.storage)
    torch.cuda.synchronize()

    # headline: FP32 single-scene simulation, library resident
    ms = _timed(torch, lambda: lib.apply(scene, out=image), args.steps, args.warmup)
    lib_bytes = M * ncols * 4 if args.storage == "fp32" else M * ((ncols + 63) // 64 * 64) * 2
    alg_bytes = lib_bytes + 4 * (M + ncols)
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    print(f"[bench] {args.storage} apply {ms * 1e3:.1f} us/scene, {achieved:.0f} GB/s", file=sys.stderr, flush=True)
    if args.with_adjoint:
        gq = torch.randn(M, device=dev, dtype=torch.float32)
        gout = torch.empty(ncols, device=dev, dtype=torch.float32)
        t_adj = _timed(torch, lambda: lib.apply_adjoint(gq, out=gout), args.steps, args.warmup)
        print(f"[bench] {args.storage} adjoint {t_adj * 1e3:.1f} us, {lib_bytes / (t_adj * 1e-3) / 1e9:.0f} GB/s",
              file=sys.stderr, flush=True)
    gpu_images["fp32"] = (0, lib.apply(scene).cpu().numpy())
    ceil = None if args.no_probes else probes(torch, psflib, dev)
    if args.copy_probe:
        src = torch.empty(2**28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        t_copy = _timed(torch, lambda: dst.copy_(src), 20, 3)
        rows["copy_probe_1GiB"] = {"ms": t_copy, "GB_per_s_read_plus_write": 2 * 2**30 / (t_copy * 1e-3) / 1e9}
        del src, dst

    if not args.no_rows:
        # library build (a1-a3), rebuilt into the same buffer
        t_build = _time_build(torch, psflib, lib.desc, cube, d["radii"], lib.buf, lib.nbytes)
        rows["build_fp32"] = {"ms": t_build, "GB_per_s_written": lib_bytes / (t_build * 1e-3) / 1e9,
                              "columns_per_s": ncols / (t_build * 1e-3)}
        g = torch.randn(M, device=dev, dtype=torch.float32)
        grad = torch.empty(ncols, device=dev, dtype=torch.float32)
        t_adj = _timed(torch, lambda: lib.apply_adjoint(g, out=grad), args.steps // 2, 10)
        rows["adjoint_fp32"] = {"us": t_adj * 1e3, "GB_per_s": alg_bytes / (t_adj * 1e-3) / 1e9}
        ref_img = lib.apply(scene).double()
        # the linear-vs-nearest comparison of the paper's Sec. 4.2, on this workload:
        # |S_linear - S_nearest| in percent of the image peak
        ln = psflib.Library(cube, d["radii"], N, S, interp="nearest", storage="fp32")
        t_bn = _time_build(torch, psflib, ln.desc, cube, d["radii"], ln.buf, ln.nbytes)
        pct = 100.0 * (ln.apply(scene).double() - ref_img).abs() / ref_img.abs().max()
        rows["nearest_vs_linear_fp32"] = {"build_ms": t_bn, "build_ratio_vs_linear": t_bn / t_build,
                                          "max_pct_of_peak": float(pct.max()),
                                          "mean_pct_of_peak": float(pct.mean())}
        ln.close()
        del ln, pct
        # cubic-spline rotation (the interpolation of the paper's rotate() calls)
        lc = psflib.Library(cube, d["radii"], N, S, rotate="cubic", storage="fp32")
        t_bc = _time_build(torch, psflib, lc.desc, cube, d["radii"], lc.buf, lc.nbytes)
        pct = 100.0 * (lc.apply(scene).double() - ref_img).abs() / ref_img.abs().max()
        rows["cubic_rotation_fp32"] = {"build_ms": t_bc, "build_ratio_vs_bilinear": t_bc / t_build,
                                       "max_pct_of_peak_vs_bilinear": float(pct.max()),
                                       "mean_pct_of_peak_vs_bilinear": float(pct.mean())}
        lc.close()
        del lc, pct
        # flux-preserving columns: build time and the spread of the column scales
        lf = psflib.Library(cube, d["radii"], N, S, flux="preserve", storage="fp32")
        t_bf = _time_build(torch, psflib, lf.desc, cube, d["radii"], lf.buf, lf.nbytes)
        t0, t1 = lib.column_sums(), lf.column_sums()
        live = t0 != 0
        sc = (t1[live] / t0[live]).cpu().numpy()
        rows["flux_preserve_fp32"] = {"build_ms": t_bf, "build_ratio_vs_plain": t_bf / t_build,
                                      "column_scale_min": float(sc.min()),
                                      "column_scale_max": float(sc.max())}
        lf.close()
        del lf
        for B in (1, 8, 64, 256):
            Zb = torch.from_numpy(synth.scene_batch(N, S, B, config=2, rmax_mask=8.0)).to(dev)
            out = torch.empty((B, M), device=dev, dtype=torch.float32)
            t_b = _timed(torch, lambda: lib.apply_batched(Zb, out=out), 10, 3)
            fl = 2.0 * M * ncols * B
            ent = {"ms": t_b, "scenes_per_s": B / (t_b * 1e-3), "TFLOP_per_s": fl / (t_b * 1e-3) / 1e12,
                   "frac_mfma_fp32": fl / (t_b * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS["fp32"]}
            if ceil:
                ent["frac_mfma_fp32_of_measured"] = fl / (t_b * 1e-3) / 1e12 / ceil["mfma_fp32_TFLOP_per_s"]
            if B < 40:  # below the ridge (157.3 TF / 8 TB/s): the library read binds
                gbs = (lib_bytes + 4 * B * (M + ncols)) / (t_b * 1e-3) / 1e9
                ent.update({"bound": "hbm", "GB_per_s": gbs, "frac_hbm": gbs / HBM_PEAK_GBS})
            rows[f"batched_fp32_B{B}"] = ent
            del Zb, out
        # differentiation: one fitting step (render disk, simulate, chi-square,
        # backward through the adjoint and the renderer) on the 128^2 library
        from paper_2106_09122_amd import fit
        Ztrue = fit.render_disk(torch.tensor(synth.DISK_TRUE, dtype=torch.float64, device=dev),
                                N, S, 8.0)
        counts, Kc, var = synth.noisy_counts(lib.apply(Ztrue).cpu().numpy(), 2e4,
                                             synth.rng_for(4, synth.STREAM_NOISE))
        ct = torch.from_numpy(counts).to(dev)
        vt = torch.from_numpy(var).to(dev)
        th0 = torch.tensor(synth.DISK_START, dtype=torch.float64, device=dev)
        t_fit = _timed(torch, lambda: fit.loss_and_grad(lib, th0, ct, vt, Kc, 8.0), 50, 5)
        rows["fit_step_fp32"] = {"ms": t_fit, "steps_per_s": 1e3 / t_fit,
                                 "note": "render + A Z + chi2 + A^T g + render gradient"}
        # the paper's own shape (its IPAC set): 128^2 PSFs at 0.2 lambda/D with 86
        # non-uniform offsets to 11 lambda/D, a 256^2 scene at 3.529 mas: a
        # 16384 x 65536 library (4 GiB FP32); the paper's CPU times for this
        # shape (FP64, 8 cores) are quoted beside it as context
        dp = synth.config_inputs(6)
        cp = torch.from_numpy(dp["cube"]).to(dev)
        zp = torch.from_numpy(dp["scene"]).to(dev)
        lp = psflib.Library(cp, dp["radii"], dp["N"], dp["S"], storage="fp32")
        t_bp = _time_build(torch, psflib, lp.desc, cp, dp["radii"], lp.buf, lp.nbytes)
        ip = torch.empty(dp["n"] ** 2, dtype=torch.float32, device=dev)
        t_ap = _timed(torch, lambda: lp.apply(zp, out=ip), 100, 10)
        pbytes = dp["n"] ** 2 * dp["N"] ** 2 * 4
        rows["paper_shape_fp32"] = {
            "shape": "n=128 (s=0.2 lambda/D), N=256 (S=3.529 mas), 86 non-uniform offsets, A 16384 x 65536",
            "build_ms": t_bp, "apply_ms": t_ap, "apply_GB_per_s": pbytes / (t_ap * 1e-3) / 1e9,
            "paper_cpu_fp64_build_s": 506.680, "paper_cpu_fp64_apply_s": 0.1642,
            "paper_source": "Table 2 (IPAC, linear, time to create) and Table 4 (IPAC, linear)"}
        lp.close()
        del lp, cp, zp, ip
        # the large library (256^2 PSFs and scene, 128 PSFs: 65536 x 65536, 2^32
        # entries): build, matvec and a 64-scene batched product, FP32 and BF16
        d5 = synth.config_inputs(5)
        c5 = torch.from_numpy(d5["cube"]).to(dev)
        z5 = torch.from_numpy(d5["scene"]).to(dev)
        M5, K5 = d5["n"] ** 2, d5["N"] ** 2
        Zb5 = torch.from_numpy(synth.scene_batch(d5["N"], d5["S"], 64, config=5, rmax_mask=8.0)).to(dev)
        o5 = torch.empty((64, M5), device=dev, dtype=torch.float32)
        i5 = torch.empty(M5, device=dev, dtype=torch.float32)
        ent5 = {"shape": "n = N = 256, 128 PSFs: A 65536 x 65536 (2^32 entries)"}
        for fmt in ("fp32", "bf16"):
            l5 = psflib.Library(c5, d5["radii"], d5["N"], d5["S"], storage=fmt)
            t_b5 = _time_build(torch, psflib, l5.desc, c5, d5["radii"], l5.buf, l5.nbytes, reps=2)
            t_a5 = _timed(torch, lambda: l5.apply(z5, out=i5), 20, 3)
            t_g5 = _timed(torch, lambda: l5.apply_batched(Zb5, out=o5), 3, 1)
            abytes = M5 * K5 * (4 if fmt == "fp32" else 2)
            fl = 2.0 * M5 * K5 * 64
            ent5[fmt] = {"build_ms": t_b5, "apply_ms": t_a5,
                         "apply_GB_per_s": abytes / (t_a5 * 1e-3) / 1e9,
                         "batched_B64_ms": t_g5,
                         "batched_B64_TFLOP_per_s": fl / (t_g5 * 1e-3) / 1e12,
                         "batched_B64_frac_mfma": fl / (t_g5 * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS[fmt],
                         "batched_B64_GB_per_s": abytes / (t_g5 * 1e-3) / 1e9}
            l5.close()
            del l5
        rows["large_256"] = ent5
        del c5, z5, Zb5, o5, i5
        # mixed sizes and wavelengths: 256 scenes over 33 libraries, one graph launch
        libs_m, scene_lib, scenes_m = synth.mixed_workload()
        Zm = [torch.from_numpy(z).to(dev) for z in scenes_m]
        for fmt in ("fp32", "fp16"):
            Ls = [psflib.Library(torch.from_numpy(l["cube"]).to(dev), l["radii"], l["N"], l["S"],
                                 storage=fmt) for l in libs_m]
            torch.cuda.synchronize()
            gp = psflib.Grouped(Ls, scene_lib, Zm, autotune=True)
            t_g = _timed_cold(torch, lambda: gp.run(), 10, 2)
            used = sorted(set(scene_lib))
            nbytes = sum(Ls[L].M * (Ls[L].ncols if fmt == "fp32" else (Ls[L].ncols + 63) // 64 * 64)
                         * (4 if fmt == "fp32" else 2) for L in used)
            rows[f"grouped_{fmt}"] = {"ms": t_g, "timing": "median of 10, MALL flushed before each",
                                      "scenes_per_s": len(scene_lib) / (t_g * 1e-3),
                                      "GB_per_s": nbytes / (t_g * 1e-3) / 1e9,
                                      "frac_hbm": nbytes / (t_g * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                      "libraries": len(used), "scenes": len(scene_lib),
                                      "tile_shape": gp.shape()}
            gp.close()
            for Lb in Ls:
                Lb.close()
            del Ls, gp
        del Zm
        batches = {B: synth.scene_batch(N, S, B, config=2, rmax_mask=8.0) for B in (256, 512, 1024)}
        NREF = 16  # scenes per batch whose FP64 images the CPU leg computes
        for B, Zb_h in batches.items():
            ref_scenes.extend(Zb_h[:NREF])
        for fmt in ("bf16", "fp16"):
            lh = psflib.Library(cube, d["radii"], N, S, storage=fmt)
            torch.cuda.synchronize()
            t_b16 = _time_build(torch, psflib, lh.desc, cube, d["radii"], lh.buf, lh.nbytes)
            ms16 = _timed(torch, lambda: lh.apply(scene, out=image), args.steps, args.warmup)
            img16 = lh.apply(scene)
            gpu_images[fmt] = (0, img16.cpu().numpy())
            img16 = img16.double()
            err = float((img16 - ref_img).abs().max() / ref_img.abs().max())
            ent = {"build_ms": t_b16, "apply_us": ms16 * 1e3, "scenes_per_s": 1e3 / ms16,
                   "GB_per_s": (M * ((ncols + 63) // 64 * 64) * 2 + 4 * (M + 2 * ncols)) / (ms16 * 1e-3) / 1e9,
                   "speedup_vs_fp32": ms / ms16,
                   "peak_normalised_error_vs_fp32": err}
            t_adj16 = _timed(torch, lambda: lh.apply_adjoint(g, out=grad), args.steps // 2, 10)
            ent["adjoint_us"] = t_adj16 * 1e3
            ent["adjoint_GB_per_s"] = M * ((ncols + 63) // 64 * 64) * 2 / (t_adj16 * 1e-3) / 1e9
            ent["frac_hbm"] = ent["GB_per_s"] / HBM_PEAK_GBS
            ent["adjoint_frac_hbm"] = ent["adjoint_GB_per_s"] / HBM_PEAK_GBS
            for bi, (B, Zb_h) in enumerate(batches.items()):
                Zb = torch.from_numpy(Zb_h).to(dev)
                out = torch.empty((B, M), device=dev, dtype=torch.float32)
                t_b = _timed(torch, lambda: lh.apply_batched(Zb, out=out), 10, 3)
                fl = 2.0 * M * ncols * B
                ent[f"batched_B{B}"] = {"ms": t_b, "scenes_per_s": B / (t_b * 1e-3),
                                        "TFLOP_per_s": fl / (t_b * 1e-3) / 1e12,
                                        "frac_mfma": fl / (t_b * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS[fmt]}
                if ceil:
                    ent[f"batched_B{B}"]["frac_mfma_of_measured"] = (
                        fl / (t_b * 1e-3) / 1e12 / ceil[f"mfma_{fmt}_TFLOP_per_s"])
                lh.apply_batched(Zb, out=out)
                host = out[:NREF].cpu().numpy()
                for r in range(NREF):
                    gpu_images[f"{fmt}_B{B}_{r}"] = (1 + bi * NREF + r, host[r])
                del Zb, out
            rows[f"{fmt}_pow2"] = ent
            lh.close()
            del lh

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        cpu, refs = cpu_baseline(d, ref_scenes)
        # every image against the exact FP64 image of the same scene
        errs = {"fp32": image_errors(gpu_images["fp32"][1], refs[0])}
        for fmt in ("bf16", "fp16"):
            if fmt not in gpu_images:
                continue
            e16 = image_errors(gpu_images[fmt][1], refs[0])
            ent = rows[f"{fmt}_pow2"]
            ent["error_vs_fp64"] = e16
            ent["meets_1e-3_vs_fp64"] = e16["peak_normalised"] <= 1e-3
            for key in list(ent):
                if key.startswith("batched_B"):
                    B = key[len("batched_B"):]
                    worst = max(image_errors(img, refs[i])["peak_normalised"]
                                for name, (i, img) in gpu_images.items()
                                if name.startswith(f"{fmt}_B{B}_"))
                    ent[key]["peak_normalised_error_vs_fp64_worst_of_16"] = worst
        rows["fp32_error_vs_fp64"] = errs["fp32"]

    line = {
        "metric": "scenes/sec + % HBM (matvec) / % MFMA (batched) at 128², FP32 vs BF16-scaled",
        "value": 1e3 / ms,
        "unit": "scenes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "fp32" else args.storage,
        "data": "synthetic (seeded Fraunhofer PSF cube with Zernike aberrations and a coronagraph "
                "throughput ramp; inclined power-law ring + 5 planets)",
        "config": {"workload": "single-scene matvec, 128x128 image and scene, 64 PSFs of 128x128, "
                               "16384x16384 float32 library (1 GiB) resident in HBM",
                   "n": n, "N": N, "n_psf": K, "pixscale_lod": S, "library_bytes": lib_bytes,
                   "parallelism": "single GPU", "storage": args.storage},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": _profiled_traffic() if args.storage == "fp32" else None,
                     "kernel": "matvec_f32_kernel" if args.storage == "fp32" else "matvec_h16_kernel",
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "measured_peak": ceil["hbm_read_GB_per_s"] if ceil else None,
                     "frac_of_measured": achieved / ceil["hbm_read_GB_per_s"] if ceil else None},
        "measured_ceilings": ceil,
        "cpu_baseline": cpu,
        "rows": rows,
    }
    print(json.dumps(line), flush=True)
    lib.close()


if __name__ == "__main__":
    main()
