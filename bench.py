#!/usr/bin/env python3
"""Benchmark of the batched 1D depth inversions of extended diffraction tomography.

Metric: 1D subproblems (k_m values) solved per second on one MI355X, for the
mixed-precision path (split-half Gram on MFMA -- FP16x3 by default, BF16x3
also timed -- + FP64 Cholesky + FP64 refinement) next to the plain FP64 path
(FP64 MFMA Gram + FP64 Cholesky), at relative error <= 1e-6 (mixed) /
<= 1e-10 (FP64) against the FP64 CPU oracle.

Workload (default): the 2D layered survey -- 512 surface positions at 12.5 m
(512 k_m, 257 +-k_m pairs), 8-layer reference, nz = 256 at 8 m, 128
frequencies 3-60 Hz, smooth random model, 5% complex Gaussian data noise.
A step is one pass of green -> assemble -> solve(-> refine -> recombine) over
the whole survey with inputs resident in HBM, captured once into a HIP graph
and replayed; per-kernel times come from an eager pass with the library's
HIP-event timer.

Inputs are synthesised on the GPU (Born forward map of the seeded model plus
counter-based noise); the CPU-baseline leg re-derives its own data with the
oracle, times the oracle on a sample of pairs, and feeds that same oracle
data through the GPU path once more to state the error on identical inputs.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "1D subproblems solved/s, mixed vs FP64 plain, at rel err ≤1e-6 vs FP64 oracle"
PEAK = {"bf16": 2500.0, "fp16": 2500.0, "fp32": 157.3, "fp64": 78.6, "hbm": 8000.0}   # TFLOP/s, GB/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--mixed", default="fp16x3", choices=["bf16x3", "fp16x3", "fp32"],
                    help="mixed path of the headline value")
    ap.add_argument("--also", default="bf16x3", help="comma-separated further mixed paths timed for the detail "
                    "('' for none)")
    ap.add_argument("--refine-tol", type=float, default=3e-6)
    ap.add_argument("--max-refine", type=int, default=8)
    ap.add_argument("--chunk", type=int, default=0, help="rows per Gram item (0 = planner default)")
    ap.add_argument("--band", type=int, default=0, help="frequencies per Gram band (0 = planner default)")
    ap.add_argument("--cpu-pairs", type=int, default=0,
                    help="pairs in the oracle leg (0: 160 for the 2D surveys, 512 for the 3D 128 x 128 one)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg (profiling runs)")
    ap.add_argument("--only", choices=["both", "mixed", "fp64"], default="both")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the work-item shapes per precision first and store them in the tuned-shape "
                         "table (EDT_TUNE_CACHE, else the package's table)")
    ap.add_argument("--default-shapes", action="store_true",
                    help="use the planner's default work-item shapes instead of the tuned-shape table")
    ap.add_argument("--stream", action="store_true",
                    help="solve in pair-range batches (always on for config 5, the 3D 256 x 256 survey)")
    ap.add_argument("--batch-rows", type=int, default=100_000_000, help="data rows per batch at most")
    ap.add_argument("--batch-pairs", type=int, default=4096, help="pairs per batch at most")
    ap.add_argument("--data", choices=["c128", "c64"], default=None,
                    help="storage of the data rows (default: complex64 for the 3D 256 x 256 survey, whose "
                         "data are complex FP32, else complex128)")
    ap.add_argument("--hbm-budget", type=float, default=None,
                    help="device bytes the batch stream may hold (default: 200e9 for the 3D 256 x 256 survey)")
    ap.add_argument("--tsvd", type=float, default=1e-2,
                    help="relative tolerance of the truncated-SVD leg (the paper's own solver), "
                         "timed after the main passes; 0 skips it")
    ap.add_argument("--lines-only", action="store_true",
                    help="time only the 3D survey of parallel lines (profiling runs of its kernels)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run three plain 1 GiB device copies (the reference for the HBM byte "
                         "counters FETCH_SIZE / WRITE_SIZE) and exit")
    return ap.parse_args()


def copy_calibration(torch):
    """Three launches of a plain device copy that reads and writes exactly 1 GiB:
    under rocprofv3 --pmc it gives the counter reading of known traffic."""
    n = 1 << 27   # 128 Mi doubles
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_launch": n * 8, "launches": 3}))


def synth_inputs(s, plan, vel, torch):
    """Data rows from the HIP forward map plus counter-based noise (no oracle)."""
    from edt_inputs import noise, vhat
    g64, _ = plan.green(vel, want32=False)
    d = plan.forward(g64, torch.from_numpy(vhat(s)).cuda())
    if s.noise_rel == 0.0:
        return d
    m = plan.rowmap()
    dn = d.cpu().numpy()
    f = m["rows"][:, 0].astype(np.int64)
    mx = np.zeros(s.n_freq)
    np.maximum.at(mx, f, np.maximum(np.abs(dn[:, 0]), np.abs(dn[:, 1])))
    scale = s.noise_rel * mx
    keys = m["keys"].astype(np.int64)
    if s.dim == 2:
        N = s.n_mid
        k0 = (keys[:, 0], keys[:, 1])
        k1 = ((-keys[:, 1]) % N, (-keys[:, 0]) % N)
    else:
        pair = np.repeat(np.arange(plan.n_pairs), np.diff(m["row_off"]))
        k0 = (m["pair_km"][pair, 0], keys[:, 0])
        k1 = (m["pair_km"][pair, 1], keys[:, 0])
    dn[:, 0] += scale[f] * noise(s.seed, f, *k0)
    dn[:, 1] += scale[f] * noise(s.seed, f, *k1)
    return torch.from_numpy(dn).cuda()


def time_steps(pipe, steps, warmup, torch):
    """ms per step of the captured pass (HIP graph replays bracketed by
    device synchronisations and events on the replay stream), and of the
    eager pass for reference."""
    pipe.capture(warmup=max(1, warmup))
    for _ in range(warmup):
        pipe.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        pipe.replay()
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    graph_ms = e0.elapsed_time(e1) / steps
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        pipe.step()
    e1.record()
    torch.cuda.synchronize()
    return graph_ms, wall, e0.elapsed_time(e1) / steps


def kernel_times(pipe, steps, torch):
    """Average duration per launch of every kernel over `steps` eager passes,
    measured with HIP events recorded by the library on the launch stream."""
    pipe.p.timing(True)
    pipe.p.timing_read()
    for _ in range(steps):
        pipe.step()
    torch.cuda.synchronize()
    t = pipe.p.timing_read()
    pipe.p.timing(False)
    return {k: {"avg_ms": ms / max(n, 1), "launches_per_step": n / steps, "ms_per_step": ms / steps}
            for k, (ms, n) in t.items()}


def _bf16_mfma_flops(plan, nz):
    """FP flops the BF16x3 Gram kernel issues to MFMA: per stage of 8 unique
    rows, every lower 32x32 tile gets three 32x32x16 products."""
    items, _ = plan.schedule("gram")
    stages = int(np.sum((items[:, 2] - items[:, 1] + 7) // 8))
    nt = (nz + 31) // 32
    return stages * (nt * (nt + 1) // 2) * 3 * 32 * 32 * 16 * 2.0


def _f64_mfma_flops(plan, nz):
    """FP64 flops the FP64 Gram kernel issues to MFMA: per stage of 8 unique
    rows (16 real rows), every lower 16x16 tile gets four 16x16x4 products."""
    items, _ = plan.schedule("gram")
    stages = int(np.sum((items[:, 2] - items[:, 1] + 7) // 8))
    nb = 2 * ((nz + 31) // 32)
    return stages * (nb * (nb + 1) // 2) * 4 * 16 * 16 * 4 * 2.0


def measured_traffic(kernel, workload, prec, shape):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes scaled by a plain-copy calibration), or
    None if there is none for this workload, precision and work-item shape
    (chunk_rows, gram_band, resid_group as the plan uses them), or if the
    kernel's source changed since it was taken."""
    import glob
    import hashlib
    for fn in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")):
        with open(fn) as fh:
            t = json.load(fh)
        if t.get("kernel") != kernel or t.get("workload") != workload or t.get("precision") != prec:
            continue
        if t.get("shape") != shape:
            continue
        with open(os.path.join(ROOT, t["source"]), "rb") as fh:
            if hashlib.sha1(fh.read()).hexdigest() != t["source_sha1"]:
                return None
        return float(t["hbm_bytes_per_launch"])
    return None


def roofline(plan, s, ktimes, prec, steps):
    """Roofline entry of the dominant kernel of one step.  Algorithmic work
    counts the distinct Born rows (rows merged by reciprocity are formed once):
    the symmetric Gram is 2 U nz (nz+1) flops; a refinement residual is 22 nz
    FP64 flops per unique row of every pair still iterating (6 to form the row,
    8 for A x, 8 for A^H e)."""
    info = plan.info
    dom = max(ktimes, key=lambda k: ktimes[k]["ms_per_step"])
    kt = ktimes[dom]
    avg_s = kt["avg_ms"] * 1e-3
    U = info["n_urows"]
    if dom.startswith("gram_"):
        dt = {"gram_bf16x3": "bf16", "gram_fp16x3": "fp16", "gram_fp32": "fp32", "gram_fp64": "fp64"}[dom]
        fl = 2.0 * U * s.nz * (s.nz + 1)
        ach = fl / avg_s / 1e12
        out = {"bound": "mfma", "achieved": ach, "peak": PEAK[dt], "unit": "TFLOP/s",
               "frac": ach / PEAK[dt], "traffic": None,
               "per_launch": f"2 U nz (nz+1) = {fl:.4g} flop (U = {U} unique rows)"}
        ex = {"bf16": _bf16_mfma_flops, "fp16": _bf16_mfma_flops, "fp64": _f64_mfma_flops}.get(dt)
        if ex is not None:
            out["mfma_issued_frac"] = ex(plan, s.nz) / avg_s / 1e12 / PEAK[dt]
        return dom, out
    if dom == "refine residual":
        uo = plan.urows()["urow_off"]
        per_pair = np.diff(uo).astype(np.float64)
        fl_step = 22.0 * s.nz * float(np.sum(per_pair * steps))   # over all launches of one step
        ach = fl_step / (kt["ms_per_step"] * 1e-3) / 1e12
        return dom, {"bound": "alu", "achieved": ach, "peak": PEAK["fp64"], "unit": "TFLOP/s",
                     "frac": ach / PEAK["fp64"], "traffic": None,
                     "per_launch": f"22 nz x (unique rows of the pairs still iterating); "
                                   f"{fl_step / kt['launches_per_step']:.4g} flop per launch on average"}
    if dom == "green":
        by = info["table_elems"] * (16 + (8 if prec != "fp64" else 0))
        ach = by / avg_s / 1e9
        return dom, {"bound": "hbm", "achieved": ach, "peak": PEAK["hbm"], "unit": "GB/s",
                     "frac": ach / PEAK["hbm"], "traffic": None,
                     "per_launch": f"table writes {by:.4g} B"}
    # Cholesky / solves: the Gram is read and the factor written once
    by = 2.0 * plan.n_pairs * s.nz * (s.nz + 1) / 2 * 8
    ach = by / avg_s / 1e9
    return dom, {"bound": "hbm", "achieved": ach, "peak": PEAK["hbm"], "unit": "GB/s",
                 "frac": ach / PEAK["hbm"], "traffic": None,
                 "per_launch": f"lower triangles read + written {by:.4g} B"}


def gram_mfma(plan, s, ktimes):
    """MFMA use of one precision's Gram kernel: the algorithmic 2 U nz (nz+1)
    flop per launch and, for the split and FP64 kernels, the MFMA work the
    kernel actually issues (three 16-bit products per algorithmic product,
    padding stages included), each against the dense peak of its input type."""
    name = next((k for k in ktimes if k.startswith("gram_") and k != "gram_reduce"), None)
    if name is None:
        return None
    dt = {"gram_bf16x3": "bf16", "gram_fp16x3": "fp16", "gram_fp32": "fp32", "gram_fp64": "fp64"}[name]
    avg_s = ktimes[name]["avg_ms"] * 1e-3
    alg = 2.0 * plan.info["n_urows"] * s.nz * (s.nz + 1) / avg_s / 1e12
    out = {"kernel": name, "avg_ms": ktimes[name]["avg_ms"], "peak_tflops": PEAK[dt],
           "algorithmic_tflops": alg, "algorithmic_frac": alg / PEAK[dt]}
    ex = {"bf16": _bf16_mfma_flops, "fp16": _bf16_mfma_flops, "fp64": _f64_mfma_flops}.get(dt)
    if ex is not None:
        out["issued_frac"] = ex(plan, s.nz) / avg_s / 1e12 / PEAK[dt]
    return out


def tsvd_leg(plan, vel, d, tol_rel, reps, torch):
    """The paper's truncated-SVD solve (edt_tsvd) on the FP64 Gram of the same
    data, plain and restricted to the paper's (k_m, k_z) disk (edt_kz_restrict
    first, radius 2.2 w_max / c_top): time per solve (the Gram and rhs are
    copied in first, since the solve overwrites them; the copy is not timed),
    sign steps, and two MFMA rates over the library timer's kernel times,
    against the FP64 MFMA peak:
    * the sign iteration's products -- symmetric, so nz^2 (nz + 1) flop each
      (the lower triangle), two per step of every pair still iterating;
    * the restriction's Q G Q -- 2 nz^3 flop for G Q and nz^2 (nz + 1) for the
      lower triangle of Q (G Q), every pair."""
    g64, _ = plan.green(vel, want32=False)
    gram0, rhs0, _ = plan.assemble(g64, None, d, "fp64")
    gram, rhs = torch.empty_like(gram0), torch.empty_like(rhs0)
    work = plan.tsvd_work()
    P, nz = plan.n_pairs, plan.nz
    out = (torch.empty(P, 2, nz, dtype=torch.float64, device="cuda"),
           torch.empty(plan.n_km, nz, dtype=torch.complex128, device="cuda"),
           torch.empty(P, dtype=torch.int32, device="cuda"), torch.zeros(P, dtype=torch.int32, device="cuda"))
    n_keep = torch.empty(P, dtype=torch.int32, device="cuda")
    K = plan.kz_disk_radius(2.2)

    def solve(kz):
        if kz:
            plan.kz_restrict(gram, rhs, K, work, n_keep=n_keep)
        plan.tsvd(gram, rhs, tol_rel, out=out, tsvd_work=work)

    def leg(kz):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tot = 0.0
        for r in range(reps + 1):
            gram.copy_(gram0)
            rhs.copy_(rhs0)
            ev0.record()
            solve(kz)
            ev1.record()
            torch.cuda.synchronize()
            if r > 0:
                tot += ev0.elapsed_time(ev1)
        gram.copy_(gram0)
        rhs.copy_(rhs0)
        torch.cuda.synchronize()
        plan.timing(True)
        plan.timing_read()
        solve(kz)
        kt = plan.timing_read()
        plan.timing(False)
        it = out[3].cpu().numpy().astype(np.float64)
        info = out[2].cpu().numpy()
        fl = float(np.sum(it)) * 2 * float(nz) ** 2 * (nz + 1)
        sign_ms = kt.get("tsvd sign step", (float("nan"), 0))[0]
        ach = fl / (sign_ms * 1e-3) / 1e12
        res = {"ms_per_solve": tot / reps,
               "sign_steps": {"max": int(it.max()), "mean": float(it.mean())},
               "info_noconv": int(np.sum(info == -2)),
               "kernels_ms": {k: round(v[0], 4) for k, v in kt.items()},
               "sign_gemm": {"bound": "mfma", "achieved": ach, "peak": PEAK["fp64"], "unit": "TFLOP/s",
                             "frac": ach / PEAK["fp64"],
                             "per_solve": f"2 symmetric products x nz^2 (nz+1) flop x sign steps summed over "
                                          f"pairs = {fl:.4g} flop"}}
        if kz:
            nk = n_keep.cpu().numpy()
            fk = P * (2.0 * nz ** 3 + float(nz) ** 2 * (nz + 1))
            kz_ms = kt.get("kz restrict", (float("nan"), 0))[0]
            ak = fk / (kz_ms * 1e-3) / 1e12
            res["disk"] = {"radius": K, "factor": 2.2, "kept_modes_mean": float(nk.mean()),
                           "pairs_cut": int(np.sum(nk < nz)), "pairs_empty": int(np.sum(nk == 0))}
            res["kz_gemm"] = {"bound": "mfma", "achieved": ak, "peak": PEAK["fp64"], "unit": "TFLOP/s",
                              "frac": ak / PEAK["fp64"],
                              "per_solve": f"P (2 nz^3 + nz^2 (nz+1)) = {fk:.4g} flop"}
        return res

    out_d = {"tol_rel": tol_rel}
    out_d.update(leg(False))
    out_d["kz_disk"] = leg(True)
    return out_d


def shots_leg(plan, reps, torch):
    """The transforms on either side (2D surveys): seeded records
    [n_freq][N][N] (complex128, resident) -> d_mid * DFT2 in place ->
    packed rows, and the solution spectrum -> model.  Time per call and the
    HBM rate of the transform over the library timer's time: each of its two
    passes reads and writes the records once, so 4 * 16 * n_freq * N^2 bytes
    per call; the pack reads two values and writes two per row."""
    if plan.dim != 2:
        return None
    g = torch.Generator(device="cuda").manual_seed(5)
    shape = (plan.n_freq, plan.n_mid, plan.n_mid)
    rec0 = torch.complex(torch.randn(shape, generator=g, device="cuda", dtype=torch.float64),
                         torch.randn(shape, generator=g, device="cuda", dtype=torch.float64))
    rec = torch.empty_like(rec0)
    d = plan.shots_pack(rec0)
    v = torch.complex(torch.randn(plan.n_km, plan.nz, generator=g, device="cuda", dtype=torch.float64),
                      torch.randn(plan.n_km, plan.nz, generator=g, device="cuda", dtype=torch.float64))
    m = plan.model(v)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tot = 0.0
    for r in range(reps + 1):
        rec.copy_(rec0)
        ev0.record()
        plan.shots_fft(rec)
        plan.shots_pack(rec, out=d)
        ev1.record()
        torch.cuda.synchronize()
        if r > 0:
            tot += ev0.elapsed_time(ev1)
    rec.copy_(rec0)
    torch.cuda.synchronize()
    plan.timing(True)
    plan.timing_read()
    plan.shots_fft(rec)
    plan.shots_pack(rec, out=d)
    plan.model(v, out=m)
    kt = plan.timing_read()
    plan.timing(False)
    nb = 4.0 * 16 * plan.n_freq * plan.n_mid ** 2
    fft_ms = kt.get("shots fft", (float("nan"), 0))[0]
    ach = nb / (fft_ms * 1e-3) / 1e9
    return {"records": list(shape), "ms_per_call": tot / reps,
            "kernels_ms": {k: round(v_[0], 4) for k, v_ in kt.items()},
            "fft_hbm": {"bound": "hbm", "achieved": ach, "peak": PEAK["hbm"], "unit": "GB/s", "frac": ach / PEAK["hbm"],
                        "per_call": f"2 passes x (read + write) x 16 B x n_freq N^2 = {nb:.4g} B"}}


def lines_leg(reps, torch):
    """3D survey of parallel lines (FP64): 128 positions at 12.5 m on 32
    lines 25 m apart, nz = 128, 32 frequencies 4-40 Hz, four layers, with the
    evanescent cut; data from the device Born map of the seeded model.  Times
    per call of green + assemble + damped solve, of the finite-aperture Gram
    (b = 0.15 N_x dx) and of the adjoint.  The Gram's algorithmic work is 2 nz (nz + 1)
    flop per row; its rate over the whole pass (the rows' forming, a sum of
    up to N_y products per value, is inside the time) against the FP64 MFMA
    peak."""
    import paper_0905_0238_amd as E
    from edt_inputs import make_lines, vhat
    s = make_lines(Nx=128, Ny=32, dx=12.5, dy=25.0, nz=128, dz=10.0, freqs=tuple(np.linspace(4.0, 40.0, 32)),
                   vel=(1600.0, 2200.0, 2900.0, 3500.0), zif=(150.0, 450.0, 900.0), kappa=1.0, seed=7)
    p = E.Plan(s)
    vel = torch.tensor(np.asarray(s.vel, np.float64), device="cuda")
    g64, _ = p.green(vel, want32=False)
    d = p.forward(g64, torch.from_numpy(np.ascontiguousarray(vhat(s))).cuda())
    b = 0.15 * s.n_mid * s.d_mid
    work = p.aperture_work()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_solve = t_ap = 0.0
    for r in range(reps + 1):
        ev[0].record()
        g64, _ = p.green(vel, want32=False)
        gram, rhs, trace = p.assemble(g64, None, d, "fp64")
        x, v, info, _ = p.solve(g64, d, gram, rhs, trace, s.lambda_rel)
        ev[1].record()
        p.aperture_gram(g64, b, work=work)
        ev[2].record()
        torch.cuda.synchronize()
        if r > 0:
            t_solve += ev[0].elapsed_time(ev[1])
            t_ap += ev[1].elapsed_time(ev[2])
    t_solve /= reps
    t_ap /= reps
    # the adjoint of the last pass (data, damping and velocity gradients)
    g = torch.Generator(device="cuda").manual_seed(3)
    gv = torch.complex(torch.randn(p.n_km, s.nz, generator=g, device="cuda", dtype=torch.float64),
                       torch.randn(p.n_km, s.nz, generator=g, device="cuda", dtype=torch.float64))
    t_adj = 0.0
    for r in range(reps + 1):
        ev[0].record()
        p.adjoint(vel, g64, d, gram, trace, x, s.lambda_rel, gv)
        ev[1].record()
        torch.cuda.synchronize()
        if r > 0:
            t_adj += ev[0].elapsed_time(ev[1])
    t_adj /= reps
    fl = float(p.n_rows) * 2 * s.nz * (s.nz + 1)
    ach = fl / (t_solve * 1e-3) / 1e12
    return {"survey": "128 positions x 32 lines, nz 128, 32 frequencies", "pairs": int(p.n_pairs),
            "rows": int(p.n_rows), "ms_per_pass": t_solve, "subproblems_per_s": p.n_km / (t_solve * 1e-3),
            "aperture_ms_per_call": t_ap, "aperture_b_m": b, "adjoint_ms_per_call": t_adj,
            "assembly_products": {"bound": "mfma", "achieved": ach, "peak": PEAK["fp64"], "unit": "TFLOP/s",
                                  "frac": ach / PEAK["fp64"],
                                  "per_pass": f"rows x 2 nz (nz+1) = {fl:.4g} flop over the whole pass "
                                              f"(rows, products, right-hand sides and solve inside the time)"}}


def aperture_leg(plan, vel, d_mid, reps, torch):
    """Finite aperture (2D): the windowed Gram of every pair with the paper's
    aperture-to-line ratio (a 6 km full-offset window on its 40 km line, so
    b = 0.075 N dx), timed per call; rate of the lower-tile products over the
    whole call: 2 nW real parts x nz (nz + 1) flop per pair and frequency
    (nW kept offsets), against the FP64 MFMA peak."""
    if plan.dim != 2:
        return None
    g64, _ = plan.green(vel, want32=False)
    N = plan.n_mid
    b = 0.075 * N * d_mid
    sidx = np.arange(-(N // 2), (N - 1) // 2 + 1)
    nW = int(np.sum(np.abs(sidx) * d_mid <= 2.0 * b))
    work = plan.aperture_work()
    gram, trace = plan.aperture_gram(g64, b, work=work)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tot = 0.0
    for r in range(reps + 1):
        ev0.record()
        plan.aperture_gram(g64, b, out=(gram, trace), work=work)
        ev1.record()
        torch.cuda.synchronize()
        if r > 0:
            tot += ev0.elapsed_time(ev1)
    ms = tot / reps
    fl = float(plan.n_pairs) * plan.n_freq * 2 * nW * plan.nz * (plan.nz + 1)
    ach = fl / (ms * 1e-3) / 1e12
    return {"b_max_m": b, "offsets_kept": nW, "n_mid": N, "ms_per_call": ms,
            "gram_products": {"bound": "mfma", "achieved": ach, "peak": PEAK["fp64"], "unit": "TFLOP/s",
                              "frac": ach / PEAK["fp64"],
                              "per_call": f"P n_freq 2 nW nz (nz+1) = {fl:.4g} flop (rows, transforms and products "
                                          f"all inside the timed call)"}}


_CPU_JOB = None   # (survey, oracle plan, sampled pairs, their data): read by forked workers


def _oracle_chunk(idx):
    """One host process: the FP64 oracle solve of the sampled pairs idx
    (their G0 tables, Born rows, normal equations, Cholesky) on one core."""
    from threadpoolctl import threadpool_limits
    from oracle.rows import row_values
    from oracle.solve import gtables, solve_pair
    s, pl, sub, data = _CPU_JOB
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        pairs = [sub[i] for i in idx]
        tabs = gtables(s, pl, pairs=pairs)
        xs = []
        for i, q in zip(idx, pairs):
            A = row_values(s, q, tabs.lookup)
            xs.append(solve_pair(s, q, A, *data[i])[0])
        return idx, xs, time.perf_counter() - t0


def cpu_baseline_leg(s, plan, pipes, n_pairs_sample, torch):
    """Time the FP64 oracle on a seeded sample of pairs on the host cores, one
    single-threaded process per core (forked; each builds the tables its own
    pairs need), and once more on one core alone; then state the GPU error on
    the same oracle data for those pairs."""
    global _CPU_JOB
    import multiprocessing as mp
    from edt_inputs import vhat
    from oracle.rows import plan as oplan
    from oracle.solve import gtables, forward, noise_scale, add_noise
    cores = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()))
    rows = E_pair_rows(s)
    rng = np.random.default_rng(1234)
    nonempty = np.nonzero(rows > 0)[0]
    pick = sorted(rng.choice(nonempty, size=min(n_pairs_sample, nonempty.size), replace=False).tolist())
    pl = oplan(s, only=pick)
    sub = pl.pairs
    # data of the sampled pairs: oracle forward map plus the counter-based
    # noise, scaled by the sample's largest datum per frequency (an input)
    tabs0 = gtables(s, pl)
    clean = forward(s, pl, vhat(s), tabs0)
    data = add_noise(s, pl, clean, noise_scale(s, pl, clean))
    del tabs0, clean
    # chunks of about equal Gram work per core (longest first)
    cost = np.array([q.n_rows for q in sub], np.float64)
    chunks = [[] for _ in range(cores)]
    load = np.zeros(cores)
    for i in np.argsort(-cost, kind="stable"):
        c = int(np.argmin(load))
        chunks[c].append(int(i))
        load[c] += cost[i]
    chunks = [c for c in chunks if c]
    _CPU_JOB = (s, pl, sub, data)
    xs = [None] * len(sub)
    with mp.get_context("fork").Pool(len(chunks)) as pool:
        pool.map(len, [[0]] * len(chunks))          # workers started before the clock
        t0 = time.perf_counter()
        for idx, xx, _ in pool.imap_unordered(_oracle_chunk, chunks):
            for i, x in zip(idx, xx):
                xs[i] = x
        dt = time.perf_counter() - t0
    n_km = sum(1 if q.self_conjugate else 2 for q in sub)
    # one core alone, on the heaviest chunk
    one = chunks[0]
    _, _, dt1 = _oracle_chunk(one)
    n_km1 = sum(1 if sub[i].self_conjugate else 2 for i in one)
    _CPU_JOB = None
    # GPU on identical inputs: the oracle's data overwrite the sampled pairs
    m = plan.rowmap()
    off = m["row_off"]
    d_keep = pipes[0].d.clone()
    d_host = d_keep.cpu().numpy()
    for i, (d0, d1) in zip(pick, data):
        d_host[off[i]:off[i + 1], 0] = d0
        d_host[off[i]:off[i + 1], 1] = d1
    d_mix = torch.from_numpy(d_host).cuda()
    errs = {}
    for r in pipes:
        r.set_data(d_mix)
        r.step()
        torch.cuda.synchronize()
        v = r.v.cpu().numpy()
        r.set_data(d_keep)
        num = den = 0.0
        per = []
        norms = []
        for q, x in zip(sub, xs):
            ref = x[0] + 1j * x[1]
            e = np.linalg.norm(v[q.u] - ref) ** 2
            n = np.linalg.norm(ref) ** 2
            if not q.self_conjugate:
                e += np.linalg.norm(v[q.u_neg] - np.conj(ref)) ** 2
                n += np.linalg.norm(ref) ** 2
            num += e
            den += n
            per.append(np.sqrt(e))
            norms.append(np.sqrt(n))
        norms = np.array(norms)
        fl = 1e-3 * norms.max()
        errs[r.prec] = {"global": float(np.sqrt(num / den)),
                        "per_pair_max": float(np.max(np.array(per) / np.maximum(norms, fl))),
                        "pairs": len(sub), "largest_pair_rows": int(cost.max())}
    base = {"value": n_km / dt, "unit": "subproblems/s", "cores": len(chunks), "kind": "oracle",
            "sample": f"{len(sub)} of {plan.n_pairs} +-k_m pairs ({n_km} k_m, seeded), FP64 NumPy/SciPy "
                      f"(G0 tables, Born rows, Re(A^H A), Cholesky), one single-threaded process per core over "
                      f"pairs: {dt:.1f} s wall",
            "single_core": {"value": n_km1 / dt1, "unit": "subproblems/s",
                            "sample": f"{len(one)} pairs ({n_km1} k_m) on one core: {dt1:.1f} s"},
            "host_cpus": os.cpu_count()}
    return base, errs


def E_pair_rows(s):
    import paper_0905_0238_amd as E
    return E.pair_rows(s)


def stream_main(a, s, torch, E, CONFIG_NAMES):
    """Pair-range batches of one survey on one GPU: plans built on host threads
    (not timed), data synthesised per batch on the GPU and kept resident, then
    each pass (green once, assemble -> solve per batch) captured in one HIP
    graph and replayed."""
    extra = [m for m in a.also.split(",") if m and m != a.mixed] if a.only == "both" else []
    precs = {"both": ["fp64"] + extra + [a.mixed], "mixed": [a.mixed], "fp64": ["fp64"]}[a.only]
    from edt_inputs import vhat
    t0 = time.perf_counter()
    data = a.data or ("c64" if a.config == 5 else "c128")
    budget = int(a.hbm_budget if a.hbm_budget is not None else (200e9 if a.config == 5 else 0))
    st = E.Stream(s, prec=precs[-1], also=precs[:-1], refine_tol=a.refine_tol, max_refine=a.max_refine,
                  batch_rows=a.batch_rows, batch_pairs=a.batch_pairs, chunk_rows=a.chunk, gram_band=a.band,
                  threads=16, data=data, hbm_budget=budget)
    plan_s = time.perf_counter() - t0
    print(f"# {len(st.batches)} batches planned in {plan_s:.1f} s", file=sys.stderr, flush=True)
    # synthetic data: Born forward map of the seeded model on the GPU plus
    # complex Gaussian noise of 5% of the batch's largest datum (torch RNG)
    t0 = time.perf_counter()
    st.plans[0].green(st.vel, want32=False, out=(st.G64, None))
    vh = torch.from_numpy(vhat(s)).cuda()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(int(s.seed))
    for b, p in enumerate(st.plans):
        if p.n_rows == 0:
            st.set_data(b, torch.zeros(0, 2, dtype=p.data_dtype))
            continue
        d = p.forward(st.G64, vh)
        if s.noise_rel:
            rdt = torch.float32 if d.dtype == torch.complex64 else torch.float64
            sc = s.noise_rel * float(d.abs().amax()) / np.sqrt(2.0)
            re = torch.randn(d.shape, generator=gen, device="cuda", dtype=rdt)
            im = torch.randn(d.shape, generator=gen, device="cuda", dtype=rdt)
            d += sc * torch.complex(re, im)
            del re, im
        st.set_data(b, d)
        del d
    del vh
    torch.cuda.synchronize()
    synth_s = time.perf_counter() - t0
    res = {}
    for pr in precs:
        st.capture(pr, warmup=max(1, a.warmup))
        for _ in range(a.warmup):
            st.replay(pr)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(a.steps):
            st.replay(pr)
        e1.record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / a.steps
        ms = e0.elapsed_time(e1) / a.steps
        # per-kernel times: one eager pass with every batch plan's timer on
        for p in st.plans:
            p.timing(True)
            p.timing_read()
        st.step(pr)
        torch.cuda.synchronize()
        kt = {}
        for p in st.plans:
            for k, (t, n) in p.timing_read().items():
                acc = kt.setdefault(k, [0.0, 0])
                acc[0] += t
                acc[1] += n
            p.timing(False)
        steps = st.steps.cpu().numpy()
        info = st.info.cpu().numpy()
        res[pr] = {"ms_per_step": ms, "wall_ms_per_step": wall,
                   "kernels": {k: {"ms_per_step": t, "launches_per_step": n, "avg_ms": t / max(n, 1)}
                               for k, (t, n) in kt.items()},
                   "refine_steps": {"max": int(steps.max()), "mean": float(steps.mean())},
                   "info_nonzero": int(np.sum((info != 0) & (info != -1)))}
        st.graphs.pop(pr)
    main_prec = precs[-1]
    t_main = res[main_prec]["ms_per_step"]
    U = sum(int(p.info["n_urows"]) for p in st.plans)
    kt = res[main_prec]["kernels"]
    dom = max(kt, key=lambda k: kt[k]["ms_per_step"])
    roof = {"kernel": dom, "traffic": None}
    if dom.startswith("gram_"):
        dt = {"gram_bf16x3": "bf16", "gram_fp16x3": "fp16", "gram_fp32": "fp32", "gram_fp64": "fp64"}[dom]
        fl = 2.0 * U * s.nz * (s.nz + 1)
        ach = fl / (kt[dom]["ms_per_step"] * 1e-3) / 1e12
        roof.update({"bound": "mfma", "achieved": ach, "peak": PEAK[dt], "unit": "TFLOP/s",
                     "frac": ach / PEAK[dt],
                     "per_launch": f"2 U nz (nz+1) over the batches' launches (U = {U} unique rows)"})
    elif dom == "refine residual":
        per_pair = np.concatenate([np.diff(p.urows()["urow_off"]) for p in st.plans]).astype(np.float64)
        fl = 22.0 * s.nz * float(np.sum(per_pair * st.steps.cpu().numpy()))
        ach = fl / (kt[dom]["ms_per_step"] * 1e-3) / 1e12
        roof.update({"bound": "alu", "achieved": ach, "peak": PEAK["fp64"], "unit": "TFLOP/s",
                     "frac": ach / PEAK["fp64"], "per_launch": "22 nz per unique row of the pairs still iterating"})
    out = {
        "metric": METRIC, "value": st.n_km / (t_main * 1e-3), "unit": "subproblems/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": t_main, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"bf16x3": "bf16x3+f64", "fp16x3": "f16x3+f64", "fp32": "f32+f64"}.get(main_prec, "f64"),
        "data": "synthetic",
        "config": {"workload": CONFIG_NAMES[a.config], "n_km": st.n_km, "n_pairs": st.n_pairs, "nz": s.nz,
                   "n_freq": s.n_freq, "rows": int(st.rows.sum()), "unique_rows": U, "precision": main_prec,
                   "refine_tol": a.refine_tol, "max_refine": a.max_refine, "batches": len(st.batches),
                   "batch_rows": a.batch_rows, "batch_pairs": a.batch_pairs, "data_rows": data,
                   "hbm_budget": budget},
        "roofline": roof,
    }
    if "fp64" in res and main_prec != "fp64":
        out["fp64_plain"] = {"value": st.n_km / (res["fp64"]["ms_per_step"] * 1e-3),
                             "ms_per_step": res["fp64"]["ms_per_step"]}
        out["speedup_vs_fp64"] = res["fp64"]["ms_per_step"] / t_main
    out["detail"] = res
    out["detail"]["plan_s"] = plan_s
    out["detail"]["synth_s"] = synth_s
    out["detail"]["resident_bytes"] = st.resident_bytes()
    out["detail"]["hbm_peak_allocated"] = int(torch.cuda.max_memory_allocated())
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {a.gpus} is not supported "
              "(the +-k_m pairs are independent problems: a multi-GPU run would give each GPU "
              "its own pair range, with no exchange)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if a.copy_calibration:
        return copy_calibration(torch)
    if a.lines_only:
        print(json.dumps({"lines": lines_leg(max(1, a.steps), torch)}), flush=True)
        return None
    import paper_0905_0238_amd as E
    from edt_inputs import make_config, CONFIG_NAMES
    s = make_config(a.config)
    if a.stream or a.config == 5:
        return stream_main(a, s, torch, E, CONFIG_NAMES)
    extra = [m for m in a.also.split(",") if m and m != a.mixed] if a.only == "both" else []
    precs = {"both": ["fp64"] + extra + [a.mixed], "mixed": [a.mixed], "fp64": ["fp64"]}[a.only]
    vel = torch.tensor(s.vel, dtype=torch.float64, device="cuda")
    from paper_0905_0238_amd.tune import autotune, shapes_for, DEFAULT_SHAPE
    shapes, tuned, source = {}, {}, {}
    for pr in precs:
        if a.tune:
            tuned[pr] = autotune(s, prec=pr, refine_tol=a.refine_tol, max_refine=a.max_refine,
                                 log=lambda r: print("# tune", json.dumps(r), file=sys.stderr, flush=True))
            shapes[pr] = {k: tuned[pr][k] for k in DEFAULT_SHAPE}
            source[pr] = "tuned now"
        elif a.chunk or a.band or a.default_shapes:
            shapes[pr] = {"chunk_rows": a.chunk, "gram_band": a.band, "resid_group": 0}
            source[pr] = "command line" if (a.chunk or a.band) else "planner default"
        else:
            shapes[pr] = shapes_for(s, pr)
            source[pr] = "tuned-shape table" if shapes[pr] != DEFAULT_SHAPE else "planner default (not in table)"
    t0 = time.perf_counter()
    plans = {}
    for pr in precs:
        opts = tuple(shapes[pr][k] for k in ("chunk_rows", "gram_band", "resid_group"))
        if opts not in plans:
            plans[opts] = E.Plan(s, chunk_rows=opts[0], gram_band=opts[1], resid_group=opts[2]).upload()
        plans[pr] = plans[opts]
    plan_s = time.perf_counter() - t0
    plan = plans[precs[-1]]
    d = synth_inputs(s, plan, vel, torch)
    torch.cuda.synchronize()
    pipes = [E.Pipeline(plans[pr], vel, d, s.lambda_rel, pr, a.refine_tol, a.max_refine) for pr in precs]
    res = {}
    for pipe in pipes:
        ms, wall, eager_ms = time_steps(pipe, a.steps, a.warmup, torch)
        kt = kernel_times(pipe, max(2, min(a.steps, 5)), torch)
        st = pipe.steps.cpu().numpy()
        info = pipe.info.cpu().numpy()
        res[pipe.prec] = {"ms_per_step": ms, "wall_ms_per_step": wall, "eager_ms_per_step": eager_ms,
                          "kernels": kt, "_steps": st,
                          "refine_steps": {"max": int(st.max()), "mean": float(st.mean())},
                          "info_nonzero": int(np.sum((info != 0) & (info != -1))),
                          "items": {"chunk_rows": pipe.p.info["chunk_rows"], "gram_band": pipe.p.info["gram_band"],
                                    "resid_group": pipe.p.info["resid_group"], "n_items": pipe.p.info["n_items"],
                                    "shape_source": source[pipe.prec]}}
        if pipe.prec in tuned:
            res[pipe.prec]["tuner"] = tuned[pipe.prec]["table"]
    main_prec = precs[-1]
    t_main = res[main_prec]["ms_per_step"]
    value = plan.n_km / (t_main * 1e-3)
    dom, roof = roofline(plans[main_prec], s, res[main_prec]["kernels"], main_prec, res[main_prec]["_steps"])
    for pr, v in res.items():
        v.pop("_steps")
        v["gram_mfma"] = gram_mfma(plans[pr], s, v["kernels"])
    roof["kernel"] = dom
    mp = plans[main_prec]
    roof["traffic"] = measured_traffic(dom, CONFIG_NAMES[a.config], main_prec,
                                       {k: int(mp.info[k]) for k in ("chunk_rows", "gram_band", "resid_group")})
    if roof["traffic"] is not None:
        roof["traffic_unit"] = "HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)"
    out = {
        "metric": METRIC, "value": value, "unit": "subproblems/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": t_main, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16x3": "bf16x3+f64", "fp16x3": "f16x3+f64", "fp32": "f32+f64"}.get(main_prec, "f64"),
        "data": "synthetic",
        "config": {"workload": CONFIG_NAMES[a.config], "n_km": plan.n_km, "n_pairs": plan.n_pairs,
                   "nz": s.nz, "n_freq": s.n_freq, "rows": plan.n_rows, "unique_rows": plan.info["n_urows"],
                   "precision": main_prec, "refine_tol": a.refine_tol, "max_refine": a.max_refine,
                   "chunk_rows": plan.info["chunk_rows"], "gram_band": plan.info["gram_band"],
                   "resid_group": plan.info["resid_group"], "shapes": source[main_prec]},
        "roofline": roof,
    }
    if "fp64" in res and main_prec != "fp64":
        out["fp64_plain"] = {"value": plan.n_km / (res["fp64"]["ms_per_step"] * 1e-3),
                             "ms_per_step": res["fp64"]["ms_per_step"]}
        out["speedup_vs_fp64"] = res["fp64"]["ms_per_step"] / t_main
    out["detail"] = {k: {kk: vv for kk, vv in v.items()} for k, v in res.items()}
    out["detail"]["plan_s"] = plan_s
    if a.tsvd > 0 and "fp64" in plans:
        out["detail"]["tsvd"] = tsvd_leg(plans["fp64"], vel, d, a.tsvd, 3, torch)
    if "fp64" in plans:
        al = aperture_leg(plans["fp64"], vel, s.d_mid, 2, torch)
        if al is not None:
            out["detail"]["aperture"] = al
        sl = shots_leg(plans["fp64"], 3, torch)
        if sl is not None:
            out["detail"]["shots"] = sl
        out["detail"]["lines"] = lines_leg(2, torch)
    if not a.no_cpu:
        n_cpu = a.cpu_pairs or (512 if s.dim == 3 else 160)
        base, errs = cpu_baseline_leg(s, plan, pipes, n_cpu, torch)
        out["cpu_baseline"] = base
        out["rel_err_vs_oracle"] = errs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
