"""Benchmark: DGP field solve inside a PM step on one MI355X.

Workload (the configuration the headline metric is quoted on): a 256^3 periodic
mesh, box 512 Mpc/h, with a 256^3-particle Zel'dovich load (seeded Gaussian
field, P(k) ~ k^-1.5 exp(-k^2/k_c^2), k_c = 1 h/Mpc, rms displacement 2 Mpc/h),
z = 1 (a = 0.5), Omega_m0 = 0.27, w = 1/3.  One step = CIC deposit -> field solve
from the linear guess to normalised residual 1e-8 -> modified-Poisson forces ->
CIC interpolation + leapfrog kick-drift.  Inputs are resident on the GPU before
the timed region; particles advance from step to step.  Particles are stored in
Lagrangian blocks of 8^3 (a spatially coherent order, as a PM code keeps them).

Other modes:
  --probe                 a short run for hardware-counter passes (two precision-form
                          steps plus a plain 512 MiB device copy for calibration);
                          with --stages: the same at 512^3 (one precision-form step)
  --pmc-summary F W       turn the counter CSVs of two such passes (FETCH_SIZE, then
                          WRITE_SIZE) into the traffic summary kept under profiles/
  --trace-summary T       per-kernel duration table of a rocprofv3 kernel trace
  --stages                per-stage times of a PM step on a 512^3 mesh with 512^3 float32
                          particles (box 1024 Mpc/h), precision form and plain float64 form;
                          with --cpu also the CPU oracle on that step (sampled, extrapolated)
  --wscan                 the w-scan of Fig. 3 at the paper's size (z = 24, box 64 Mpc/h,
                          256^3 mesh, 128^3 particles): residual and bad fraction per pass
  --adjoint               the implicit adjoint of 8 batched 128^3 log-normal fields (float64,
                          backward to 1e-12): time per backward and per iteration

The solve runs in the precision form (float32 FFTs and pointwise storage,
float64 residual / discriminant / root / reductions, float64 polish); the plain
float64 form is timed on the same load for the FP32-vs-FP64 comparison.

value = field-solve cells*iterations per second over whole PM steps:
N^3 x (relaxation passes executed) / (step wall time).  One JSON line on stdout.
"""
import argparse
import csv
import glob
import hashlib
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

N, BOX, SEED, A, OM0 = 256, 512.0, 3, 0.5, 0.27
TOL = 1e-8
RNL = 1.78          # nonlinear ratio lambda max|u_lin| / alpha: screened, and below the value (~3) at which
                    # the deepest voids of a one-particle-per-cell load leave the discrete equation without a root
DLNA = 0.005
PEAK_HBM = 8.0e12   # bytes/s, MI355X
BLOCK = 8           # particles stored in Lagrangian blocks of BLOCK^3
BREAKDOWN_STEPS = 3
COPY_BYTES = 512 * 1024 * 1024   # calibration copy of the probe: reads and writes this many bytes
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_pm_step_256.md")
# timing class of the library -> device kernel names (prefixes) it launches
CLASS_KERNELS = {
    "relax_fp32": ("dgp::k_relax<float, 256>", "dgp::k_relax_w<float, 256>"),
    "relax": ("dgp::k_relax<double, 256>", "dgp::k_relax_w<double, 256>"),
    "deposit": ("dgp::k_deposit_bin<double>", "dgp::k_deposit<double>"),
}


def kernel_source_digest():
    """sha256 over the device sources: counter figures are valid only for the code they measured."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_0906_4548_amd", "csrc", "*"))):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(os.path.basename(f).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def kernel_name(sig):
    """'void dgp::k<T, 256>(args...)' -> 'dgp::k<T, 256>'."""
    sig = sig.strip()
    if sig.startswith("void "):
        sig = sig[5:]
    if sig.endswith(")"):
        depth = 0
        for i in range(len(sig) - 1, -1, -1):
            depth += {")": 1, "(": -1}.get(sig[i], 0)
            if depth == 0:
                return sig[:i]
    return sig


def read_counters(path):
    """rocprofv3 counter_collection CSV -> {kernel name: [values in bytes per dispatch]}."""
    out = {}
    with open(path, newline="") as fh:
        for row in csv.DictReader(fh):
            name = kernel_name(row.get("Kernel_Name") or row.get("Kernel-Name") or "")
            val = float(row.get("Counter_Value") or row.get("Counter-Value") or 0.0)
            out.setdefault(name, []).append(val * 1024.0)   # FETCH_SIZE / WRITE_SIZE count KiB
    return out


def pmc_summary(fetch_csv, write_csv, mesh=256):
    """Markdown summary of HBM traffic per dispatch, calibrated on the probe's plain copy."""
    fetch, write = read_counters(fetch_csv), read_counters(write_csv)
    copy = [k for k in fetch if "copy" in k.lower() or "elementwise" in k.lower()]
    big = [k for k in copy if max(fetch[k]) > 0.25 * COPY_BYTES]
    if not big:
        raise SystemExit("no calibration copy kernel found in %s" % fetch_csv)
    ck = big[0]
    f_scale = COPY_BYTES / max(fetch[ck])
    w_scale = COPY_BYTES / max(write.get(ck, [COPY_BYTES]))
    def working(vals):
        # dispatches that did their work: launches after an element has stopped exit at once
        top = max(vals)
        return [v for v in vals if v >= 0.05 * top] if top > 0 else vals

    rows, table = {}, []
    for name in sorted(fetch):
        if not name.startswith("dgp::"):
            continue
        fv = working(fetch[name])
        f = sum(fv) / len(fv) * f_scale
        wv = working(write[name]) if name in write else None
        w = sum(wv) / len(wv) * w_scale if wv else None
        rows[name] = {"fetch_bytes": f, "write_bytes": w, "dispatches": len(fetch[name]), "working": len(fv)}
        table.append("| `%s` | %d | %d | %.1f | %s |" % (name, len(fetch[name]), len(fv), f / 2 ** 20,
                                                         "%.1f" % (w / 2 ** 20) if w is not None else "-"))
    probe = "--probe" if mesh == 256 else "--stages --probe"
    lines = [
        "# HBM traffic per dispatch: PM step at %d^3 (FETCH_SIZE / WRITE_SIZE, calibrated)" % mesh,
        "",
        "Commands (repository root `$R`, any output directory `$OUT`, one MI355X; one counter per pass):",
        "",
        "    cd /tmp && rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/pmc_fetch -o run -- "
        "python3 $R/bench.py %s" % probe,
        "    cd /tmp && rocprofv3 --pmc WRITE_SIZE --output-format csv -d $OUT/pmc_write -o run -- "
        "python3 $R/bench.py %s" % probe,
        "    python3 bench.py --pmc-summary <pmc_fetch>/run_counter_collection.csv "
        "<pmc_write>/run_counter_collection.csv%s" % ("" if mesh == 256 else " --pmc-mesh %d" % mesh),
        "",
        "Calibration: the probe's plain copy `%s` moves %d MiB each way; its raw counters read "
        "%.1f MiB fetched and %.1f MiB written, so fetch values are scaled by %.3f and write values by %.3f."
        % (ck, COPY_BYTES // 2 ** 20, max(fetch[ck]) / 2 ** 20, max(write.get(ck, [0.0])) / 2 ** 20, f_scale, w_scale),
        "",
        "Per-dispatch figures average the dispatches that did their work (those above 5 % of the",
        "kernel's largest; relaxation launches after convergence exit at once).",
        "",
        "| kernel | dispatches | working | fetch MiB/dispatch | write MiB/dispatch |",
        "|---|---:|---:|---:|---:|",
    ] + table + [
        "",
        "Machine-readable copy (bench.py reports `roofline.traffic` from it while the device sources "
        "still hash to `source_sha256`):",
        "",
        "```json",
        json.dumps({"source_sha256": kernel_source_digest(), "kernels": rows}, indent=1),
        "```",
        "",
    ]
    return "\n".join(lines)


def trace_summary(trace_csv, stats_csv=None):
    """Markdown table of per-kernel durations from a rocprofv3 kernel trace; besides the
    statistics over every dispatch it gives the average over working dispatches (those
    above 5 % of the kernel's longest: relaxation launches after convergence exit at once)."""
    durs = {}
    with open(trace_csv, newline="") as fh:
        for row in csv.DictReader(fh):
            name = kernel_name(row["Kernel_Name"])
            durs.setdefault(name, []).append((int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) * 1e-3)
    total = sum(sum(v) for v in durs.values())
    lines = ["| kernel | calls | avg us | working | working avg us | min us | max us | total ms | % |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for name, v in sorted(durs.items(), key=lambda kv: -sum(kv[1])):
        top = max(v)
        w = [x for x in v if x >= 0.05 * top]
        lines.append("| `%s` | %d | %.1f | %d | %.1f | %.1f | %.1f | %.2f | %.1f |" % (
            name, len(v), sum(v) / len(v), len(w), sum(w) / len(w), min(v), top, sum(v) * 1e-3,
            100.0 * sum(v) / total))
    return "\n".join(lines)


def stored_traffic(cls):
    """Calibrated HBM bytes per dispatch of the kernel behind timing class `cls`, or None when
    no summary exists or the device sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            text = fh.read()
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("source_sha256") != kernel_source_digest():
        return None
    for name in CLASS_KERNELS.get(cls, ()):
        k = blob["kernels"].get(name)
        if k and k.get("write_bytes") is not None:
            return k["fetch_bytes"] + k["write_bytes"]
    return None


def algorithmic_bytes(cls, n, elem):
    """Bytes one launch of a relaxation-pass kernel must move (one batch element)."""
    hs = (n // 2 + 1) * n * n
    n3 = n ** 3
    c = 2 * elem
    return {
        "axis1_fwd": 2 * hs * c,                 # read + write one half spectrum
        "fanout": 4 * hs * c,                    # read 1, write 3 spectra (1/|n|^2 and axis-2 factors)
        "axis1_inv": 9 * hs * c,                 # read 3, write 6 spectra (axis-1 and axis-0 factors)
        "relax": 7 * hs * c + 3 * n3 * elem,     # read 6 spectra, u, S; write u, 1 spectrum
    }.get(cls)


def stages_512(args, torch, dgp, inputs, dev):
    """One JSON line: per-stage milliseconds per PM step at 512^3 (512^3 float32 particles in
    Lagrangian 8^3 blocks, box 1024 Mpc/h, seed 4) for the precision form and the float64 form,
    from the plan's HIP-event timing of every kernel class."""
    n, box, seed, steps = 512, 1024.0, 4, max(1, min(args.steps, 3))
    print("bench: building the 512^3 load", file=sys.stderr, flush=True)
    pos_h, psi_h = inputs.zeldovich_load(n, box, seed, dtype=np.float32, block=BLOCK)
    npart = pos_h.shape[1]
    pos0 = torch.from_numpy(pos_h).to(dev)
    prm0 = dgp.params(OM0, A)
    growth = A * A * prm0.E * ((prm0.eta - 1.0) / prm0.eta) ** 0.55
    vel0 = torch.from_numpy((growth * psi_h).astype(np.float32)).to(dev)
    sub = CPU512_SUB
    cpu_pos, cpu_vel = (pos_h[:, ::sub].copy(), (growth * psi_h[:, ::sub]).astype(np.float32)) if args.cpu else (None, None)
    del pos_h, psi_h
    with dgp.Plan(n, box) as p64:
        delta = torch.zeros(n ** 3, dtype=torch.float64, device=dev)
        p64.deposit(pos0, None, delta)
        ulin = torch.zeros_like(delta)
        p64.solve_field(dgp.params(OM0, A, tol=0.0, max_iter=0), delta, ulin)
        lam = RNL * prm0.alpha / float(ulin.abs().max())
    del delta, ulin
    torch.cuda.empty_cache()
    if args.probe:   # counter pass at 512^3: calibration copy, one warm-up and one timed precision-form step
        x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
        plan = dgp.Plan(n, box, precision=dgp.FP32)
        prm = dgp.params(OM0, A, lam=lam, tol=TOL, max_iter=200, init=dgp.INIT_LINEAR, check_every=8)
        u = torch.zeros(n ** 3, dtype=torch.float64, device=dev)
        for _ in range(2):
            plan.step(prm, pos0, vel0, u, DLNA)
        torch.cuda.synchronize()
        plan.close()
        print("probe done", file=sys.stderr, flush=True)
        return
    out = {"mode": "stages", "config": {"workload": "Zel'dovich PM step, 512^3 mesh, 512^3 float32 particles, "
                                                    "box 1024 Mpc/h, z=1, r_nl=%.2f, tol 1e-8" % RNL,
                                        "mesh": n, "particles": npart, "lambda": lam, "steps": steps}}
    for name, precision in (("precision_form", dgp.FP32), ("fp64_form", dgp.FP64)):
        print("bench: stages of the %s" % name, file=sys.stderr, flush=True)
        plan = dgp.Plan(n, box, precision=precision)
        prm = dgp.params(OM0, A, lam=lam, tol=TOL, max_iter=200, init=dgp.INIT_LINEAR, check_every=8)
        pos, vel = pos0.clone(), vel0.clone()
        u = torch.zeros(n ** 3, dtype=torch.float64, device=dev)
        plan.step(prm, pos, vel, u, DLNA)
        torch.cuda.synchronize()
        plan.timing(True)
        t0 = time.perf_counter()
        infos = [plan.step(prm, pos, vel, u, DLNA) for _ in range(steps)]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tim = plan.timing_read()
        plan.timing(False)
        plan.close()
        del pos, vel, u
        torch.cuda.empty_cache()
        out[name] = {
            "ms_per_step": 1e3 * dt / steps,
            "passes_per_step": sum(i["passes"] for _, i in infos) / steps,
            "passes_fp64_per_step": sum(i["passes_fp64"] for _, i in infos) / steps,
            "resid": [i["resid"] for _, i in infos],
            "status": [st for st, _ in infos],
            "stage_ms_per_step": {k: v[0] / steps for k, v in tim.items()},
            "stage_launches_per_step": {k: v[1] / steps for k, v in tim.items()},
        }
    if args.cpu:
        print("bench: the oracle at 512^3 on the host", file=sys.stderr, flush=True)
        out["cpu_oracle"] = oracle_512(cpu_pos, cpu_vel, lam, n, box, npart, out["fp64_form"]["passes_per_step"])
    print(json.dumps(out))


CPU512_SUB = 8   # the oracle's particle stages at 512^3 run on every 8th particle and are scaled by 8


def oracle_512(pos_s, vel_s, lam, n, box, npart, passes):
    """The CPU oracle on the 512^3 step, timed on the host and extrapolated linearly: the deposit,
    interpolation and kick-drift on every CPU512_SUB-th particle (times scaled by CPU512_SUB), the
    solve's set-up plus one residual evaluation and one further pass (update + evaluation) on the
    subsample's delta (scaled to `passes` passes), and the force mesh; one thread and all cores."""
    from oracle import field as fld, pm, spectral
    sub = CPU512_SUB
    prm = fld.SolveParams.from_cosmology(OM0, A, lam=lam, tol=TOL, max_iter=200)

    def say(msg):
        print("bench: oracle 512^3 " + msg, file=sys.stderr, flush=True)

    def leg():
        t = {}
        t0 = time.perf_counter()
        _, delta = pm.deposit(pos_s, n, box)
        t["deposit"] = (time.perf_counter() - t0) * sub
        say("deposit done")
        t0 = time.perf_counter()
        u, _ = fld.solve(delta, box, prm, fixed_iters=0)
        say("first evaluation done")
        t_first = time.perf_counter() - t0
        t0 = time.perf_counter()
        fld.solve(delta, box, prm, fixed_iters=1)
        t_pass = time.perf_counter() - t0 - t_first
        t["solve"] = t_first + (passes - 1) * t_pass
        say("pass done")
        t0 = time.perf_counter()
        mesh = pm.force_mesh(pm.phi_spectrum(delta, u, box, prm, OM0, A), box)
        t["force_mesh"] = time.perf_counter() - t0
        say("force mesh done")
        t0 = time.perf_counter()
        force = pm.cic_interpolate(mesh, pos_s, box)
        t["interpolation"] = (time.perf_counter() - t0) * sub
        t0 = time.perf_counter()
        pm.kick_drift(pos_s, vel_s, force, A, DLNA, OM0, box)
        t["kick_drift"] = (time.perf_counter() - t0) * sub
        return t, t_first, t_pass

    cores = os.cpu_count() or 1
    t1, f1, p1 = leg()
    with spectral.fft_workers(cores):
        tn, fn, pn = leg()
    step1, stepn = sum(t1.values()), sum(tn.values())
    return {"unit": "cells*iter/s", "cpu_model": cpu_model(), "host_logical_cpus": cores,
            "sample": "deposit, interpolation and kick-drift on 1/%d of the %d particles (x%d); the solve's "
                      "set-up + first evaluation and one further pass timed, extrapolated to %g passes; "
                      "the force mesh once" % (sub, npart, sub, passes),
            "one_thread": {"value": n ** 3 * passes / step1, "step_seconds": step1, "stage_seconds": t1,
                           "first_evaluation_seconds": f1, "pass_seconds": p1},
            "all_cores": {"value": n ** 3 * passes / stepn, "cores": cores, "step_seconds": stepn,
                          "stage_seconds": tn, "first_evaluation_seconds": fn, "pass_seconds": pn}}


def adjoint_bench(args, torch, dgp, inputs, dev):
    """One JSON line: the implicit adjoint of the batched differentiation workload (8 seeded
    log-normal 128^3 fields, sigma 0.3/1/3, box 256 Mpc/h, lambda for a nonlinear ratio of 3),
    float64: the backward solve to 1e-12 from a converged forward solve, timed over repeats."""
    n, box, sig = 128, 256.0, [0.3, 0.3, 0.3, 1.0, 1.0, 1.0, 3.0, 3.0]
    B = len(sig)
    deltas = np.stack([inputs.lognormal_delta(n, box, s, 500 + i) for i, s in enumerate(sig)])
    d = torch.from_numpy(deltas).to(dev)
    prm0 = dgp.params(OM0, A)
    with dgp.Plan(n, box, batch=B) as plan:
        ulin = torch.zeros_like(d)
        plan.solve_field(dgp.params(OM0, A, tol=0.0, max_iter=0), d, ulin)
        lam = float(np.median([3.0 * prm0.alpha / float(ulin[b].abs().max()) for b in range(B)]))
        u = torch.zeros_like(d)
        st, _ = plan.solve_field(dgp.params(OM0, A, lam=lam, tol=1e-12, max_iter=200), d, u)
        g = torch.from_numpy(np.random.default_rng(77).standard_normal((B, n, n, n))).to(dev)
        gd = torch.zeros_like(d)
        bwd = dgp.params(OM0, A, lam=lam, tol=1e-12, max_iter=200)
        plan.solve_field_backward(bwd, d, u, g, gd)
        torch.cuda.synchronize()
        reps = max(1, min(args.steps, 10))
        t0 = time.perf_counter()
        for _ in range(reps):
            st, info = plan.solve_field_backward(bwd, d, u, g, gd)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
    iters = [i["iters"] for i in info]
    evals = [i["passes"] for i in info]
    hs, n3 = (n // 2 + 1) * n * n, n ** 3
    # algorithmic bytes of one iteration of one element: axis-1 forward of the six product
    # spectra summed into three groups (6 in, 3 out), the combine (3 in, 1 out), axis-1 inverse
    # (2 hs); the fused axis-0 step reads the combined spectrum and nine real fields (mu, u, g,
    # five Hessians), writes mu' and six spectra.  Elements stop at their own iteration counts;
    # the setup (Hessians of u*, the first products) and the final S mu transform are in the time
    # but not in these bytes.
    it_bytes = (9 + 4 + 2 + 1 + 6) * hs * 16 + (9 + 1) * n3 * 8
    total = it_bytes * sum(evals)
    out = {"mode": "adjoint", "config": {"workload": "implicit adjoint of 8 batched 128^3 log-normal fields "
                                                     "(sigma 0.3/1/3), float64, backward to 1e-12",
                                         "mesh": n, "batch": B, "lambda": lam},
           "status": st, "ms_backward": ms, "iters": iters, "evaluations": evals,
           "bytes_per_element_iteration": it_bytes, "algorithmic_GB": total * 1e-9,
           "GBps": total / ms * 1e-6, "resid": [i["resid"] for i in info]}
    print(json.dumps(out))


def wscan(args, torch, dgp, inputs, dev):
    """One JSON line: the convergence histories of Fig. 3 (Sec. III C) at the paper's size.  A seeded
    Zel'dovich load of 128^3 particles (P ~ k^-1.5 exp(-k^2/k_c^2), k_c = 4 h/Mpc, rms displacement
    0.15 Mpc/h) deposited on a 256^3 mesh of a 64 Mpc/h box, z = 24, lam = 1 (the paper's
    equation); for each w the solve starts from the same linear solution and runs 40 updates
    (float64), recording the normalised residual of every evaluated iterate and the bad fraction
    of every update."""
    n, box, nside, k = 256, 64.0, 128, 40
    print("bench: building the z = 24 load", file=sys.stderr, flush=True)
    pos, _ = inputs.zeldovich_load(nside, box, 24, slope=-1.5, kc=4.0, rms_disp=0.15)
    out = {"mode": "wscan", "config": {"workload": "Fig. 3 w-scan: Zel'dovich load 128^3 particles on a 256^3 mesh, "
                                                   "box 64 Mpc/h, z=24, lam=1, 40 updates from the linear solution",
                                       "mesh": n, "particles": nside ** 3, "updates": k}, "runs": {}}
    with dgp.Plan(n, box) as plan:
        delta = torch.zeros(n ** 3, dtype=torch.float64, device=dev)
        plan.deposit(torch.from_numpy(pos).to(dev), None, delta)
        out["config"]["delta_min"] = float(delta.min())
        out["config"]["delta_rms"] = float(delta.std())
        for w in (0.0, 0.25, 1.0 / 3.0, 0.5, 0.8):
            u = torch.zeros_like(delta)
            st, info = plan.solve_field(dgp.params(OM0, 1.0 / 25.0, lam=1.0, w=w, tol=-1.0, max_iter=k), delta, u)
            hist, bad = plan.history(cap=k + 1)
            out["runs"]["%.4f" % w] = {"status": st, "resid": hist.tolist(), "bad_fraction": bad[:k].tolist(),
                                       "ms": info[0]["ms_total"]}
    print(json.dumps(out))


def fft_comparison(torch, dgp, dev, n=N, reps=10):
    """The library's 3D real transform (three axis passes, float64) against torch.fft (rocFFT) on
    the same 256^3 field: milliseconds per forward (R2C) and inverse (C2R) transform, HIP events
    on the current stream, after a warm-up call of each."""
    x = torch.randn(n, n, n, dtype=torch.float64, device=dev)
    spec = torch.zeros((n // 2 + 1, n, n), dtype=torch.complex128, device=dev)
    back = torch.zeros_like(x)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    with dgp.Plan(n, BOX) as plan:
        ours_f = timed(lambda: plan.fft_forward(x, spec))
        ours_i = timed(lambda: plan.fft_inverse(spec, back))
    tk = {}
    tk["r2c"] = timed(lambda: torch.fft.rfftn(x))
    xk = torch.fft.rfftn(x)
    tk["c2r"] = timed(lambda: torch.fft.irfftn(xk, s=(n, n, n)))
    x32 = x.float()
    tk["r2c_fp32"] = timed(lambda: torch.fft.rfftn(x32))
    xk32 = torch.fft.rfftn(x32)
    tk["c2r_fp32"] = timed(lambda: torch.fft.irfftn(xk32, s=(n, n, n)))
    del x, spec, back, xk, x32, xk32
    torch.cuda.empty_cache()
    return {"mesh": n, "dgp_fp64_forward_ms": ours_f, "dgp_fp64_inverse_ms": ours_i,
            "torch_fft_fp64_r2c_ms": tk["r2c"], "torch_fft_fp64_c2r_ms": tk["c2r"],
            "torch_fft_fp32_r2c_ms": tk["r2c_fp32"], "torch_fft_fp32_c2r_ms": tk["c2r_fp32"],
            "note": "dgp forward includes writing the spectrum in the plan's layout (half axis first); "
                    "torch.fft dispatches to rocFFT"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline leg")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain float64 comparison")
    ap.add_argument("--probe", action="store_true", help="short run for hardware-counter passes")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the calibrated traffic summary from two counter passes to stdout")
    ap.add_argument("--pmc-mesh", type=int, default=256, help="mesh size the counter passes ran at")
    ap.add_argument("--stages", action="store_true",
                    help="per-stage times of a 512^3 PM step with 512^3 float32 particles, both forms")
    ap.add_argument("--cpu", action="store_true",
                    help="with --stages: also time the CPU oracle on the 512^3 step (sampled, extrapolated)")
    ap.add_argument("--wscan", action="store_true", help="the w-scan of Fig. 3 at the paper's size")
    ap.add_argument("--adjoint", action="store_true",
                    help="time the implicit adjoint of the batched 8 x 128^3 differentiation workload")
    ap.add_argument("--trace-summary", metavar="KERNEL_TRACE_CSV",
                    help="write a per-kernel duration table from a rocprofv3 kernel trace to stdout")
    args = ap.parse_args()
    if args.pmc_summary:
        print(pmc_summary(*args.pmc_summary, mesh=args.pmc_mesh))
        return
    if args.trace_summary:
        print(trace_summary(args.trace_summary))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the field solve runs on a single MI355X "
              "(slab sharding over several GPUs is described, not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0906_4548_amd import dgp, inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.stages:
        stages_512(args, torch, dgp, inputs, dev)
        return
    if args.wscan:
        wscan(args, torch, dgp, inputs, dev)
        return
    if args.adjoint:
        adjoint_bench(args, torch, dgp, inputs, dev)
        return
    print("bench: building inputs", file=sys.stderr, flush=True)
    pos_h, psi_h = inputs.zeldovich_load(N, BOX, SEED, block=BLOCK)
    npart = pos_h.shape[1]
    pos0 = torch.from_numpy(pos_h).to(dev)
    prm0 = dgp.params(OM0, A)
    growth = A * A * prm0.E * ((prm0.eta - 1.0) / prm0.eta) ** 0.55
    vel0 = torch.from_numpy(growth * psi_h).to(dev)

    # nonlinear coefficient: lambda = RNL alpha / max|u_lin|, u_lin from the library (zero updates)
    with dgp.Plan(N, BOX) as p64:
        delta = torch.zeros(N ** 3, dtype=torch.float64, device=dev)
        p64.deposit(pos0, None, delta)
        ulin = torch.zeros_like(delta)
        p64.solve_field(dgp.params(OM0, A, tol=0.0, max_iter=0), delta, ulin)
        lam = RNL * prm0.alpha / float(ulin.abs().max())
    del delta, ulin

    def run_form(precision, steps, warmup, classes=None):
        """Run warmup + timed steps; `classes` restricts the event timing (None: every class)."""
        plan = dgp.Plan(N, BOX, precision=precision)
        prm = dgp.params(OM0, A, lam=lam, tol=TOL, max_iter=200, init=dgp.INIT_LINEAR, check_every=8)
        pos = pos0.clone()
        vel = vel0.clone()
        u = torch.zeros(N ** 3, dtype=torch.float64, device=dev)
        for _ in range(warmup):
            plan.step(prm, pos, vel, u, DLNA)
        torch.cuda.synchronize()
        plan.timing(True)
        plan.timing_classes(classes)
        infos = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            st, info = plan.step(prm, pos, vel, u, DLNA)
            infos.append((st, info))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tim = plan.timing_read()
        plan.timing(False)
        plan.close()
        return dt, infos, tim

    if args.probe:
        x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
        run_form(dgp.FP32, 2, 0)
        torch.cuda.synchronize()
        print("probe done", file=sys.stderr, flush=True)
        return

    def table(tim):
        return {k: {"ms_total": v[0], "launches": v[1], "ms_avg": v[0] / v[1]} for k, v in tim.items()}

    # Per-class breakdown on a short run with every class timed (two event records per launch).
    # The timed run that gives `value` then carries events on the dominant class only.
    print("bench: kernel breakdown", file=sys.stderr, flush=True)
    _, infos_all, tim_all = run_form(dgp.FP32, BREAKDOWN_STEPS, 1)
    dom = max((k for k in tim_all if (k[:-5] if k.endswith("_fp32") else k) in
               ("axis1_fwd", "fanout", "axis1_inv", "relax")), key=lambda k: tim_all[k][0])
    print("bench: timing precision form", file=sys.stderr, flush=True)
    dt32, infos32, tim32 = run_form(dgp.FP32, args.steps, args.warmup, [dom])
    passes32 = sum(i["passes"] for _, i in infos32)
    value = N ** 3 * passes32 / dt32
    res = {
        "metric": "field-solve cells*iter/s (PM step, 256^3, residual 1e-8, FP32+FP64-polish)",
        "value": value,
        "unit": "cells*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt32 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 FFT + f64 pointwise/polish",
        "data": "synthetic (seeded Zel'dovich load)",
        "config": {"workload": "Zel'dovich PM step, 256^3 mesh, 256^3 particles, box 512 Mpc/h, z=1, "
                               "r_nl=%.2f, w=1/3, tol 1e-8 from the linear guess" % RNL,
                   "mesh": N, "particles": npart, "lambda": lam, "tol": TOL},
        "solve": {
            "status": [s for s, _ in infos32],
            "passes_per_step": passes32 / args.steps,
            "passes_fp64_per_step": sum(i["passes_fp64"] for _, i in infos32) / args.steps,
            "resid": [i["resid"] for _, i in infos32],
            "ms_solve_per_step": sum(i["ms_total"] for _, i in infos32) / args.steps,
        },
        "kernels_fp32_form": table(tim_all),
        "kernels_note": "per-class HIP-event times from a %d-step run with every class timed" % BREAKDOWN_STEPS,
    }
    # dominant relaxation kernel of the timed region.  Passes launched after an element has
    # stopped exit at once; the per-launch figure divides the class time by the launches that
    # did a pass (FP32-phase passes for *_fp32 classes, FP64 passes otherwise).
    base = dom[:-5] if dom.endswith("_fp32") else dom
    elem = 4 if dom.endswith("_fp32") else 8
    bpl = algorithmic_bytes(base, N, elem)
    p64 = sum(i["passes_fp64"] for _, i in infos32)
    working = (passes32 - p64) if dom.endswith("_fp32") else p64
    avg_s = tim32[dom][0] * 1e-3 / max(1, working)
    res["roofline"] = {"kernel": dom, "bound": "hbm", "achieved": bpl / avg_s / 1e9, "peak": PEAK_HBM / 1e9,
                       "unit": "GB/s", "frac": bpl / avg_s / PEAK_HBM, "traffic": stored_traffic(dom),
                       "bytes_per_launch": bpl, "avg_us": avg_s * 1e6, "launches": tim32[dom][1],
                       "working_launches": working}
    # per-class rates over the launches that did a pass (launches after convergence exit at once)
    pa = sum(i["passes"] for _, i in infos_all)
    pa64 = sum(i["passes_fp64"] for _, i in infos_all)
    gbs = {}
    for k, (ms, cnt) in tim_all.items():
        b = k[:-5] if k.endswith("_fp32") else k
        e = 4 if k.endswith("_fp32") else 8
        bb = algorithmic_bytes(b, N, e)
        if bb:
            gbs[k] = bb * ((pa - pa64) if k.endswith("_fp32") else pa64) / (ms * 1e-3) / 1e9
    res["kernel_GBps"] = gbs
    res["kernel_GBps_note"] = "algorithmic bytes x working launches / class time (breakdown run)"
    print("bench: FFT comparison", file=sys.stderr, flush=True)
    res["fft_comparison"] = fft_comparison(torch, dgp, dev)

    if not args.no_fp64:
        print("bench: timing float64 form", file=sys.stderr, flush=True)
        _, _, tim64 = run_form(dgp.FP64, BREAKDOWN_STEPS, 1)
        dt64, infos64, _ = run_form(dgp.FP64, args.steps, args.warmup, ["relax"])
        passes64 = sum(i["passes"] for _, i in infos64)
        t32 = sum(i["ms_total"] for _, i in infos32) / args.steps
        t64 = sum(i["ms_total"] for _, i in infos64) / args.steps
        res["fp64_form"] = {
            "value": N ** 3 * passes64 / dt64, "ms_per_step": 1e3 * dt64 / args.steps,
            "passes_per_step": passes64 / args.steps, "ms_solve_per_step": t64,
            "status": [s for s, _ in infos64], "resid": [i["resid"] for _, i in infos64],
            "kernels": table(tim64),
        }
        res["fp32_polish_vs_fp64_solve_speedup"] = t64 / t32 if t32 > 0 else None

    if not args.no_cpu:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(pos_h, growth * psi_h, lam)
    print(json.dumps(res))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_step(pos_h, vel_h, lam, tols):
    """One PM step of the CPU oracle on the benchmark's load: deposit, the field solve from the
    linear guess to each tolerance in `tols` (the step uses the first), forces, kick-drift.
    Returns per-stage seconds and the passes of each solve."""
    from oracle import field as fld, pm
    t = {}
    t0 = time.perf_counter()
    _, delta = pm.deposit(pos_h, N, BOX)
    t["deposit"] = time.perf_counter() - t0
    solves = {}
    u = None
    for tol in tols:
        prm = fld.SolveParams.from_cosmology(OM0, A, lam=lam, tol=tol, max_iter=200)
        t0 = time.perf_counter()
        uu, info = fld.solve(delta, BOX, prm)
        solves["%g" % tol] = {"seconds": time.perf_counter() - t0, "passes": info.iters + 1, "resid": info.resid}
        u = uu if u is None else u
    prm = fld.SolveParams.from_cosmology(OM0, A, lam=lam, tol=tols[0], max_iter=200)
    t0 = time.perf_counter()
    force, _ = pm.pm_forces(delta, u, pos_h, BOX, prm, OM0, A)
    t["forces"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    pm.kick_drift(pos_h, vel_h, force, A, DLNA, OM0, BOX)
    t["kick_drift"] = time.perf_counter() - t0
    t["solve"] = solves["%g" % tols[0]]["seconds"]
    return t, solves


def cpu_baseline(pos_h, vel_h, lam):
    """The CPU oracle (float64 NumPy, pocketfft) on one PM step of the same 256^3 workload, timed on
    the host: (i) as it stands, one thread; (ii) its transforms on all host cores (scipy.fft
    workers).  value = N^3 x passes / step seconds, the GPU headline's unit, from variant (i)."""
    from oracle import spectral
    cores = os.cpu_count() or 1
    t1, s1 = oracle_step(pos_h, vel_h, lam, [TOL])
    step1 = sum(t1.values())
    with spectral.fft_workers(cores):
        tn, sn = oracle_step(pos_h, vel_h, lam, [TOL, 1e-10])
    stepn = tn["deposit"] + tn["solve"] + tn["forces"] + tn["kick_drift"]
    passes = s1["%g" % TOL]["passes"]
    return {"value": N ** 3 * passes / step1, "unit": "cells*iter/s", "cores": 1, "kind": "oracle",
            "sample": "one PM step of the benchmark's 256^3 load (deposit, solve from the linear guess to 1e-8, "
                      "forces, kick-drift), float64 NumPy on 1 thread",
            "cpu_model": cpu_model(), "host_logical_cpus": cores,
            "stage_seconds": t1, "seconds_to_tol": {k: v["seconds"] for k, v in s1.items()},
            "passes": passes,
            "all_cores": {"value": N ** 3 * sn["%g" % TOL]["passes"] / stepn, "cores": cores,
                          "transforms": "scipy.fft, workers = %d" % cores, "stage_seconds": tn,
                          "seconds_to_tol": {k: v["seconds"] for k, v in sn.items()},
                          "passes_to_tol": {k: v["passes"] for k, v in sn.items()}}}


if __name__ == "__main__":
    main()
