"""Benchmark: HB-UGKS pseudo steps per second on one MI355X.

One step = one pass of the whole pseudo step (moments, faces, cells,
local steps + residual, interior and boundary-ring update) over the
64 x 64-cell, 48 x 48-velocity (on [-5, 5]), N_H = 4 (nine levels) thermal
cavity (Kn = 1, St = 1, bottom wall T0 (1 + 0.5 sin wt), Shakhov) in the
mixed form (FP32 storage of the deviation from the rest Maxwellian and FP32
per-velocity arithmetic; FP64 moment sums, W and residual), state resident in
HBM.  value = cell x velocity x level updates per second, from K steps
timed on the host clock between stream synchronisations; a second run of
the same K steps with HIP events around every kernel gives the per-kernel
times and the roofline of the dominant kernel.

Prints one JSON line (stdout).  Progress goes to stderr.
  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
                  [--precision fp64|mixed] [--workload thermal|shear] [--no-extra] [--copy-mib N]
                  [--only batch|batch_converge|serving|hbtd] [--form batched|plain]
                  [--first I] [--count N] [--cap S] [--requests N] [--rate R] [--td-cap S]
Besides the headline, the JSON line carries: the headline case's one-step
error against the FP64 oracle at full size, the oracle timed on the host
(all threads and one), the time to converge from rest, the 16 x 16-cell FP64
correctness case solved to convergence on the GPU and by the oracle (wall
times and converged harmonics against each other), the 64 x 64-cell,
32 x 32-velocity, N_H = 1 shear cavity in both forms, per-step times over
the Kn x St grids, and the 64-case batched sweep.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell·ξ·instance updates/s per pseudo-step (%HBM peak); cases/h; p50/p99"
HBM_PEAK_GBS = 8000.0
# converged cases/h of the 64-case sweep in the batched mixed form (bench.py --only batch_converge:
# 64 of 64 converged in 781 s);
# the serving run's Poisson rate is 0.8 of it
BATCHED_CAPACITY_PER_H = 295.0
KERNEL_SOURCES = ("paper_2605_03479_amd/csrc/hb_kernels.h", "paper_2605_03479_amd/csrc/hb_device.h",
                  "paper_2605_03479_amd/csrc/hb_layout.h", "paper_2605_03479_amd/csrc/hb_mixed.h")
# rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE, KiB per dispatch x 1024 x calibration
# (fetch x2.0, write x1.0 from a 256 MiB copy), averaged over the profiled launches
MEASURED_TRAFFIC = {
    "sources_sha256_16": "d6f78dbca9155cd5",
    "bytes": {
        "shear64_v32_nh1_kn1_st1/fp64/moments": 263871898,
        "shear64_v32_nh1_kn1_st1/fp64/update_int": 617515315,
        "shear64_v32_nh1_kn1_st1/fp64/update_bnd": 73693901,
        "shear64_v32_nh1_kn1_st1/mixed/moments": 152945766,
        "shear64_v32_nh1_kn1_st1/mixed/update_int": 247780250,
        "shear64_v32_nh1_kn1_st1/mixed/update_bnd": 38398259,
        "thermal64_v48_nh4_kn1_st1/mixed/moments": 1082988544,
        "thermal64_v48_nh4_kn1_st1/mixed/update_int": 2144916070,
        "thermal64_v48_nh4_kn1_st1/mixed/update_bnd": 257197773,
    },
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def roofline(kernel, timing, algo, traffic):
    """Roofline object of one kernel from its HIP-event timing (launches, ms)."""
    n, ms = timing
    avg_s = ms / max(n, 1) * 1e-3
    achieved = None if algo is None else algo / avg_s / 1e9
    return {"kernel": kernel, "bound": "hbm", "achieved": None if achieved is None else round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": None if achieved is None else round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_what": "bytes per launch beyond L2 (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, calibrated on a "
                            "plain device copy); includes Infinity Cache hits, so an upper bound on HBM bytes",
            "avg_launch_us": round(avg_s * 1e6, 2), "algorithmic_bytes_per_launch": algo}


def traffic_bytes(workload, precision, kernel):
    """Bytes per launch beyond L2 (FETCH_SIZE, WRITE_SIZE, calibrated on a plain
    copy), as measured on the kernel sources whose digest is recorded; None when
    the sources have changed since or no measurement exists."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != MEASURED_TRAFFIC["sources_sha256_16"]:
        return None
    return MEASURED_TRAFFIC["bytes"].get(f"{workload}/{precision}/{kernel}")


def batched_sweep(hb, hbcases, steps=5):
    """The 64-case seeded sweep: one batch step of the tuned mixed batch
    against the plain FP64 solver stepping the same cases one at a time."""
    cases = hbcases.batch_sweep()
    tot = sum(c.updates for c in cases)
    B = hb.Batch(max_cases=len(cases))
    for c in cases:
        B.add(c, hb.HB_MIXED)
    B.tune(2)
    B.step(1)
    B.residuals()
    t0 = time.perf_counter()
    B.step(steps)
    r = B.residuals()
    t_batch = (time.perf_counter() - t0) / steps
    diverged = sum(1 for v in r.values() if v[2])
    B.close()
    t_plain = 0.0
    for c in cases:
        s = hb.Solver(c)
        s.step(1)
        s.residual()
        t0 = time.perf_counter()
        s.step(3)
        s.residual()
        t_plain += (time.perf_counter() - t0) / 3
        s.close()
    log(f"batched sweep: mixed batch {t_batch * 1e3:.1f} ms/step, plain fp64 one at a time {t_plain * 1e3:.1f} ms")
    return {"workload": "batch_sweep_64_seed260503479", "updates_per_step": tot,
            "batched_mixed_ms_per_step": t_batch * 1e3, "batched_mixed_updates_per_s": tot / t_batch,
            "plain_fp64_ms_per_step": t_plain * 1e3, "plain_fp64_updates_per_s": tot / t_plain,
            "speedup_batched_vs_plain": t_plain / t_batch, "diverged": diverged}


def batch_converge(hb, hbcases, form, tol=1e-8, check_every=200, max_steps=60000, cap_s=900.0, first=0,
                   count=64):
    """The 64-case seeded sweep to R_rho <= tol.  form "batched": all cases
    present at once in the serving loop, mixed form, each retired when it
    converges (converged cases/h = converged / wall).  form "plain": the FP64
    solver on cases [first, first + count) one at a time, residual read every
    check_every steps, each case capped at max_steps and the whole run at
    cap_s (cases not reached are listed)."""
    cases = hbcases.batch_sweep()
    out = {"workload": "batch_sweep_64_seed260503479", "form": form, "tol": tol, "check_every": check_every,
           "max_steps": max_steps, "cap_s": cap_s}
    if form == "batched":
        B = hb.Batch(max_cases=len(cases))
        res, _, wall = hb.serve(B, cases, [0.0] * len(cases), precision=hb.HB_MIXED, tol=tol,
                                check_every=check_every, max_steps=max_steps, var_mask=0x1, max_wall_s=cap_s)
        B.close()
        out["cases"] = [{"name": c.name, "updates": c.updates, "status": r["status"], "steps": r["steps"],
                         "t_done_s": r["t_done"], "R_rho": r["residual"][0]} for c, r in zip(cases, res)]
        conv = sum(1 for r in res if r["status"] == hb.HB_OK)
        out.update(converged=conv, wall_s=wall, cases_per_h=3600.0 * conv / wall)
        log(f"batched mixed: {conv}/{len(cases)} converged in {wall:.1f} s ({out['cases_per_h']:.0f} cases/h)")
        return out
    t_run = time.perf_counter()
    rows = []
    for idx in range(first, min(first + count, len(cases))):
        c = cases[idx]
        if time.perf_counter() - t_run > cap_s:
            rows.append({"name": c.name, "status": "not run (wall cap)"})
            continue
        s = hb.Solver(c)
        t0 = time.perf_counter()
        k, r = 0, float("inf")
        while k < max_steps:
            s.step(check_every)
            k += check_every
            try:
                r = s.residual()[0]
            except hb.HBError:
                r = float("nan")
                break
            if r <= tol:
                break
            if k % (10 * check_every) == 0:
                log(f"plain fp64 {c.name}: {k} steps, R_rho {r:.2e}")
        dt = time.perf_counter() - t0
        s.close()
        rows.append({"name": c.name, "updates": c.updates, "status": "converged" if r <= tol else "not converged",
                     "steps": k, "wall_s": dt, "R_rho": r})
        log(f"plain fp64 {c.name}: {k} steps, R_rho {r:.2e}, {dt:.1f} s")
    out["cases"] = rows
    done = [r for r in rows if r["status"] == "converged"]
    out.update(converged=len(done), wall_s=time.perf_counter() - t_run)
    return out


def serving_plain(hb, hbcases, n=48, rate_per_s=None, cap_s=900.0, check_every=200, max_steps=60000, tol=1e-8):
    """The serving workload served by the plain FP64 solver, one request at a
    time in arrival order (first in, first out): the same requests and the
    same arrival times in wall-clock time; each request is stepped until
    R_rho <= tol (residual read every check_every steps); the run stops at
    cap_s, cutting the request in progress off unconverged and leaving the
    later ones unserved (listed, not dropped)."""
    import numpy as np
    reqs = hbcases.serving_requests(n)
    arr = hbcases.poisson_arrivals(n, rate_per_s)
    t0 = time.perf_counter()
    rows = []
    capped = False
    for c, a in zip(reqs, arr):
        row = {"name": c.name, "updates": c.updates, "arrival_s": float(a), "t_start_s": None, "t_done_s": None,
               "status": "not served (wall cap)", "steps": 0, "R_rho": None}
        rows.append(row)
        if capped:
            continue
        now = time.perf_counter() - t0
        if now < a:
            time.sleep(a - now)
        if time.perf_counter() - t0 >= cap_s:
            capped = True
            continue
        row["t_start_s"] = time.perf_counter() - t0
        s = hb.Solver(c)
        k, r = 0, float("inf")
        while k < max_steps:
            s.step(check_every)
            k += check_every
            r = s.residual()[0]
            if r <= tol or time.perf_counter() - t0 >= cap_s:
                break
            if k % (10 * check_every) == 0:
                log(f"plain fp64 serving {c.name}: {k} steps, R_rho {r:.2e}")
        s.close()
        row.update(t_done_s=time.perf_counter() - t0, steps=k, R_rho=r,
                   status="converged" if r <= tol else "not converged (wall cap)")
        capped = r > tol and time.perf_counter() - t0 >= cap_s
        log(f"plain fp64 serving {c.name}: {row['status']}, {k} steps, latency {row['t_done_s'] - a:.1f} s")
    wall = time.perf_counter() - t0
    lat = np.array([r["t_done_s"] - r["arrival_s"] for r in rows if r["status"] == "converged"])
    conv = int(len(lat))
    return {"workload": f"serving_{n}_requests_seed260503480_arrivals260503481", "form": "plain fp64, one at a time",
            "requests": n, "poisson_rate_per_s": rate_per_s, "cap_s": cap_s, "check_every": check_every,
            "wall_s": wall, "converged": conv, "cases_per_h": 3600.0 * conv / wall,
            "p50_time_to_converged_s": float(np.percentile(lat, 50)) if conv else None,
            "p99_time_to_converged_s": float(np.percentile(lat, 99)) if conv else None,
            "requests_detail": rows}


def serving(hb, hbcases, n=48, rate_per_s=None, cap_s=900.0, check_every=200, max_steps=60000, tol=1e-8):
    """The serving workload: n seeded requests drawn as the batched sweep with
    1/16 outliers of 128^2 cells x 64^2 velocities x N_H = 5, arriving as a
    seeded Poisson process, served in the mixed form with admission by device
    footprint until each reaches R_rho <= tol; the run is capped at cap_s
    (requests unconverged or never admitted are listed, not dropped)."""
    import numpy as np
    reqs = hbcases.serving_requests(n)
    arr = hbcases.poisson_arrivals(n, rate_per_s)
    B = hb.Batch(max_cases=n)
    res, _, wall = hb.serve(B, reqs, arr, precision=hb.HB_MIXED, tol=tol, check_every=check_every,
                            max_steps=max_steps, var_mask=0x1, max_wall_s=cap_s)
    B.close()
    lat = np.array([r["t_done"] - r["arrival"] for r in res if r["status"] == hb.HB_OK])
    conv = int(len(lat))
    out = {"workload": f"serving_{n}_requests_seed260503480_arrivals260503481", "requests": n,
           "poisson_rate_per_s": rate_per_s, "cap_s": cap_s, "check_every": check_every, "wall_s": wall,
           "converged": conv, "cases_per_h": 3600.0 * conv / wall,
           "p50_time_to_converged_s": float(np.percentile(lat, 50)) if conv else None,
           "p99_time_to_converged_s": float(np.percentile(lat, 99)) if conv else None,
           "requests_detail": [{"name": c.name, "updates": c.updates, "arrival_s": r["arrival"],
                                "t_admit_s": r["t_admit"], "t_done_s": r["t_done"], "status": r["status"],
                                "steps": r["steps"], "R_rho": r["residual"][0]} for c, r in zip(reqs, res)]}
    log(f"serving: {conv}/{n} converged in {wall:.1f} s, {out['cases_per_h']:.0f} cases/h, "
        f"p50 {out['p50_time_to_converged_s']} s, p99 {out['p99_time_to_converged_s']} s")
    return out


def td_step_size(hb, case):
    """Physical step of the time-domain solver: the CFL bound of Eqs. (31)-(32)
    without the spectral term, for gas at rest at the hottest wall
    temperature (the flows here stay at low speed), over every cell; rounded down so that one forcing
    period holds a whole number of steps.  Returns (dt, steps per period)."""
    import numpy as np
    u, _ = hb.hb_vgrid_nodes(case.M, case.umax, case.vrule)
    v, _ = hb.hb_vgrid_nodes(case.Mv_, case.vmax_, case.vrule)
    gamma = (case.K + 4.0) / (case.K + 2.0)
    t_max = max(w[3] + np.hypot(w[4], w[5]) for w in case.walls)  # hottest wall, in T0
    cs = np.sqrt(gamma * max(1.0, t_max) / 2.0)
    ut = max(abs(u[0]), abs(u[-1])) + cs
    vt = max(abs(v[0]), abs(v[-1])) + cs
    dx = np.diff(case.x_faces) if case.x_faces is not None else np.full(case.nx, case.L / case.nx)
    dy = np.diff(case.y_faces) if case.y_faces is not None else np.full(case.ny, case.H / case.ny)
    nu = ut / dx.min() + vt / dy.min()
    period = 2.0 * np.pi / case.St
    ns = int(np.ceil(period * nu / case.cfl))
    return period / ns, ns


def _top_fundamental(case, W, thermal):
    """Cell-width-weighted mean over the top-wall cells of U (shear) or T/T0
    (thermal) from W[c][4] (rest energy (2 + K)/4 per unit density at T0)."""
    import numpy as np
    top = (case.ny - 1) * case.nx + np.arange(case.nx)
    ds = np.diff(case.x_faces)
    Wt = W[top]
    rho = Wt[:, 0]
    if thermal:
        ke = 0.5 * (Wt[:, 1] ** 2 + Wt[:, 2] ** 2) / rho
        q = 4.0 * (Wt[:, 3] - ke) / ((2.0 + case.K) * rho)
    else:
        q = Wt[:, 1] / rho
    return np.sum(ds * q) / np.sum(ds)


def hb_vs_td(hb, hbcases, St, prec, cap_s, workload="shear", drop=7.0, hb_sample=100):
    """Wall-clock to a `drop`-decade fall of the density residual (Eq. 43),
    HB-UGKS (N_H = 1, local pseudo steps, residual sampled every hb_sample
    steps) against the explicit time-domain UGKS (one level, global physical
    step, period residual), both on the GPU from the same code, on the
    paper's shear or thermal cavity (90 x 90 wall-refined cells, 28^2
    Gauss-Hermite velocities, Kn = 0.1; thermal: N_H = 2).  Each clock starts at its first residual sample,
    as the paper's shifted curves do; the unshifted totals are reported too.
    The time-domain fundamental of U (shear) or T (thermal) along the top
    wall is taken over one more period and compared with the HB one."""
    import numpy as np
    thermal = workload == "thermal"
    case = hbcases.thermal_paper(St) if thermal else hbcases.shear_paper(St)
    ua = case.walls[2][4] if thermal else case.walls[2][1]  # top-wall amplitude
    var = 3 if thermal else 1
    out = {"workload": case.name, "St": St, "precision": "mixed" if prec == hb.HB_MIXED else "fp64",
           "drop_decades": drop}
    # HB
    s = hb.Solver(case, precision=prec)
    t0 = time.perf_counter()
    k, r1, t1, hist = 0, None, None, []
    while True:
        s.step(hb_sample)
        k += hb_sample
        r = s.residual()[0]
        t = time.perf_counter() - t0
        if r1 is None:
            r1, t1 = r, t
        hist.append((k, t, r))
        if k % (50 * hb_sample) == 0:
            log(f"HB St {St}: step {k} R_rho {r:.3e} ({np.log10(r / r1):.2f} decades) {t:.1f} s")
        if r <= r1 * 10.0 ** -drop or t > cap_s:
            break
    u_hb = 2.0 * abs(s.wall_harmonic(2, var, 1)) / ua
    out["hb"] = {"steps": k, "wall_s": t, "shifted_wall_s": t - t1, "R1": r1, "R_end": r,
                 "reached": bool(r <= r1 * 10.0 ** -drop), "top_amplitude": u_hb,
                 "ms_per_step": 1e3 * t / k}
    s.close()
    log(f"HB St {St}: {k} steps, {t:.2f} s, top amplitude {u_hb:.5f}")
    # time domain
    dt, ns = td_step_size(hb, case)
    tdc = case.with_(NH=0, dt_mode=1, dt_fixed=dt)
    s = hb.Solver(tdc, precision=prec)
    t0 = time.perf_counter()
    p, r1, t1 = 0, None, None
    while True:
        r = s.td_period(ns)[0]
        p += 1
        t = time.perf_counter() - t0
        if r1 is None:
            r1, t1 = r, t
        log(f"TD St {St}: period {p} ({ns} steps) R_rho {r:.3e} ({np.log10(r / r1):.2f} decades) {t:.1f} s")
        if r <= r1 * 10.0 ** -drop or t > cap_s:
            break
    # fundamental of the top-wall quantity over one more period
    acc = 0.0j
    for j in range(ns):
        s.td_step(1)
        acc += _top_fundamental(case, s.macro()[:, 0, :], thermal) * np.exp(-1j * St * (p * ns + j + 1) * dt)
    u_td = 2.0 * abs(acc / ns) / ua
    out["td"] = {"dt": dt, "steps_per_period": ns, "periods": p, "steps": p * ns, "wall_s": t,
                 "shifted_wall_s": t - t1, "R1": r1, "R_end": r, "reached": bool(r <= r1 * 10.0 ** -drop),
                 "top_amplitude": u_td, "ms_per_step": 1e3 * t / (p * ns)}
    s.close()
    out["speedup_shifted"] = out["td"]["shifted_wall_s"] / out["hb"]["shifted_wall_s"]
    out["speedup_total"] = out["td"]["wall_s"] / out["hb"]["wall_s"]
    out["top_amplitude_what"] = "lid-averaged T/T0 fundamental / T_a" if thermal else "lid-averaged U fundamental / U_a"
    out["top_amplitude_rel_diff"] = abs(u_hb - u_td) / u_td
    log(f"TD St {St}: {p} periods, {t:.2f} s, top amplitude {u_td:.5f}; speedup {out['speedup_shifted']:.2f} "
        f"(total {out['speedup_total']:.2f})")
    return out


def timed_run(hb, case, prec, stream, sync, steps, warmup, events=True):
    """Warm up, then time `steps` pseudo steps, with per-kernel HIP events on
    the handle's stream (events=True) or without; returns (ms per step,
    per-kernel (launches, ms) or {}, residual)."""
    s = hb.Solver(case, device=0, stream=stream, precision=prec)
    s.step(warmup)
    s.residual()  # synchronises the handle's stream
    if sync:
        sync()
    s.enable_timing(events)
    t0 = time.perf_counter()
    s.step(steps)
    s.residual()
    if sync:
        sync()
    t1 = time.perf_counter()
    kt = s.kernel_times() if events else {}
    res = s.residual()
    s.close()
    return (t1 - t0) * 1e3 / steps, kt, res


def timed_median(hb, case, prec, stream, sync, steps, warmup, reps=3):
    """Median of `reps` timings of `steps` pseudo steps on one handle (ms per
    step), so that one stalled segment of a short sweep point does not stand
    for the point."""
    s = hb.Solver(case, device=0, stream=stream, precision=prec)
    s.step(warmup)
    s.residual()
    if sync:
        sync()
    t = []
    for _ in range(reps):
        t0 = time.perf_counter()
        s.step(steps)
        s.residual()
        if sync:
            sync()
        t.append((time.perf_counter() - t0) * 1e3 / steps)
    s.close()
    return sorted(t)[len(t) // 2]


def small_full_solve(hb, hbcases, oracle_mod, stream, sync, tol=1e-8, chunk=100, max_steps=200000, cap_s=120.0):
    """The FP64 correctness case (16^2 cells, 16^2 velocities on [-4, 4], BGK,
    N_H = 1, Kn = St = 1) solved from rest to R_rho <= tol on the GPU, and, with
    oracle_mod given, by the oracle on this host's cores (its CPU baseline for
    a full solve); then the converged harmonics of the two against each other,
    per variable: the largest difference over the variable's largest |q_k|, k >= 1."""
    import numpy as np
    case = hbcases.shear_small()

    def solve(step, residual):
        t0 = time.perf_counter()
        k, r = 0, float("inf")
        while k < max_steps and time.perf_counter() - t0 < cap_s:
            step(chunk)
            k += chunk
            r = residual()
            if r <= tol:
                break
        return k, r, time.perf_counter() - t0

    s = hb.Solver(case, device=0, stream=stream)
    k, r, t = solve(s.step, lambda: s.residual()[0])
    if sync:
        sync()
    re_g, im_g = s.harmonics()
    s.close()
    out = {"workload": case.name, "precision": "fp64", "tol": tol,
           "gpu": {"steps": k, "residual": r, "converged": bool(r <= tol), "wall_s": t}}
    if oracle_mod is not None:
        o = oracle_mod.Oracle(case)
        ko, ro, to = solve(o.step, lambda: o.residual()[0])
        re_o, im_o = o.harmonics()
        out["cpu_oracle"] = {"steps": ko, "residual": ro, "converged": bool(ro <= tol), "wall_s": to,
                             "cores": oracle_mod.threads(), "kind": "oracle", "host": host_cpu()}
        names = ("rho", "U", "V", "T", "P_xy", "q_x", "q_y")
        err = {}
        for v, nm in enumerate(names):
            sig = np.max(np.hypot(re_o[v, 1:], im_o[v, 1:]))
            d = np.max(np.hypot(re_g[v] - re_o[v], im_g[v] - im_o[v]))
            err[nm] = float(d / sig) if sig > 0 else None
        out["harmonics_rel_err_gpu_vs_oracle"] = err
    return out


def host_cpu():
    """CPU model and logical CPUs of this host (for the oracle baseline)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def oracle_error(hb, oracle, hbcases, case, prec):
    """One pseudo step of `case` from a seeded perturbed state on the GPU (the
    launch configuration timed above) and on the oracle; the largest
    difference of W, h, b over the step's signal (largest deviation of the
    oracle's result from the rest state, floored at 1% of the state)."""
    import numpy as np
    o = oracle.Oracle(case)
    W, h, b = o.state()
    rest = (W[:, :1, :].copy(), h[:, :1, :].copy(), b[:, :1, :].copy())
    h = h * (1.0 + 0.02 * hbcases.uniform(h.shape, 4242))
    b = b * (1.0 + 0.02 * hbcases.uniform(b.shape, 4243))
    W = W * (1.0 + 0.01 * hbcases.uniform(W.shape, 4244))
    o.set_state(W, h, b)
    s = hb.Solver(case, precision=prec)
    s.set_state(W, h, b)
    del W, h, b
    o.step(1)
    s.step(1)
    out = {}
    for name, a, r, r0 in zip("Whb", s.state(), o.state(), rest):
        scale = max(np.max(np.abs(r - r0)), 1e-2 * np.max(np.abs(r)))
        out[name] = float(np.max(np.abs(a - r)) / scale)
    s.close()
    return {"what": "one step from a seeded perturbed state, max|gpu - oracle| / signal", "rel_err": out}


def cpu_oracle(oracle, case, target_s=15.0):
    """The oracle timed on this host's cores for about target_s seconds."""
    o = oracle.Oracle(case)
    o.step(1)  # first touch / page-in
    t = time.perf_counter()
    o.step(1)
    per = time.perf_counter() - t
    steps = max(1, min(200, int(target_s / max(per, 1e-6))))
    t = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t
    return {"value": case.updates * steps / dt, "unit": "updates/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{steps} pseudo steps of {case.name} ({case.nc} cells x {case.nv} velocities x "
                      f"{case.NT} levels), {dt:.1f} s", "host": host_cpu()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--kn", type=float, default=1.0)
    ap.add_argument("--st", type=float, default=1.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default=None,
                    help="default: mixed for the thermal workload, fp64 for the shear one")
    ap.add_argument("--workload", choices=("shear", "thermal"), default="thermal",
                    help="thermal: 64x64 cells, 48x48 velocities on [-5,5], NH=4 (the HBM-roofline case); "
                         "shear: 64x64, 32x32, NH=1")
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary workloads")
    ap.add_argument("--only", choices=("batch", "batch_converge", "serving", "hbtd"), default=None,
                    help="run only the batched sweep's step time, the sweep to convergence, the serving "
                         "measurement or the HB-vs-time-domain comparison (prints its JSON)")
    ap.add_argument("--form", choices=("batched", "plain"), default="batched",
                    help="batch_converge / serving: all cases batched (mixed) or one at a time (FP64)")
    ap.add_argument("--first", type=int, default=0, help="batch_converge plain: first case")
    ap.add_argument("--count", type=int, default=64, help="batch_converge plain: number of cases")
    ap.add_argument("--cap", type=float, default=900.0, help="batch_converge / serving: wall-clock cap (s)")
    ap.add_argument("--requests", type=int, default=48, help="serving: number of requests")
    ap.add_argument("--rate", type=float, default=None,
                    help="serving: Poisson arrival rate (1/s); default 0.8 x the measured batched capacity")
    ap.add_argument("--td-cap", type=float, default=600.0,
                    help="hbtd: wall-clock cap (s) of each solver's run")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run 5 plain device copies of this many MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(batched cases would shard by case with no communication).", file=sys.stderr)
        sys.exit(2)
    if args.precision is None:
        args.precision = "mixed" if args.workload == "thermal" else "fp64"

    import hbcases
    import paper_2605_03479_amd as hb
    from paper_2605_03479_amd import build as hb_build

    if not os.path.exists(hb_build.LIB):
        import __graft_entry__
        __graft_entry__.build()

    stream = None
    sync = None
    try:
        import torch
        if torch.cuda.is_available():
            stream = torch.cuda.current_stream().cuda_stream
            sync = torch.cuda.synchronize
    except Exception:  # torch is plumbing only
        pass

    if args.copy_mib > 0:
        import torch
        src = torch.ones(args.copy_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 5 x {args.copy_mib} MiB device copies")
        del src, dst

    if args.only == "hbtd":
        prec = hb.HB_MIXED if args.precision == "mixed" else hb.HB_FP64
        print(json.dumps(hb_vs_td(hb, hbcases, args.st, prec, args.td_cap, args.workload)), flush=True)
        return
    if args.only == "batch":
        print(json.dumps(batched_sweep(hb, hbcases)), flush=True)
        return
    if args.only in ("batch_converge", "serving"):
        os.environ.setdefault("HB_SERVE_PROGRESS", "1")  # the serving loop's per-chunk lines on stderr
    if args.only == "batch_converge":
        print(json.dumps(batch_converge(hb, hbcases, args.form, cap_s=args.cap, first=args.first,
                                        count=args.count)), flush=True)
        return
    if args.only == "serving":
        rate = args.rate if args.rate is not None else 0.8 * BATCHED_CAPACITY_PER_H / 3600.0
        fn = serving if args.form == "batched" else serving_plain
        print(json.dumps(fn(hb, hbcases, n=args.requests, rate_per_s=rate, cap_s=args.cap)), flush=True)
        return

    prec = hb.HB_MIXED if args.precision == "mixed" else hb.HB_FP64
    case = hbcases.shear_cavity(args.kn, args.st) if args.workload == "shear" else \
        hbcases.thermal_cavity(args.kn, args.st)
    log(f"case {case.name}: {case.nc} cells x {case.nv} velocities x {case.NT} levels = {case.updates} updates/step")
    # the step time without per-kernel events; then the same run with them,
    # for the per-kernel times and the roofline
    ms_step, _, res = timed_run(hb, case, prec, stream, sync, args.steps, args.warmup, events=False)
    ms_events, kt, _ = timed_run(hb, case, prec, stream, sync, args.steps, args.warmup)
    ups = case.updates / (ms_step * 1e-3)
    log(f"ms/step {ms_step:.4f}  updates/s {ups:.4e}  residual {res}  (with per-kernel events {ms_events:.4f})")
    for k, (n, ms) in kt.items():
        log(f"  kernel {k:9s} launches {n:6d}  avg {ms / max(n, 1) * 1e3:9.2f} us")

    # roofline of the dominant kernel: algorithmic HBM bytes per launch
    #   update_int/_bnd: read h, b and write h, b once per (cell, velocity, level) of its cells -> 4 words
    #   moments: read h, b once per (cell, velocity, level) -> 2 words
    wb = 4.0 if prec == hb.HB_MIXED else 8.0  # bytes per stored word of h or b
    n_int = max(case.nx - 4, 0) * max(case.ny - 4, 0)
    per_cell = case.nv * case.NT
    algo_bytes = {"update_int": 4 * wb * n_int * per_cell, "update_bnd": 4 * wb * (case.nc - n_int) * per_cell,
                  "moments": 2 * wb * case.updates}
    dom = max(kt, key=lambda k: kt[k][1])
    roof = roofline(dom, kt[dom], algo_bytes.get(dom), traffic_bytes(case.name, args.precision, dom))
    # the method's own floor: read (h, b) once and write them once per update
    step_bytes = 4 * wb * case.updates
    kernels = {k: round(ms / max(n, 1) * 1e3, 2) for k, (n, ms) in kt.items()}

    import oracle
    err = None
    if not args.no_extra:
        err = oracle_error(hb, oracle, hbcases, case, prec)
        log(f"oracle error, one step: {err['rel_err']}")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_oracle(oracle, case)
        log(f"cpu oracle: {cpu['value']:.4e} updates/s on {cpu['cores']} threads ({cpu['host']['model']})")

    # the oracle on one host thread, in a child process (OpenMP reads its thread count at start-up)
    cpu1 = None
    if cpu is not None and not args.no_extra:
        import subprocess
        mk = "shear_cavity" if args.workload == "shear" else "thermal_cavity"
        code = ("import sys, time; sys.path.insert(0, %r); import hbcases, oracle; "
                "c = hbcases.%s(%r, %r); o = oracle.Oracle(c); o.step(1); t = time.perf_counter(); "
                "o.step(1); print(c.updates / (time.perf_counter() - t), oracle.threads())") % (
            ROOT, mk, args.kn, args.st)
        env = dict(os.environ, OMP_NUM_THREADS="1")
        try:
            r1 = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
            v1, th1 = r1.stdout.split()[-2:]
            cpu1 = {"value": float(v1), "unit": "updates/s", "cores": int(th1), "kind": "oracle",
                    "sample": f"1 pseudo step of {case.name}"}
            log(f"cpu oracle, one thread: {cpu1['value']:.4e} updates/s")
        except Exception as e:  # the baseline is context; the GPU numbers stand without it
            log(f"cpu oracle, one thread: not measured ({e})")

    # time to converge: the same case from rest to R_rho <= 1e-8 (Eq. 43), residual read every 100 steps
    conv = None
    if not args.no_extra:
        s = hb.Solver(case, device=0, stream=stream, precision=prec)
        t0 = time.perf_counter()
        k = 0
        r = float("inf")
        while k < 200000 and time.perf_counter() - t0 < 60.0:
            s.step(100)
            k += 100
            try:
                r = s.residual()[0]
            except hb.HBError:
                r = float("nan")
                break
            if r <= 1e-8:
                break
        tconv = time.perf_counter() - t0
        s.close()
        conv = {"tol": 1e-8, "steps": k, "residual": r, "converged": bool(r <= 1e-8), "wall_s": tconv,
                "cases_per_h": 3600.0 / tconv if r <= 1e-8 else None, "wall_cap_s": 60.0}
        if cpu is not None:
            cpu_step = case.updates / cpu["value"]
            conv["cpu_oracle_wall_s_extrapolated"] = k * cpu_step
        log(f"converge: {k} steps to R_rho {r:.2e} in {tconv:.2f} s")

    # the correctness case: a full solve on the GPU and by the oracle on the host
    small = None
    if not args.no_extra:
        small = small_full_solve(hb, hbcases, None if args.no_cpu else oracle, stream, sync)
        g = small["gpu"]
        log(f"correctness case {small['workload']}: GPU {g['steps']} steps to R_rho {g['residual']:.2e} in "
            f"{g['wall_s']:.2f} s" + (f"; oracle {small['cpu_oracle']['steps']} steps in "
                                       f"{small['cpu_oracle']['wall_s']:.1f} s; harmonics "
                                       f"{small['harmonics_rel_err_gpu_vs_oracle']}" if "cpu_oracle" in small else ""))

    extra = []
    if not args.no_extra:
        others = []
        if args.workload == "thermal":
            others += [(hbcases.shear_cavity(1.0, 1.0), hb.HB_FP64, "fp64"),
                       (hbcases.shear_cavity(1.0, 1.0), hb.HB_MIXED, "mixed")]
        else:
            if prec == hb.HB_FP64:
                others.append((case, hb.HB_MIXED, "mixed"))
            others.append((hbcases.thermal_cavity(1.0, 1.0), hb.HB_MIXED, "mixed"))
        for c2, p2, pname in others:
            steps2 = max(10, min(args.steps, 100))
            ms2, kt2, _ = timed_run(hb, c2, p2, stream, sync, steps2, 5)
            n2 = max(c2.nx - 4, 0) * max(c2.ny - 4, 0)
            d2 = max(kt2, key=lambda k: kt2[k][1])
            wb2 = 4.0 if p2 == hb.HB_MIXED else 8.0
            a2 = {"update_int": 4 * wb2 * n2 * c2.nv * c2.NT, "moments": 2 * wb2 * c2.updates}.get(d2)
            extra.append({"workload": c2.name, "precision": pname, "updates_per_s": c2.updates / (ms2 * 1e-3),
                          "ms_per_step": ms2, "steps": steps2,
                          "effective_GBps_per_step": 4 * wb2 * c2.updates / (ms2 * 1e-3) / 1e9,
                          "kernel_avg_us": {k: round(ms / max(n, 1) * 1e3, 2) for k, (n, ms) in kt2.items()},
                          "roofline": roofline(d2, kt2[d2], a2, traffic_bytes(c2.name, pname, d2))})
            log(f"extra {c2.name} {pname}: ms/step {ms2:.4f} updates/s {c2.updates / (ms2 * 1e-3):.4e}")
            if c2.name.startswith("shear64") and p2 == hb.HB_FP64:
                # a full solve of this case from rest (residual read every 100 steps, capped at 60 s)
                s2 = hb.Solver(c2, device=0, stream=stream, precision=p2)
                t0 = time.perf_counter()
                k2, r2 = 0, float("inf")
                while k2 < 200000 and time.perf_counter() - t0 < 60.0:
                    s2.step(100)
                    k2 += 100
                    r2 = s2.residual()[0]
                    if r2 <= 1e-8:
                        break
                t2 = time.perf_counter() - t0
                s2.close()
                extra[-1]["converge"] = {"tol": 1e-8, "steps": k2, "residual": r2, "converged": bool(r2 <= 1e-8),
                                         "wall_s": t2, "wall_cap_s": 60.0}
                if cpu is not None:  # the oracle's rate on the headline case, applied to these steps
                    extra[-1]["converge"]["cpu_oracle_wall_s_extrapolated"] = k2 * c2.updates / cpu["value"]
                log(f"extra {c2.name} {pname}: converge {k2} steps to R_rho {r2:.2e} in {t2:.2f} s")

    # per-step time over the Kn x St grids of the shear and thermal cases (the arithmetic per step does not
    # depend on them)
    knst = None
    if not args.no_extra:
        knst = []
        for kn in hbcases.SHEAR_KN:
            for st in hbcases.SHEAR_ST:
                c3 = hbcases.shear_cavity(kn, st)
                for p3, pn in ((hb.HB_FP64, "fp64"), (hb.HB_MIXED, "mixed")):
                    ms3 = timed_median(hb, c3, p3, stream, sync, 30, 5)
                    knst.append({"workload": c3.name, "precision": pn, "Kn": kn, "St": st, "ms_per_step": ms3,
                                 "updates_per_s": c3.updates / (ms3 * 1e-3)})
        log("shear Kn x St: ms/step " + " ".join(f"{d['ms_per_step']:.3f}" for d in knst))
        for kn in hbcases.THERMAL_KN:
            for st in hbcases.THERMAL_ST:
                c3 = hbcases.thermal_cavity(kn, st)
                ms3 = timed_median(hb, c3, hb.HB_MIXED, stream, sync, 20, 5)
                knst.append({"workload": c3.name, "precision": "mixed", "Kn": kn, "St": st, "ms_per_step": ms3,
                             "updates_per_s": c3.updates / (ms3 * 1e-3)})
        log("thermal Kn x St: ms/step " + " ".join(f"{d['ms_per_step']:.3f}" for d in knst[-4:]))

    batched = None
    if not args.no_extra:
        batched = batched_sweep(hb, hbcases)

    out = {
        "metric": METRIC, "value": ups, "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == hb.HB_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": case.name, "cells": case.nc, "velocities": case.nv, "levels": case.NT,
                   "Kn": case.Kn, "St": case.St, "precision": args.precision},
        "effective_GBps_per_step": step_bytes / (ms_step * 1e-3) / 1e9,
        "effective_frac_per_step": step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "kernel_avg_us": kernels,
        "ms_per_step_with_kernel_events": ms_events,
        "roofline": roof,
        "oracle_error": err,
        "cpu_baseline": cpu,
        "cpu_baseline_1thread": cpu1,
        "converge": conv,
        "correctness_case_full_solve": small,
        "kn_st_sweep": knst,
        "other_workloads": extra,
        "batched": batched,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
