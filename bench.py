"""Benchmark of the boosted-frame EM-PIC step on one MI355X.

Default workload: the large 3D3V boosted-frame laser-wakefield box,
512(z) x 256(x) x 256(y) cells, 16 electrons per cell (537M electrons in the
box), gamma_boost 30, a0 2, split FP32 positions with the FP64 gamma solve.
One step = injection/sort (every 20 steps, amortised), the fused particle
kernel (gather, modified-Lorentz push, move, charge-conserving deposit) and
the Yee update.  Synthetic inputs of the paper's LWFA shape (no dataset).

Prints one JSON line: particle-steps/s of the split-precision path (value),
the plain FP64 path on the same workload and the speedup, serving latency
p50/p99 for a Poisson stream of 2D runs, the roofline fraction of the
particle kernel measured with HIP events, and the CPU oracle timed on a
bounded sample on this host.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (full PIC step) FP32 vs FP64 + p50/p99 batched-run latency"
HBM_PEAK_GBS = 8000.0

# Measured HBM traffic of the particle kernel (rocprofv3 FETCH_SIZE and
# WRITE_SIZE, calibrated against a copy kernel of known size).  It is reported
# only while the kernel sources still hash to the value recorded with it.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_particles_3d_fp32_512x256x256_traffic.txt")
KERNEL_SOURCES = ["paper_0909_5603_amd/csrc/k_step.hip", "paper_0909_5603_amd/csrc/pusher.hpp",
                  "paper_0909_5603_amd/csrc/pic_dev.hpp"]
PARTICLE_KERNEL = "k_particles<3, float,"
COPY_KERNEL = "k_copy_bench"
COPY_BYTES = 1 << 30


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(n_particles: float, n_cells: float, dims: int, rsz: int):
    """Algorithmic HBM bytes per step.  Particle kernel: read + write of the
    particle state (int32 cell, offsets, momenta) plus the gather read of
    E and B and the current write per cell; field kernel: read E, B, J and
    write E, B per cell."""
    part = (4 + dims * rsz + 3 * rsz) * 2
    return {
        "particle_kernel": n_particles * part + n_cells * 9 * rsz,
        "field_kernel": n_cells * 15 * rsz,
        "per_particle": part,
    }


def run_main(cfg, precision, steps, warmup, pic, torch):
    run = pic.Run(cfg, precision)
    d0 = run.diag(pic.PIC_DIAG_PARTICLES)
    log(f"[{precision}] init done: {d0['n_particles']} electrons in the box, "
        f"{run.nbytes / 2**30:.1f} GiB state")
    run.step(warmup)
    run.synchronize()
    t0 = time.perf_counter()
    run.step(steps)
    run.synchronize()
    t1 = time.perf_counter()
    d1 = run.diag(pic.PIC_DIAG_ALL)
    n_box = 0.5 * (d0["n_particles"] + d1["n_particles"])
    sec = t1 - t0
    out = {"ms_per_step": 1e3 * sec / steps, "value": n_box * steps / sec, "n_box": n_box,
           "diag": {k: d1[k] for k in ("step", "U_E", "U_B", "Ez_max", "KE", "n_particles",
                                       "gauss_drift", "err_bits")},
           "slow_path_fraction": d1["n_slow"] / max(1.0, n_box * (steps + warmup))}
    log(f"[{precision}] {out['ms_per_step']:.3f} ms/step, {out['value']:.3e} particle-steps/s, "
        f"slow-path fraction {out['slow_path_fraction']:.2e}")
    return run, out


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def read_traffic(workload: str):
    """HBM bytes per launch of the particle kernel from the committed counter
    summary, or None if there is none or the kernel changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#") and "=" in line:
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_hash() or kv.get("workload") != workload:
        return None
    return float(kv["traffic_bytes_per_launch"])


def _counter_means(path: str, counter: str):
    """Mean counter value per dispatch of the particle and the copy kernel."""
    vals = {PARTICLE_KERNEL: [], COPY_KERNEL: []}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            for k in vals:
                if k in r["Kernel_Name"]:
                    vals[k].append(float(r["Counter_Value"]))
    if not vals[PARTICLE_KERNEL] or not vals[COPY_KERNEL]:
        raise SystemExit(f"{path}: no {counter} samples for both kernels")
    return {k: sum(v) / len(v) for k, v in vals.items()}, {k: len(v) for k, v in vals.items()}


def summarize_traffic(fetch_csv: str, write_csv: str, workload: str, commands: list):
    """Writes the traffic summary from two rocprofv3 --pmc runs (FETCH_SIZE,
    then WRITE_SIZE; KiB per dispatch), each scaled by the reading of the
    same counter for the copy kernel (COPY_BYTES read and written)."""
    f, nf = _counter_means(fetch_csv, "FETCH_SIZE")
    w, nw = _counter_means(write_csv, "WRITE_SIZE")
    kf = COPY_BYTES / (f[COPY_KERNEL] * 1024.0)  # true bytes per counted byte
    kw = COPY_BYTES / (w[COPY_KERNEL] * 1024.0)
    fetch_b = f[PARTICLE_KERNEL] * 1024.0 * kf
    write_b = w[PARTICLE_KERNEL] * 1024.0 * kw
    lines = [
        f"# HBM traffic of {PARTICLE_KERNEL} ({workload})",
        "# rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE (KiB per dispatch), one run each;",
        f"# calibration: {COPY_KERNEL} reading and writing {COPY_BYTES} bytes in the same runs",
        *[f"# command: {c}" for c in commands],
        f"workload = {workload}",
        f"source_sha256 = {kernel_source_hash()}",
        f"dispatches_fetch = {nf[PARTICLE_KERNEL]}",
        f"dispatches_write = {nw[PARTICLE_KERNEL]}",
        f"fetch_kib_per_dispatch = {f[PARTICLE_KERNEL]:.1f}",
        f"write_kib_per_dispatch = {w[PARTICLE_KERNEL]:.1f}",
        f"copy_fetch_kib = {f[COPY_KERNEL]:.1f}",
        f"copy_write_kib = {w[COPY_KERNEL]:.1f}",
        f"fetch_scale = {kf:.4f}",
        f"write_scale = {kw:.4f}",
        f"fetch_bytes_per_launch = {fetch_b:.4e}",
        f"write_bytes_per_launch = {write_b:.4e}",
        f"traffic_bytes_per_launch = {fetch_b + write_b:.6e}",
    ]
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def copy_calibration(pic, torch, reps=3):
    """Launches the plain copy kernel on COPY_BYTES (the counter reference)."""
    a = torch.full((COPY_BYTES,), 1, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    s = torch.cuda.current_stream()
    for _ in range(reps):
        pic.pic_copy_bench(a.data_ptr(), b.data_ptr(), COPY_BYTES, s.cuda_stream)
    torch.cuda.synchronize()
    assert bool((b == 1).all())
    del a, b


def hbm_achievable(pic, torch, nbytes=4 << 30, reps=5):
    """The HBM bandwidth tuned streaming kernels reach on this device (copy,
    read only, write only), timed with events on the stream they run on."""
    a = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    s = torch.cuda.current_stream()
    out = {}
    for mode, name, mult in ((0, "copy", 2), (1, "read", 1), (2, "write", 1)):
        pic.pic_stream_bench(mode, a.data_ptr(), b.data_ptr(), nbytes, s.cuda_stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            pic.pic_stream_bench(mode, a.data_ptr(), b.data_ptr(), nbytes, s.cuda_stream)
        e1.record(s)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[f"{name}_GBs"] = mult * nbytes / (ms * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    out["peak_GBs"] = HBM_PEAK_GBS
    out["copy_frac_of_peak"] = out["copy_GBs"] / HBM_PEAK_GBS
    return out


def kernel_roofline(run, pic, nsteps, workload=None):
    ms = pic.pic_step_timed(run.handle, nsteps)
    slots, live = pic.pic_particle_count(run.handle)
    ncell = run.npts
    rsz = 8 if run.params.precision == pic.PIC_FP64 else 4
    b = algorithmic_bytes(live, ncell, run.params.dims, rsz)
    ach = b["particle_kernel"] / (ms["particles"] * 1e-3) / 1e9
    achf = b["field_kernel"] / (ms["fields"] * 1e-3) / 1e9
    traffic = read_traffic(workload) if (workload and rsz == 4 and run.params.dims == 3) else None
    return ms, {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "k_particles (gather+push+move+deposit)",
                "algorithmic_bytes_per_launch": b["particle_kernel"],
                "bytes_per_particle": b["per_particle"], "particles_per_launch": live,
                "ms_per_launch": ms["particles"],
                "field_kernel": {"achieved": achf, "frac": achf / HBM_PEAK_GBS,
                                 "ms_per_launch": ms["fields"]},
                "sort_ms_per_step": ms["sort"], "step_ms_events": ms["step"]}


def filter_cost(cfg, pic, torch, fields_ms_plain, nsteps=10, passes=1, compensate=1):
    """The same workload with the low-pass current filter (binomial passes plus
    compensation between deposit and field update): step and field-stage
    times, and the filter's own share of the field stage."""
    fcfg = dict(cfg, filter_passes=passes, filter_compensate=compensate)
    run = pic.Run(fcfg, "fp32")
    run.step(5)
    run.synchronize()
    ms = pic.pic_step_timed(run.handle, nsteps)
    naxes = 3 if cfg["dims"] == 3 else 2
    stages = (passes + compensate) * naxes
    npts = run.npts
    run.close()
    del run
    torch.cuda.empty_cache()
    fms = ms["fields"] - fields_ms_plain
    # algorithmic bytes: one launch per axis applies all of that axis's
    # passes; the z launch reads the fixed-point current (3 x 8 B) and writes
    # the filtered one (3 x 4 B), the x and y launches read and write 3 x 4 B
    fbytes = npts * (36 + 24 * (naxes - 1))
    return {"passes": passes, "compensate": compensate, "stages": stages, "launches": naxes,
            "ms_per_step_events": ms["step"], "fields_ms_per_step": ms["fields"],
            "filter_ms_per_step": fms, "filter_GBs": fbytes / (fms * 1e-3) / 1e9 if fms > 0 else None}


def lab_io_cost(cfg, pic, torch, fields_ms_plain, nsteps=10, n_stations=32, stride=4):
    """The same workload with the laboratory-frame input and output switched
    on: the laser emitted by an antenna plane (starting at 3/4 of the box,
    the pulse crossing it during the timed steps) and n_stations lab-fixed
    stations spread over the box, every stride-th transverse node.  Returns
    the field-stage time (where both run) against the plain run's."""
    probe = pic.Run(dict(cfg, ppc=0, nz=16, nx=8, ny=8), "fp32")  # derived quantities only
    d = probe.derived
    probe.close()
    g, b = d["gamma_b"], d["beta_b"]
    Lz = cfg["nz"] * cfg["dz"]
    Za = g * 0.75 * Lz
    lcfg = dict(cfg, laser_antenna=1, antenna_z_lab=Za,
                antenna_t_peak=b * Za + 8.0 * d["dt"] / g,  # the envelope peak after 8 steps
                n_stations=n_stations, station_z0=g * 0.05 * Lz, station_dz=g * 0.9 * Lz / n_stations,
                station_stride=stride, station_cap=64)
    run = pic.Run(lcfg, "fp32")
    run.step(2)
    run.synchronize()
    ms = pic.pic_step_timed(run.handle, nsteps)
    nys, nxs = pic.station_shape(run.params)
    run.close()
    del run
    torch.cuda.empty_cache()
    return {"n_stations": n_stations, "station_points": n_stations * nys * nxs, "antenna": True,
            "ms_per_step_events": ms["step"], "fields_ms_per_step": ms["fields"],
            "lab_io_ms_per_step": ms["fields"] - fields_ms_plain}


def full_run(cfg, pic, torch, passes, compensate, unfiltered=False):
    """The workload's whole configured run (cfg["steps"] steps from t = 0) with
    the current filter (passes + compensation), and on request without it:
    whole-run rate, its fraction of the HBM roofline at the algorithmic bytes
    per particle-step of the whole step (particle state read and written,
    plus 96 B per cell-step over the electrons per cell: 62 B at 16 per
    cell), and the state at the end.  Without a filter the short-wavelength
    instability of the boosted frame grows and heats the plasma, which sends
    electrons through the out-of-window path; the filter is the paper's cure."""
    out = {"steps": cfg["steps"]}
    cases = [("filtered", passes, compensate)] + ([("unfiltered", 0, 0)] if unfiltered else [])
    bps = 56 + 96 / cfg["ppc"]
    for name, fp, fc in cases:
        run = pic.Run(dict(cfg, filter_passes=fp, filter_compensate=fc), "fp32")
        d0 = run.diag(pic.PIC_DIAG_PARTICLES)
        run.synchronize()
        t0 = time.perf_counter()
        run.step(cfg["steps"])
        run.synchronize()
        sec = time.perf_counter() - t0
        d1 = run.diag(pic.PIC_DIAG_FIELDS | pic.PIC_DIAG_PARTICLES)
        run.close()
        del run
        torch.cuda.empty_cache()
        n_box = 0.5 * (d0["n_particles"] + d1["n_particles"])
        rate = n_box * cfg["steps"] / sec
        out[name] = {"filter_passes": fp, "filter_compensate": fc,
                     "value": rate, "ms_per_step": 1e3 * sec / cfg["steps"],
                     "bytes_per_particle_step": bps,
                     "roofline_frac": rate * bps / 1e9 / HBM_PEAK_GBS,
                     "U_E": d1["U_E"], "Ez_max": d1["Ez_max"], "KE": d1["KE"],
                     "slow_path_fraction": d1["n_slow"] / max(1.0, n_box * cfg["steps"])}
    return out


def pusher_cost(pic, torch, nsteps=50, n=1 << 27):
    """Pusher microbenchmark: 2^27 particles, each in its own crossed field
    (E = -v x B, gamma log-uniform in [1e2, 1e6]), one launch per step, the
    modified Lorentz-force (Vay) and Boris pushers in split precision and
    FP64, timed with HIP events on the launching stream.  Bytes per push:
    the position and momentum state read and written plus E, counting the
    int32 cells (76 B in split precision, 128 B in FP64), and what the kernel
    moves when no cell boundary is crossed, without the cells (52 B, 104 B)."""
    from paper_0909_5603_amd import workloads

    u, Ex, B, cell, off = workloads.pusher_set(n, "crossed", seed=2)
    s = torch.cuda.current_stream()
    out = {"particles": n, "steps": nsteps,
           "fields": "crossed, E = -v x B, gamma log-uniform in [1e2, 1e6]"}
    for name, prec, dtype, abytes, kbytes in (("fp32", pic.PIC_FP32_SPLIT, torch.float32, 76, 52),
                                            ("fp64", pic.PIC_FP64, torch.float64, 128, 104)):
        tu = torch.from_numpy(np.ascontiguousarray(u.T)).to("cuda", dtype).reshape(-1)
        tE = torch.from_numpy(Ex).to("cuda", dtype)
        tc = torch.from_numpy(np.ascontiguousarray(cell.T)).to("cuda").reshape(-1)
        to = torch.from_numpy(np.ascontiguousarray(off.T)).to("cuda", dtype).reshape(-1)
        ptrs = (tE.data_ptr(), tu.data_ptr(), tc.data_ptr(), to.data_ptr(), s.cuda_stream)
        for pname, pusher in (("vay", pic.PIC_VAY), ("boris", pic.PIC_BORIS)):
            pic.pic_push_bench(prec, pusher, n, 3, workloads.PUSH_DT, B, *ptrs)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s)
            pic.pic_push_bench(prec, pusher, n, nsteps, workloads.PUSH_DT, B, *ptrs)
            e1.record(s)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / nsteps
            rate = n / (ms * 1e-3)
            out[f"{name}_{pname}"] = {"pushes_per_s": rate, "ms_per_launch": ms,
                                      "GBs_algorithmic": rate * abytes / 1e9,
                                      "frac": rate * abytes / 1e9 / HBM_PEAK_GBS,
                                      "GBs_moved_without_crossings": rate * kbytes / 1e9,
                                      "frac_moved": rate * kbytes / 1e9 / HBM_PEAK_GBS}
        del tu, tE, tc, to
        torch.cuda.empty_cache()
    return out


def serving(pic, torch, n_requests, budget_gib, chunk, depth=2):
    from paper_0909_5603_amd import serve, workloads

    reqs = workloads.serving_stream(n_requests, seed=5)
    res = serve.serve_stream(reqs, budget_bytes=int(budget_gib * 2**30), chunk_steps=chunk, depth=depth)
    res.pop("status", None)
    return res


def c3_record(pic, torch, steps=20, warmup=5, timing_steps=20):
    """The 3D 256x128x128, 8 e-/cell workload (gamma_b 13): whole-step rate
    and the particle kernel's roofline fraction."""
    from paper_0909_5603_amd import workloads

    cfg = workloads.config("c3")
    run, r = run_main(cfg, "fp32", steps, warmup, pic, torch)
    ms, roof = kernel_roofline(run, pic, timing_steps)
    run.close()
    del run
    torch.cuda.empty_cache()
    return {"workload": "3D3V boosted-frame LWFA 256x128x128 cells, 8 e-/cell, gamma_boost 13, a0 2",
            "value": r["value"], "ms_per_step": r["ms_per_step"],
            "roofline_particle_kernel": {k: roof[k] for k in ("achieved", "frac", "ms_per_launch",
                                                               "algorithmic_bytes_per_launch")}}


def host_info():
    """Core count, affinity and CPU model of the host the oracle runs on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else []
    return {"host_cores": os.cpu_count(), "affinity_cores": len(aff),
            "affinity": f"{aff[0]}-{aff[-1]}" if aff else "", "cpu_model": model}


def cpu_baseline_c1(oracle, workloads):
    """The 2D parity workload's whole run (200 steps) in the oracle, 1 thread."""
    cfg = workloads.config("c1")
    st = oracle.State(cfg)
    n0 = st.diag()["n_particles"]
    t0 = time.perf_counter()
    st.step(cfg["steps"])
    sec = time.perf_counter() - t0
    n1 = st.diag()["n_particles"]
    st.close()
    return {"value": 0.5 * (n0 + n1) * cfg["steps"] / sec, "unit": "particle-steps/s", "seconds": sec,
            "sample": f"2D 128x64, 4 e-/cell, gamma_b 5, whole 200-step run"}


def cpu_baseline_c2(oracle, workloads, n=1 << 22, steps=100):
    """The pusher microbenchmark's crossed-field set in the oracle: 2^22
    particles, 100 steps, modified Lorentz-force pusher, 1 thread."""
    import numpy as np

    u, Ex, B, cell, off = workloads.pusher_set(n, "crossed", seed=2)
    E = np.zeros((n, 3))
    E[:, 0] = Ex
    Bn = np.ascontiguousarray(np.tile(B, (n, 1)))
    pos = np.zeros((n, 3))
    oracle.push_many(u[:1024], E[:1024], Bn[:1024], pos[:1024], workloads.PUSH_DT, 1)  # load
    t0 = time.perf_counter()
    oracle.push_many(u, E, Bn, pos, workloads.PUSH_DT, steps)
    sec = time.perf_counter() - t0
    return {"value": n * steps / sec, "unit": "pushes/s", "seconds": sec,
            "sample": f"{n} particles x {steps} steps, crossed fields, gamma 1e2-1e6"}


def cpu_baseline(seconds_target=15.0):
    import oracle
    from paper_0909_5603_amd import workloads

    cfg = workloads.scaled_3d(64, 32, 32, 16)
    st = oracle.State(cfg)
    n_box = st.diag()["n_particles"]
    st.step(1)
    t0 = time.perf_counter()
    steps = 0
    while True:
        st.step(1)
        steps += 1
        if time.perf_counter() - t0 > seconds_target or steps >= 20:
            break
    sec = time.perf_counter() - t0
    st.close()
    out = {"value": n_box * steps / sec, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
           "sample": f"FP64 C oracle, one thread, 3D box 64x32x32 with every other parameter of the "
                     f"512x256x256 workload (16 ppc, {n_box} electrons in the box), {steps} steps, "
                     f"{sec:.1f} s"}
    out.update(host_info())
    out["c1"] = cpu_baseline_c1(oracle, workloads)
    out["c2"] = cpu_baseline_c2(oracle, workloads)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c5", choices=["c5", "c3"])
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-full-run", action="store_true",
                    help="skip the whole configured run (1000 steps) with and without the filter")
    ap.add_argument("--no-pusher", action="store_true",
                    help="skip the 2^27-particle pusher microbenchmark")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-filter", action="store_true",
                    help="skip the run with the low-pass current filter")
    ap.add_argument("--no-lab-io", action="store_true",
                    help="skip the run with the laser antenna and lab-frame stations")
    ap.add_argument("--timing-steps", type=int, default=20)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-chunk", type=int, default=10)
    ap.add_argument("--no-c3", action="store_true", help="skip the 256x128x128, 8 e-/cell record")
    ap.add_argument("--unfiltered", action="store_true",
                    help="also run the whole configured run without the current filter")
    ap.add_argument("--profile", action="store_true",
                    help="only the split-precision timed loop and the copy calibration kernel "
                         "(for rocprofv3 runs)")
    ap.add_argument("--profile-filter", type=int, metavar="PASSES",
                    help="only the workload with the current filter (PASSES binomial passes plus "
                         "compensation): 5 steps, then 10 event-timed steps (for rocprofv3 runs)")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the particle kernel's traffic summary from two rocprofv3 --pmc "
                         "counter_collection.csv files (FETCH_SIZE run, WRITE_SIZE run)")
    ap.add_argument("--commands", nargs="*", default=[],
                    help="with --summarize-traffic: the profiler command lines, recorded in the summary")
    args = ap.parse_args()
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic, workload=args.workload, commands=args.commands)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_0909_5603_amd import pic, workloads

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    pic.lib()
    cfg = workloads.config(args.workload)
    if args.profile_filter is not None:
        fcfg = dict(cfg, filter_passes=args.profile_filter, filter_compensate=1)
        run = pic.Run(fcfg, "fp32")
        run.step(5)
        run.synchronize()
        ms = pic.pic_step_timed(run.handle, 10)
        run.close()
        print(json.dumps({"workload": args.workload, "filter_passes": args.profile_filter,
                          "filter_compensate": 1, "stage_ms_per_step": ms}), flush=True)
        return
    line = {"metric": METRIC, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic"}
    run, r32 = run_main(cfg, "fp32", args.steps, args.warmup, pic, torch)
    line["value"] = r32["value"]
    line["ms_per_step"] = r32["ms_per_step"]
    line["config"] = {
        "workload": (f"3D3V boosted-frame LWFA {cfg['nz']}x{cfg['nx']}x{cfg['ny']} cells, "
                     f"{cfg['ppc']} e-/cell, gamma_boost {cfg['gamma_boost']}, a0 {cfg['a0']}, "
                     f"sort every {cfg['sort_every']} steps; split FP32 positions, FP64 gamma solve"),
        "particles_in_box": r32["n_box"], "cells": cfg["nz"] * cfg["nx"] * cfg["ny"],
        "parallelism": "single GPU",
    }
    ms, roof = kernel_roofline(run, pic, args.timing_steps, args.workload)
    line["roofline"] = roof
    line["diag_fp32"] = r32["diag"]
    line["slow_path_fraction"] = r32["slow_path_fraction"]
    log(f"[fp32] stage ms/step: {ms}; particle kernel {roof['achieved']:.0f} GB/s "
        f"({100 * roof['frac']:.1f}% of HBM peak)")
    run.close()
    del run
    torch.cuda.empty_cache()
    if args.profile:
        copy_calibration(pic, torch)
        print(json.dumps(line), flush=True)
        return
    hb = hbm_achievable(pic, torch)
    line["hbm_achievable"] = hb
    roof["frac_of_achievable_copy"] = roof["achieved"] / hb["copy_GBs"]
    log(f"[hbm] tuned streaming: copy {hb['copy_GBs']:.0f} GB/s, read {hb['read_GBs']:.0f}, "
        f"write {hb['write_GBs']:.0f} (peak {HBM_PEAK_GBS:.0f}); particle kernel at "
        f"{100 * roof['frac_of_achievable_copy']:.1f}% of the tuned copy")
    if not args.no_fp64:
        run64, r64 = run_main(cfg, "fp64", max(args.steps // 2, 10), max(args.warmup // 2, 2), pic, torch)
        ms64, roof64 = kernel_roofline(run64, pic, max(args.timing_steps // 2, 4))
        line["fp64"] = {"value": r64["value"], "ms_per_step": r64["ms_per_step"],
                        "roofline_particle_kernel": {k: roof64[k] for k in ("achieved", "frac", "ms_per_launch")}}
        line["speedup_fp32_vs_fp64"] = r32["value"] / r64["value"]
        run64.close()
        del run64
        torch.cuda.empty_cache()
    if not args.no_filter:
        fc = filter_cost(cfg, pic, torch, ms["fields"])
        line["filter"] = fc
        log(f"[filter] {fc['stages']} one-axis passes in {fc['launches']} launches: {fc['filter_ms_per_step']:.3f} ms/step "
            f"(step {fc['ms_per_step_events']:.3f} ms)")
    if not args.no_lab_io:
        lc = lab_io_cost(cfg, pic, torch, ms["fields"])
        line["lab_io"] = lc
        log(f"[lab io] antenna + {lc['n_stations']} stations: {lc['lab_io_ms_per_step']:.3f} ms/step "
            f"(step {lc['ms_per_step_events']:.3f} ms)")
    if not args.no_full_run:
        fr = full_run(cfg, pic, torch, passes=4, compensate=1, unfiltered=args.unfiltered)
        line["full_run"] = fr
        for k in [k for k in ("filtered", "unfiltered") if k in fr]:
            v = fr[k]
            log(f"[full run, {k}] {fr['steps']} steps: {v['ms_per_step']:.3f} ms/step, "
                f"{v['value']:.3e} particle-steps/s ({100 * v['roofline_frac']:.1f}% of HBM at "
                f"{v['bytes_per_particle_step']:.0f} B), Ez_max {v['Ez_max']:.3g}, "
                f"slow-path fraction {v['slow_path_fraction']:.2e}")
    if not args.no_pusher:
        pc = pusher_cost(pic, torch)
        line["pusher"] = pc
        log("[pusher] 2^27 particles, crossed fields: " + ", ".join(
            f"{k} {v['pushes_per_s']:.3e}/s ({100 * v['frac']:.0f}%)" for k, v in pc.items()
            if isinstance(v, dict)))
    if not args.no_c3 and args.workload == "c5":
        c3 = c3_record(pic, torch)
        line["c3"] = c3
        log(f"[c3] {c3['value']:.3e} particle-steps/s, particle kernel "
            f"{100 * c3['roofline_particle_kernel']['frac']:.1f}% of HBM")
    if not args.no_serving:
        res = serving(pic, torch, args.serve_requests, budget_gib=96.0, chunk=args.serve_chunk)
        line["serving"] = res
        log(f"[serving] {res['n_requests']} requests ({res['n_rejected']} rejected, {res['n_failed']} failed): "
            f"p50 {res['p50_ms']:.1f} ms, p99 {res['p99_ms']:.1f} ms, {res['throughput']:.3e} particle-steps/s "
            f"(offered {res['offered_load']:.3e})")
    if not args.no_cpu:
        cb = cpu_baseline()
        line["cpu_baseline"] = cb
        log(f"[cpu] oracle {cb['value']:.3e} particle-steps/s (C5 sample), C1 {cb['c1']['value']:.3e} "
            f"particle-steps/s, C2 {cb['c2']['value']:.3e} pushes/s; {cb['cpu_model']}, "
            f"{cb['host_cores']} cores, {cb['affinity_cores']} in the affinity mask")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
