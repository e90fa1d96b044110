"""Benchmark of the Rydberg state-vector hot path on one MI355X.

Workload: the 27-atom random register (30x30 um box, 5 um minimum distance, seed 0) under
the adiabatic sweep (0.5 us ramps around a 3 us plateau, Omega_max and delta_max drawn from
U[2pi, 2pi*3] rad/us), dt = 10 ns, tolerance 1e-10 (complex128) / 1e-7 (complex64).

A step is one time step of eq. (6): the Lanczos Krylov exponential (H psi passes, FP64
reductions, host tridiagonal exponential) and the Krylov combination.  W untimed steps run
first (steps 0..W-1 from |0...0>), then K steps are timed (steps W..W+K-1).  Reported:
  value      simulated microseconds per wall second of the complex128 path (whole job, state
             resident in HBM),
  roofline   H psi (the dominant operation) at the step-300 parameters: algorithmic bytes
             (40 B/amplitude c128: state in, diagonal, state out) / average duration from HIP
             events on the launch stream; the kernels form the diagonal on chip, so their
             compulsory traffic is 32 B/amplitude (reported beside it),
  c64        the same for complex64 storage with FP64 Lanczos scalars, plus its infidelity
             against the complex128 result of the same steps,
  cpu_baseline  the CPU oracle's H psi at the same size, scaled to sim-us/s.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "H*psi HBM GB/s + sim-us/sec at N=27; served solves/s, p50/p99 at fidelity 1e-6"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def hpsi_time(rsv, reg, pulses, step, dt_ns, n, prec, reps=30, warm=5):
    import torch
    dt = torch.complex128 if prec == "c128" else torch.complex64
    g = torch.Generator(device="cuda:0").manual_seed(42)
    x = torch.randn(1 << n, dtype=dt, device="cuda:0", generator=g)
    x /= torch.linalg.vector_norm(x)
    y = torch.empty_like(x)
    for _ in range(warm):
        rsv.rsv_apply_hamiltonian(reg, pulses, step, dt_ns, x, y)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        rsv.rsv_apply_hamiltonian(reg, pulses, step, dt_ns, x, y)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    return ms


def copy_gbps(n_bytes=1 << 31, reps=20):
    """A plain device-to-device copy of n_bytes: the practical HBM ceiling (read + write)."""
    import torch
    x = torch.empty(n_bytes // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    y = torch.empty_like(x)
    y.copy_(x)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        y.copy_(x)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    return 2.0 * n_bytes / (ms * 1e-3) / 1e9, ms


def evolve_timed(rsv, ctx, w, prec, warmup, steps):
    import torch
    t_reg = time.perf_counter()
    reg = rsv.rsv_register_create(ctx, w.xyz, w.c6, prec)  # U and the diagonal tables (synchronous)
    evolve_timed.register_ms = (time.perf_counter() - t_reg) * 1e3
    pulses = rsv.PulseArrays(w.omega, w.delta)
    dt = torch.complex128 if prec == "c128" else torch.complex64
    psi = torch.zeros(1 << w.n_atoms, dtype=dt, device="cuda:0")
    psi[0] = 1
    tol = w.tol if prec == "c128" else 1e-7
    st_w = rsv.rsv_evolve_device(reg, pulses, rsv.evolve_opts(w.dt_ns, tol, w.kmax, 12, 0, warmup), psi)
    log(f"{prec}: warmup {warmup} steps in {st_w.seconds:.2f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = rsv.rsv_evolve_device(reg, pulses, rsv.evolve_opts(w.dt_ns, tol, w.kmax, 12, warmup, steps), psi)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"{prec}: {steps} steps in {wall:.3f} s, {st.krylov_iters} Krylov iterations")
    return reg, psi, st, wall


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def serving_leg(rsv, wl, ctx, n_jobs, lanes):
    """Mixed-size serving stream (N ~ U{12..24}, random registers and piecewise-linear
    pulses, complex64 with FP64 reductions, tol 1e-7): the sequential complex128 plain path
    gives the service times mu_seq and the FP64 reference states; the server then takes the
    same jobs at Poisson arrivals of rate 2 mu_seq.  Sequential latencies replay the same
    arrival trace against the measured sequential service times."""
    jobs = wl.serving_stream(n_jobs, seed=0)
    ref, service = [], []
    for w in jobs:
        reg = rsv.rsv_register_create(ctx, w.xyz, w.c6, "c128")
        t0 = time.perf_counter()
        res = rsv.rsv_evolve(reg, rsv.PulseArrays(w.omega, w.delta),
                             rsv.evolve_opts(w.dt_ns, 1e-10, w.kmax, 12))
        rsv.rsv_result_occupations(res, w.n_atoms)
        service.append(time.perf_counter() - t0)
        ref.append(rsv.rsv_result_state(res, w.n_atoms))
        rsv.rsv_result_destroy(res)
        rsv.rsv_register_destroy(reg)
    mu_seq = len(jobs) / sum(service)
    log(f"serving: sequential complex128 plain path {mu_seq:.2f} solves/s over {len(jobs)} jobs")
    rate = 2.0 * mu_seq
    arrivals = wl.poisson_arrivals(len(jobs), rate, seed=1)
    seq_lat, t_free = [], 0.0
    for a, s in zip(arrivals, service):
        t_free = max(t_free, a) + s
        seq_lat.append(t_free - a)

    arena = 2 * sum(sorted(rsv.rsv_server_job_bytes(w.n_atoms, w.kmax, "c64", 0) for w in jobs)[-lanes:])
    srv = rsv.rsv_server_create(ctx, n_lanes=lanes, arena_bytes=arena, pack_max_atoms=13)
    done = []
    try:
        pulses = [rsv.PulseArrays(w.omega, w.delta) for w in jobs]
        t_start = time.perf_counter()
        for i, w in enumerate(jobs):
            while time.perf_counter() - t_start < arrivals[i]:
                done += rsv.rsv_server_poll(srv, 64, 1)
            rsv.rsv_server_submit(srv, w.xyz, w.c6, pulses[i], rsv.evolve_opts(w.dt_ns, w.tol, w.kmax, 12),
                                  "c64", return_state=True, tag=i)
        while len(done) < len(jobs):
            done += rsv.rsv_server_poll(srv, 64, 1000)
    finally:
        rsv.rsv_server_destroy(srv)
    bad = [c for c in done if c["status"] != 0]
    assert not bad, bad[0]["error"]
    lat = [c["t_end"] - c["t_submit"] for c in done]
    span = max(c["t_end"] for c in done) - min(c["t_submit"] for c in done)
    infid = []
    for c in done:
        a, b = ref[c["tag"]], c["state"]
        a = a / np.linalg.norm(a)
        b = b / np.linalg.norm(b)
        r = b - np.vdot(a, b) * a
        infid.append(float(np.vdot(r, r).real))
    seq_span = t_free - arrivals[0]
    out = {
        "jobs": len(jobs), "lanes": lanes, "arrival_rate_per_s": round(rate, 3),
        "n_atoms": [int(w.n_atoms) for w in jobs],
        "served_solves_per_s": round(len(jobs) / span, 3),
        "served_p50_s": round(percentile(lat, 50), 4), "served_p99_s": round(percentile(lat, 99), 4),
        "sequential_c128_solves_per_s": round(len(jobs) / seq_span, 3),
        "sequential_c128_service_solves_per_s": round(mu_seq, 3),
        "sequential_p50_s": round(percentile(seq_lat, 50), 4),
        "sequential_p99_s": round(percentile(seq_lat, 99), 4),
        "max_infidelity_vs_c128": max(infid),
        "packed_jobs": sum(1 for w in jobs if w.n_atoms <= 13),
        "precision": "c64 state, FP64 reductions, tol 1e-7",
    }
    log(f"serving: {out['served_solves_per_s']} solves/s, p50 {out['served_p50_s']} s, "
        f"p99 {out['served_p99_s']} s; max infidelity {out['max_infidelity_vs_c128']:.2e}")
    return out


def small_job_leg(rsv, wl, ctx, n_jobs, lanes):
    """Saturation throughput of small jobs (N ~ U{6..13}, otherwise the serving-stream
    recipe, complex64, tol 1e-7), all queued at t = 0: one server packs them (one workgroup
    per job, one launch per batch), another runs each on the plain host-driven path.  Every
    packed state is compared with the plain path's."""
    jobs = wl.serving_stream(n_jobs, seed=2, n_min=6, n_max=13)
    res = {}
    for mode, pack in (("plain", 0), ("packed", 13)):
        srv = rsv.rsv_server_create(ctx, n_lanes=lanes, arena_bytes=4 << 30, pack_max_atoms=pack)
        try:
            t0 = time.perf_counter()
            for i, w in enumerate(jobs):
                rsv.rsv_server_submit(srv, w.xyz, w.c6, rsv.PulseArrays(w.omega, w.delta),
                                      rsv.evolve_opts(w.dt_ns, w.tol, w.kmax, 12), "c64",
                                      return_state=True, tag=i)
            done = []
            while len(done) < len(jobs):
                done += rsv.rsv_server_poll(srv, 256, 1000)
            span = time.perf_counter() - t0
        finally:
            rsv.rsv_server_destroy(srv)
        bad = [c for c in done if c["status"] != 0]
        assert not bad, bad[0]["error"]
        res[mode] = ({c["tag"]: c["state"] for c in done}, span)
    infid = []
    for i in range(len(jobs)):
        a, b = res["plain"][0][i], res["packed"][0][i]
        a = a / np.linalg.norm(a)
        b = b / np.linalg.norm(b)
        r = b - np.vdot(a, b) * a
        infid.append(float(np.vdot(r, r).real))
    out = {"jobs": len(jobs), "n_atoms": "6..13", "lanes": lanes,
           "plain_solves_per_s": round(len(jobs) / res["plain"][1], 2),
           "packed_solves_per_s": round(len(jobs) / res["packed"][1], 2),
           "max_infidelity_packed_vs_plain": max(infid)}
    log(f"small jobs: plain {out['plain_solves_per_s']} solves/s, packed "
        f"{out['packed_solves_per_s']} solves/s, max infidelity {max(infid):.2e}")
    return out


# Sources the H psi kernels are compiled from; their digest ignores comments and blank lines.
HPSI_SOURCES = ("hpsi.hip", "device_common.h", "rsv_internal.h")


def hpsi_code_digest(read=None):
    """sha256 over the H psi kernel sources with // comments and blank lines removed;
    read(name) -> text (default: the working tree)."""
    if read is None:
        def read(name):
            return open(os.path.join(ROOT, "paper_2510_09813_amd", "csrc", name)).read()
    h = hashlib.sha256()
    for name in HPSI_SOURCES:
        for line in read(name).splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()


def pmc_traffic(prec):
    """HBM bytes per H psi application from the committed rocprofv3 counter summary, if it
    was taken on the current kernel code."""
    path = os.path.join(ROOT, "profiles", f"hpsi_random27_{prec}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("hpsi_code_sha256") != hpsi_code_digest():
        return None
    return rec.get("bytes_per_application")


def cpu_baseline(w, iters_per_step, budget_s=20.0):
    """The oracle on the host: rows (H psi)_b of the N = 27 H|psi> at the step-300
    parameters, evaluated one by one from the matrix elements (the oracle's form that works
    at this size), timed for about budget_s; the time per row scales to one H|psi>
    (2^27 rows) and, with the GPU run's H|psi> count per step, to simulated us per second.
    The oracle's Lanczos re-orthogonalisation and combination are not counted."""
    from oracle import model
    n = w.n_atoms
    rng = np.random.default_rng(42)
    psi = (rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)).astype(np.complex128)
    u = model.interaction_matrix(w.xyz, w.c6)
    pars = model.step_parameters(n, w.omega, w.delta, None, w.dt_ns, 300)
    rows = rng.integers(0, 1 << n, 200000)
    t0 = time.perf_counter()
    done = 0
    while done < rows.size and time.perf_counter() - t0 < budget_s:
        for b in rows[done:done + 500]:
            model.hamiltonian_row(int(b), psi, u, *pars)
        done += 500
    t_row = (time.perf_counter() - t0) / done
    t_apply = t_row * (1 << n)
    step_s = t_apply * iters_per_step
    return {
        "value": w.dt_ns * 1e-3 / step_s, "unit": "sim-us/s", "cores": 1, "kind": "oracle",
        "sample": (f"{done} rows of the N={n} H|psi> (random rows, step-300 parameters) from the "
                   f"oracle's per-row form, {t_row * 1e6:.1f} us per row on 1 host thread; "
                   f"scaled to 2^{n} rows per H|psi> and the GPU run's {iters_per_step:.2f} "
                   f"H|psi> per step; re-orthogonalisation and combination not counted"),
        "hpsi_seconds_extrapolated": t_apply,
        "host_cpus": len(os.sched_getaffinity(0)),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-c64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=40,
                    help="jobs of the mixed-size serving stream (0: skip the serving leg)")
    ap.add_argument("--lanes", type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the state vector of one job lives on one MI355X; "
              "see the design notes for how the path would shard across GPUs", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2510_09813_amd import rsv
    from paper_2510_09813_amd import workloads as wl
    torch.cuda.set_device(0)
    w = wl.random27()
    n = w.n_atoms
    K, W = args.steps, args.warmup
    if W + K > w.n_steps:
        raise SystemExit(f"warmup + steps must be <= {w.n_steps}")
    ctx = rsv.rsv_ctx_create(0)

    t0 = time.perf_counter()
    cp_gbs, cp_ms = copy_gbps()
    log(f"device copy of 2 GiB: {cp_ms:.3f} ms = {cp_gbs:.0f} GB/s (read + write)")
    reg128, psi128, st128, wall128 = evolve_timed(rsv, ctx, w, "c128", W, K)
    sim_us = K * w.dt_ns * 1e-3
    iters_per_step = st128.krylov_iters / K

    pulses = rsv.PulseArrays(w.omega, w.delta)
    ms128 = hpsi_time(rsv, reg128, pulses, 300, w.dt_ns, n, "c128")
    gbs128 = 40.0 * (1 << n) / (ms128 * 1e-3) / 1e9
    log(f"c128 H|psi>: {ms128:.3f} ms = {gbs128:.0f} GB/s algorithmic")
    occ = rsv.rsv_occupations_device(ctx, n, psi128, "c128")
    shots = rsv.rsv_sample_device(ctx, n, psi128, 0, 1000, "c128")
    out = {
        "metric": METRIC, "value": round(sim_us / wall128, 4), "unit": "sim-us/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": round(wall128 / K * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "random27-sweep", "n_atoms": n, "amplitudes": 1 << n,
                   "dt_ns": w.dt_ns, "tol": w.tol, "kmax": w.kmax,
                   "timed_steps": f"{W}..{W + K - 1} of {w.n_steps}", "precision": "complex128"},
        "krylov_iters_per_step": round(iters_per_step, 3),
        "krylov_max": int(st128.krylov_max),
        "hpsi_ms": round(ms128, 4), "hpsi_gbps": round(gbs128, 1),
        "roofline": {"bound": "hbm", "achieved": round(gbs128, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(gbs128 / PEAK_HBM_GBS, 4),
                     "kernel": "H|psi> at N=27 complex128 (high passes + low pass)",
                     "bytes_per_amplitude": 40,
                     # the state in and out only: E_b is formed on chip from small tables
                     "compulsory_bytes_per_amplitude": 32,
                     "achieved_compulsory": round(gbs128 * 32 / 40, 1),
                     "traffic": pmc_traffic("c128")},
        "register_build_ms": round(evolve_timed.register_ms, 3),
        "occupations_sum": round(float(occ.sum()), 6), "n_shots": len(shots),
        "device_copy_gbps": round(cp_gbs, 1),
    }
    rsv.rsv_register_destroy(reg128)

    if not args.no_c64:
        reg64, psi64, st64, wall64 = evolve_timed(rsv, ctx, w, "c64", W, K)
        ms64 = hpsi_time(rsv, reg64, pulses, 300, w.dt_ns, n, "c64")
        a = psi128.cpu().numpy()
        b = psi64.cpu().numpy().astype(np.complex128)
        a /= np.linalg.norm(a)
        b /= np.linalg.norm(b)
        r = b - np.vdot(a, b) * a
        infid = float(np.vdot(r, r).real)
        occ64 = rsv.rsv_occupations_device(ctx, n, psi64, "c64")
        out["c64"] = {
            "sim_us_per_s": round(sim_us / wall64, 4), "ms_per_step": round(wall64 / K * 1e3, 3),
            "hpsi_ms": round(ms64, 4), "hpsi_gbps": round(20.0 * (1 << n) / (ms64 * 1e-3) / 1e9, 1),
            "hpsi_frac": round(20.0 * (1 << n) / (ms64 * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
            "infidelity_vs_c128": infid, "max_occ_err_vs_c128": float(np.abs(occ64 - occ).max()),
            "krylov_iters_per_step": round(st64.krylov_iters / K, 3),
            "traffic": pmc_traffic("c64"),
        }
        rsv.rsv_register_destroy(reg64)
        del psi64
    del psi128
    torch.cuda.empty_cache()
    if args.serve_jobs > 0:
        out["serving"] = serving_leg(rsv, wl, ctx, args.serve_jobs, args.lanes)
        out["serving"]["small_jobs"] = small_job_leg(rsv, wl, ctx, 4 * args.serve_jobs, args.lanes)
    rsv.rsv_ctx_destroy(ctx)

    if not args.no_cpu:
        log("cpu baseline: oracle H|psi> at N=27 ...")
        out["cpu_baseline"] = cpu_baseline(w, iters_per_step)
    log(f"total {time.perf_counter() - t0:.1f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
