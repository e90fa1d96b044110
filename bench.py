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
  n30_c64    the 30-atom triangular quench in complex64: ms per step and workspace,
  serving    the mixed-size stream: saturation solves/s, steady-state p50/p99 at 0.8 x
             saturation, the sequential complex128 plain path's rate and latencies, and the
             infidelity and occupation error of every served result against complex128,
             and a shot-to-shot noise ensemble (512 members of the 10-atom chain),
  lindblad   the Liouvillian on a 12-atom density matrix (GB/s) and Arnoldi steps,
  gradient   pulse gradients at 20 atoms against the forward evolution's time,
  cpu_baseline  one time step of the CPU oracle, scaled to sim-us/s at 27 atoms.
Every leg logs its progress to stderr at least every 20 s.
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

    def run(first, count, what):
        # calls of at most 50 steps (stepping is Markov: (k, psi_k) resumes exactly), each
        # followed by a progress line
        iters, kmax = 0, 0
        for f in range(first, first + count, 50):
            c = min(50, first + count - f)
            st = rsv.rsv_evolve_device(reg, pulses, rsv.evolve_opts(w.dt_ns, tol, w.kmax, 12, f, c), psi)
            iters += st.krylov_iters
            kmax = max(kmax, st.krylov_max)
            log(f"{prec} {what}: steps {f}..{f + c - 1} done")
        return iters, kmax

    run(0, warmup, "warmup")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, kmax = run(warmup, steps, "timed")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"{prec}: {steps} steps in {wall:.3f} s, {iters} Krylov iterations")
    return reg, psi, {"krylov_iters": iters, "krylov_max": kmax}, wall


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


class Progress:
    """A line on stderr at most every `every` seconds from inside long loops."""

    def __init__(self, what, every=20.0):
        self.what, self.every, self.t = what, every, time.perf_counter()

    def __call__(self, msg):
        now = time.perf_counter()
        if now - self.t >= self.every:
            log(f"{self.what}: {msg}")
            self.t = now


def infidelity(a, b):
    a = a / np.linalg.norm(a)
    b = b / np.linalg.norm(b)
    r = b - np.vdot(a, b) * a
    return float(np.vdot(r, r).real)


def occupations_of(psi):
    """<n_i> of a host state (atom 0 = most significant bit): only used to report the
    occupation error of served results against the complex128 results."""
    p = np.abs(psi) ** 2
    n = int(round(np.log2(p.size)))
    t = p.reshape((2,) * n)
    return np.array([np.take(t, 1, axis=i).sum() for i in range(n)]) / p.sum()


def serve_jobs(rsv, ctx, jobs, lanes, arena, arrivals=None, return_state=True):
    """Runs jobs through one server (complex64, jobs of <= 13 atoms packed); arrivals[i] is
    job i's submission time in seconds from the start (None: all at once).  Returns the
    completions and the wall span from the first submission to the last completion."""
    srv = rsv.rsv_server_create(ctx, n_lanes=lanes, arena_bytes=arena, pack_max_atoms=13)
    done, prog = [], Progress("serving")
    try:
        pulses = [rsv.PulseArrays(w.omega, w.delta) for w in jobs]
        t_start = time.perf_counter()
        for i, w in enumerate(jobs):
            if arrivals is not None:
                while time.perf_counter() - t_start < arrivals[i]:
                    done += rsv.rsv_server_poll(srv, 64, 1)
                    prog(f"{len(done)} of {len(jobs)} done, {i} submitted")
            rsv.rsv_server_submit(srv, w.xyz, w.c6, pulses[i],
                                  rsv.evolve_opts(w.dt_ns, w.tol, w.kmax, 12), "c64",
                                  return_state=return_state, tag=i)
        while len(done) < len(jobs):
            done += rsv.rsv_server_poll(srv, 64, 1000)
            prog(f"{len(done)} of {len(jobs)} done")
    finally:
        rsv.rsv_server_destroy(srv)
    bad = [c for c in done if c["status"] != 0]
    assert not bad, bad[0]["error"]
    span = max(c["t_end"] for c in done) - min(c["t_submit"] for c in done)
    return sorted(done, key=lambda c: c["tag"]), span


def serving_leg(rsv, wl, ctx, n_jobs, lanes):
    """Mixed-size serving stream: the first n_jobs jobs of the 2000-job recipe (N ~
    U{12..24}, random registers and piecewise-linear pulses, complex64 with FP64
    reductions, tol 1e-7; job i's inputs do not depend on n_jobs).
      1. the sequential complex128 plain path, job after job: its service rate and the FP64
         reference state and occupations of every job;
      2. saturation: every job submitted at t = 0 to the server, served solves/s;
      3. steady state: Poisson arrivals at 0.8 x the saturation throughput, served p50/p99
         latency, and the sequential path's latency on the same arrival trace (replayed
         against its measured service times).
    Every served result of runs 2 and 3 is compared with its complex128 result."""
    jobs = wl.serving_stream(n_jobs, seed=0)
    ref, ref_occ, service = [], [], []
    prog = Progress("serving reference")
    for i, w in enumerate(jobs):
        reg = rsv.rsv_register_create(ctx, w.xyz, w.c6, "c128")
        t0 = time.perf_counter()
        res = rsv.rsv_evolve(reg, rsv.PulseArrays(w.omega, w.delta),
                             rsv.evolve_opts(w.dt_ns, 1e-10, w.kmax, 12))
        ref_occ.append(rsv.rsv_result_occupations(res, w.n_atoms))
        service.append(time.perf_counter() - t0)
        ref.append(rsv.rsv_result_state(res, w.n_atoms))
        rsv.rsv_result_destroy(res)
        rsv.rsv_register_destroy(reg)
        prog(f"{i + 1} of {len(jobs)} jobs")
    mu_seq = len(jobs) / sum(service)
    log(f"serving: sequential complex128 plain path {mu_seq:.2f} solves/s over {len(jobs)} jobs")

    arena = 2 * sum(sorted(rsv.rsv_server_job_bytes(w.n_atoms, w.kmax, "c64", 0) for w in jobs)[-lanes:])
    sat, sat_span = serve_jobs(rsv, ctx, jobs, lanes, arena)
    capacity = len(jobs) / sat_span
    log(f"serving: saturation {capacity:.3f} solves/s (all {len(jobs)} jobs at t = 0)")
    rate = 0.8 * capacity
    arrivals = wl.poisson_arrivals(len(jobs), rate, seed=1)
    arrivals = arrivals - arrivals[0]
    steady, span = serve_jobs(rsv, ctx, jobs, lanes, arena, arrivals)
    lat = [c["t_end"] - c["t_submit"] for c in steady]
    wait = [c["t_start"] - c["t_submit"] for c in steady]
    seq_lat, t_free = [], 0.0
    for a, s_ in zip(arrivals, service):
        t_free = max(t_free, a) + s_
        seq_lat.append(t_free - a)

    def errors(done):
        inf = [infidelity(ref[c["tag"]], c["state"]) for c in done]
        docc = [float(np.abs(c["occupations"] - ref_occ[c["tag"]]).max()) for c in done]
        return inf, docc

    inf_sat, docc_sat = errors(sat)
    inf_st, docc_st = errors(steady)
    out = {
        "config": {"jobs": len(jobs), "of_stream": 2000, "n_atoms": "12..24", "lanes": lanes,
                   "precision": "c64 state, FP64 reductions, tol 1e-7; jobs <= 13 atoms packed",
                   "reference": "sequential complex128 plain path, tol 1e-10"},
        "n_atoms": [int(w.n_atoms) for w in jobs],
        "saturation_solves_per_s": round(capacity, 3),
        "arrival_rate_per_s": round(rate, 3),
        "served_solves_per_s": round(len(jobs) / span, 3),
        "served_p50_s": round(percentile(lat, 50), 4), "served_p99_s": round(percentile(lat, 99), 4),
        "served_queue_wait_p50_s": round(percentile(wait, 50), 4),
        "served_queue_wait_p99_s": round(percentile(wait, 99), 4),
        "sequential_c128_service_solves_per_s": round(mu_seq, 3),
        "sequential_p50_s": round(percentile(seq_lat, 50), 4),
        "sequential_p99_s": round(percentile(seq_lat, 99), 4),
        "max_infidelity_vs_c128": max(inf_sat + inf_st),
        "max_occ_err_vs_c128": max(docc_sat + docc_st),
        "per_job_infidelity": [float(f"{x:.3g}") for x in inf_sat],
        "per_job_max_occ_err": [float(f"{x:.3g}") for x in docc_sat],
        "packed_jobs": sum(1 for w in jobs if w.n_atoms <= 13),
    }
    log(f"serving: steady state at {rate:.3f}/s: {out['served_solves_per_s']} solves/s, p50 "
        f"{out['served_p50_s']} s, p99 {out['served_p99_s']} s; max infidelity "
        f"{out['max_infidelity_vs_c128']:.2e}")
    return out


def serving_full(rsv, wl, ctx, n_jobs, rate, lanes):
    """The whole serving stream (n_jobs of the N ~ U{12..24} recipe, complex64, jobs of <= 13
    atoms packed) at Poisson arrivals of the given rate: served solves/s, latency and queue
    wait percentiles, overall and by register size.  No complex128 reference here: the
    precision of served results is measured on the stream's prefix by the default run."""
    jobs = wl.serving_stream(n_jobs, seed=0)
    arrivals = wl.poisson_arrivals(len(jobs), rate, seed=1)
    arrivals = arrivals - arrivals[0]
    arena = 2 * sum(sorted(rsv.rsv_server_job_bytes(w.n_atoms, w.kmax, "c64", 0) for w in jobs)[-lanes:])
    done, span = serve_jobs(rsv, ctx, jobs, lanes, arena, arrivals, return_state=False)
    lat = [c["t_end"] - c["t_submit"] for c in done]
    wait = [c["t_start"] - c["t_submit"] for c in done]
    by_n = {}
    for w, c in zip(jobs, done):
        by_n.setdefault(int(w.n_atoms), []).append(c["t_end"] - c["t_submit"])
    return {
        "jobs": len(jobs), "lanes": lanes, "arrival_rate_per_s": rate,
        "precision": "c64 state, FP64 reductions, tol 1e-7; jobs <= 13 atoms packed",
        "served_solves_per_s": round(len(jobs) / span, 3), "span_s": round(span, 2),
        "served_p50_s": round(percentile(lat, 50), 4), "served_p99_s": round(percentile(lat, 99), 4),
        "queue_wait_p50_s": round(percentile(wait, 50), 4),
        "queue_wait_p99_s": round(percentile(wait, 99), 4),
        "p50_by_n_atoms": {n: round(percentile(v, 50), 4) for n, v in sorted(by_n.items())},
        "sim_us_served": round(sum(w.t_ns for w in jobs) * 1e-3, 1),
    }


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
            done, prog = [], Progress(f"small jobs ({mode})")
            while len(done) < len(jobs):
                done += rsv.rsv_server_poll(srv, 256, 1000)
                prog(f"{len(done)} of {len(jobs)} done")
            span = time.perf_counter() - t0
        finally:
            rsv.rsv_server_destroy(srv)
        bad = [c for c in done if c["status"] != 0]
        assert not bad, bad[0]["error"]
        res[mode] = ({c["tag"]: c["state"] for c in done}, span)
    infid = [infidelity(res["plain"][0][i], res["packed"][0][i]) for i in range(len(jobs))]
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


def ensemble_leg(rsv, wl, ctx, members, lanes):
    """Shot-to-shot noise ensemble of the 10-atom chain (constant drive, 1 us, dt = 10 ns):
    `members` noisy copies (5 % drive amplitude, 2pi x 0.25 rad/us detuning per atom, 150 nm
    positions), complex64, one shot each, packed by the server."""
    w = wl.chain10()
    srv = rsv.rsv_server_create(ctx, n_lanes=lanes, arena_bytes=2 << 30, pack_max_atoms=13)
    try:
        t0 = time.perf_counter()
        rsv.rsv_server_submit_ensemble(srv, w.xyz, w.c6, rsv.PulseArrays(w.omega, w.delta),
                                       rsv.evolve_opts(w.dt_ns, 1e-7, w.kmax, 12),
                                       (0.05, 2 * np.pi * 0.25, 0.15), 9, members, "c64",
                                       n_shots=1, seed=0)
        done, prog = [], Progress("ensemble")
        while len(done) < members:
            done += rsv.rsv_server_poll(srv, 256, 1000)
            prog(f"{len(done)} of {members} done")
        span = time.perf_counter() - t0
    finally:
        rsv.rsv_server_destroy(srv)
    assert all(c["status"] == 0 for c in done), done[0]["error"]
    occ = np.mean([c["occupations"] for c in done], axis=0)
    out = {"workload": "chain10 with shot-to-shot noise", "members": members,
           "noise": {"omega_rel_sigma": 0.05, "delta_sigma_rad_per_us": 2 * np.pi * 0.25,
                     "position_sigma_um": 0.15},
           "precision": "complex64, packed", "member_solves_per_s": round(members / span, 2),
           "ensemble_mean_occupations": [round(float(x), 5) for x in occ]}
    log(f"ensemble: {members} members in {span:.2f} s ({out['member_solves_per_s']} solves/s)")
    return out


def lindblad_leg(rsv, wl, ctx, n, steps):
    """The Lindblad master equation on the random-register sweep recipe at n atoms
    (relaxation 0.5/us, dephasing 1/us per atom, complex128, density matrix of 4^n
    amplitudes): the Liouvillian application timed with HIP events (algorithmic bytes: the
    density matrix read once and written once, 32 B per element), then `steps` plateau
    steps of the Arnoldi evolution from |0...0><0...0|."""
    import torch
    w = wl.random27(n_atoms=n)
    rates = (0.5, 1.0)
    pulses = rsv.PulseArrays(w.omega, w.delta)
    reg = rsv.rsv_register_create(ctx, w.xyz, w.c6, "c128")
    g = torch.Generator(device="cuda:0").manual_seed(7)
    x = torch.randn(1 << (2 * n), dtype=torch.complex128, device="cuda:0", generator=g)
    y = torch.empty_like(x)
    for _ in range(3):
        rsv.rsv_lindblad_apply(reg, pulses, 200, w.dt_ns, rates, x, y)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(20):
        rsv.rsv_lindblad_apply(reg, pulses, 200, w.dt_ns, rates, x, y)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 20
    rho = torch.zeros_like(x)
    rho[0] = 1
    del x, y
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = rsv.rsv_lindblad_evolve_device(reg, pulses, rsv.evolve_opts(w.dt_ns, 1e-10, 40, 12, 200, steps),
                                        rates, rho)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    occ, tr = rsv.rsv_lindblad_occupations(ctx, n, rho, "c128")
    rsv.rsv_register_destroy(reg)
    del rho
    torch.cuda.empty_cache()
    elems = 1 << (2 * n)
    out = {"workload": f"random{n}-sweep, Lindblad (relaxation 0.5/us, dephasing 1/us)",
           "n_atoms": n, "density_matrix_elements": elems, "precision": "complex128",
           "liouvillian_ms": round(ms, 4),
           "liouvillian_gbps": round(32.0 * elems / (ms * 1e-3) / 1e9, 1),
           "steps": steps, "ms_per_step": round(wall / steps * 1e3, 2),
           "arnoldi_iters_per_step": round(st.krylov_iters / steps, 2), "substeps": int(st.substeps),
           "trace": tr, "occupations_sum": round(float(occ.sum()), 6)}
    log(f"lindblad N={n}: L rho {ms:.3f} ms ({out['liouvillian_gbps']} GB/s on 32 B/element), "
        f"{steps} steps in {wall:.2f} s")
    return out


def gradient_leg(rsv, wl, ctx, n, steps):
    """Pulse gradients of sum_i <n_i> on the random-register sweep recipe at n atoms over
    `steps` plateau steps (complex128, tol 1e-10): wall time against the forward evolution of
    the same window."""
    import torch
    w = wl.random27(n_atoms=n)
    pulses = rsv.PulseArrays(w.omega, w.delta)
    reg = rsv.rsv_register_create(ctx, w.xyz, w.c6, "c128")
    opts = rsv.evolve_opts(w.dt_ns, 1e-10, 40, 12, 200, steps)
    psi = torch.zeros(1 << n, dtype=torch.complex128, device="cuda:0")
    psi[0] = 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rsv.rsv_evolve_device(reg, pulses, opts, psi)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    c, go, gd, st = rsv.rsv_gradient_occupations(reg, pulses, opts, np.ones(n))
    t_grad = time.perf_counter() - t0
    rsv.rsv_register_destroy(reg)
    out = {"workload": f"random{n}-sweep, d(sum <n_i>)/d(Omega_j, delta_j)", "n_atoms": n,
           "steps": steps, "precision": "complex128", "forward_s": round(t_fwd, 4),
           "gradient_s": round(t_grad, 4), "ratio": round(t_grad / t_fwd, 2),
           "value": c, "grad_omega_norm": float(np.linalg.norm(go)),
           "grad_delta_norm": float(np.linalg.norm(gd)), "krylov_iters": int(st.krylov_iters)}
    log(f"gradient N={n}: {steps} steps forward {t_fwd:.3f} s, gradient {t_grad:.3f} s")
    return out


def capacity_leg(rsv, wl, ctx, steps):
    """The 5x6 triangular quench at 30 atoms in complex64 (FP64 Lanczos scalars and host
    tridiagonal exponential, kmax 20, dt = 5 ns) from |0...0>: step 0 acquires the 192 GiB
    workspace (timed apart), steps 1..steps are timed."""
    import torch
    w = wl.triangular30()
    ws = rsv.rsv_workspace_bytes(w.n_atoms, w.kmax, "c64")
    reg = rsv.rsv_register_create(ctx, w.xyz, w.c6, "c64")
    psi = torch.zeros(1 << w.n_atoms, dtype=torch.complex64, device="cuda:0")
    psi[0] = 1
    pulses = rsv.PulseArrays(w.omega, w.delta)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rsv.rsv_evolve_device(reg, pulses, rsv.evolve_opts(w.dt_ns, w.tol, w.kmax, 12, 0, 1), psi)
    torch.cuda.synchronize()
    first = time.perf_counter() - t0
    t0 = time.perf_counter()
    st = rsv.rsv_evolve_device(reg, pulses, rsv.evolve_opts(w.dt_ns, w.tol, w.kmax, 12, 1, steps), psi)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    occ = rsv.rsv_occupations_device(ctx, w.n_atoms, psi, "c64")
    out = {"workload": "triangular30-quench", "n_atoms": w.n_atoms, "precision": "complex64",
           "steps": steps, "timed_steps": f"1..{steps}", "ms_per_step": round(wall / steps * 1e3, 2),
           "first_step_with_workspace_s": round(first, 3),
           "sim_us_per_s": round(steps * w.dt_ns * 1e-3 / wall, 5),
           "krylov_iters_per_step": round(st.krylov_iters / steps, 2),
           "krylov_max": int(st.krylov_max), "norm_final": st.norm_final,
           "workspace_bytes": int(ws), "workspace_gib": round(ws / 2**30, 2),
           "device_bytes_in_use": int(rsv.rsv_ctx_bytes_in_use(ctx)),
           "occupations_sum": round(float(occ.sum()), 6)}
    log(f"N=30 c64: step 0 with the workspace {first:.2f} s; {steps} steps in {wall:.2f} s, "
        f"workspace {ws / 2**30:.1f} GiB")
    rsv.rsv_register_destroy(reg)
    del psi
    torch.cuda.empty_cache()
    return out


def observables_leg(rsv, ctx, w, reg, psi, first_step, steps=10, reps=5):
    """Observables of the 27-atom complex128 state: <n_i n_j> (one pass over the state, HIP
    events), <H_k> (one H|psi> and a dot), and the cost of recording <n_i> after every step
    inside the final combination (steps first_step.. on a copy of the state, with and without
    the recording)."""
    import torch
    n = w.n_atoms
    pulses = rsv.PulseArrays(w.omega, w.delta)
    s = torch.cuda.current_stream()

    def timed(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        for _ in range(reps):
            fn()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    corr_ms = timed(lambda: rsv.rsv_correlations_device(ctx, n, psi, "c128"))
    corr = rsv.rsv_correlations_device(ctx, n, psi, "c128")
    occ = rsv.rsv_occupations_device(ctx, n, psi, "c128")
    energy_ms = timed(lambda: rsv.rsv_energy_device(reg, pulses, first_step, w.dt_ns, psi))
    energy = rsv.rsv_energy_device(reg, pulses, first_step, w.dt_ns, psi)
    log(f"observables: <n_i n_j> {corr_ms:.3f} ms, <H> {energy_ms:.3f} ms")
    copy = psi.clone()
    opts = rsv.evolve_opts(w.dt_ns, w.tol, w.kmax, 12, first_step, steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_plain = rsv.rsv_evolve_device(reg, pulses, opts, copy)
    torch.cuda.synchronize()
    plain = time.perf_counter() - t0
    copy.copy_(psi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_obs, rec = rsv.rsv_evolve_device_observed(reg, pulses, opts, copy, 1)
    torch.cuda.synchronize()
    observed = time.perf_counter() - t0
    log(f"observables: {steps} steps {plain:.3f} s plain, {observed:.3f} s recording <n_i> every step")
    del copy
    return {"workload": f"random27-sweep state after step {first_step - 1}, complex128",
            "correlations_ms": round(corr_ms, 4),
            "correlations_gbps": round(16.0 * (1 << n) / (corr_ms * 1e-3) / 1e9, 1),
            "correlations_diag_vs_occupations": float(np.abs(np.diag(corr) - occ).max()),
            "energy_ms": round(energy_ms, 4), "energy": energy,
            "observed_steps": steps, "plain_ms_per_step": round(plain / steps * 1e3, 3),
            "observed_ms_per_step": round(observed / steps * 1e3, 3),
            "krylov_iters": [int(st_plain.krylov_iters), int(st_obs.krylov_iters)],
            "recorded_occupations_last_sum": round(float(rec[-1].sum()), 6)}


def cpu_baseline(wl, gpu_iters_per_step):
    """The CPU oracle as it stands, on the host: one complete time step of its Krylov
    propagator (diagonal tensor, Lanczos with full re-orthogonalisation, tol 1e-13,
    combination) on the random-register sweep recipe at 20 atoms (plateau step 300, from a
    random normalised state), timed on one BLAS thread and on every core; the all-core time
    is scaled to 27 atoms by 2^7 x 27/20 (its per-iteration work is O(N 2^N) for H psi and
    O(m 2^N) for the re-orthogonalisation) and reported as simulated us per second.  The
    complete 10-atom chain run (dense eigendecomposition, 100 steps) is timed as well."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import evolve
    n = 20
    w = wl.random27(n_atoms=n)
    psi0 = wl.random_state(n, np.random.default_rng(42))
    cores = len(os.sched_getaffinity(0))
    blas = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
    times = {}
    for label, limit in (("all_cores", None), ("one_thread", 1)):
        with threadpool_limits(limits=limit):
            t0 = time.perf_counter()
            _, st = evolve.evolve_workload(w, psi0=psi0, steps=1, first_step=300, tol=1e-13,
                                           return_stats=True)
            times[label] = time.perf_counter() - t0
        log(f"cpu baseline: oracle step at N={n} ({label}) {times[label]:.1f} s, "
            f"{st['iters']} Krylov iterations")
    c1 = wl.chain10()
    t0 = time.perf_counter()
    evolve.evolve_workload(c1, method="dense")
    t_chain = time.perf_counter() - t0
    scale = 2.0 ** (27 - n) * 27.0 / n
    step27 = times["all_cores"] * scale
    return {
        "value": w.dt_ns * 1e-3 / step27, "unit": "sim-us/s", "cores": cores, "kind": "oracle",
        "sample": (f"one oracle time step (Krylov propagator with full re-orthogonalisation, "
                   f"tol 1e-13; {st['iters']} iterations) of the random-register sweep at "
                   f"N={n}, plateau step 300, random state: {times['all_cores']:.2f} s on "
                   f"{cores} cores (BLAS {blas} threads), {times['one_thread']:.2f} s on one "
                   f"thread; scaled to N=27 by 2^7 x 27/20 = {scale:.0f}"),
        "oracle_step_s_n20_all_cores": round(times["all_cores"], 3),
        "oracle_step_s_n20_one_thread": round(times["one_thread"], 3),
        "oracle_iters_n20": int(st["iters"]), "gpu_iters_per_step_n27": gpu_iters_per_step,
        "blas_threads": blas, "host_cpus": cores,
        "chain10_full_run_s": round(t_chain, 3),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-c64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=100,
                    help="jobs of the mixed-size serving stream (0: skip the serving leg)")
    ap.add_argument("--lanes", type=int, default=4)
    ap.add_argument("--n30-steps", type=int, default=3,
                    help="steps of the 30-atom complex64 leg (0: skip it)")
    ap.add_argument("--no-next", dest="next_rows", action="store_false",
                    help="skip the observables, Lindblad and gradient legs")
    ap.add_argument("--serve-full", type=int, default=0,
                    help="only serve this many jobs of the stream at --serve-rate and report")
    ap.add_argument("--serve-rate", type=float, default=2.4)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the state vector of one job lives on one MI355X; "
              "see the design notes for how the path would shard across GPUs", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2510_09813_amd import rsv
    from paper_2510_09813_amd import workloads as wl
    torch.cuda.set_device(0)
    if args.serve_full > 0:
        ctx = rsv.rsv_ctx_create(0)
        out = serving_full(rsv, wl, ctx, args.serve_full, args.serve_rate, args.lanes)
        rsv.rsv_ctx_destroy(ctx)
        print(json.dumps(out), flush=True)
        return
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
    iters_per_step = st128['krylov_iters'] / K

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
        "krylov_max": int(st128['krylov_max']),
        "hpsi_ms": round(ms128, 4), "hpsi_gbps": round(gbs128, 1),
        "roofline": {"bound": "hbm", "achieved": round(gbs128, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(gbs128 / PEAK_HBM_GBS, 4),
                     "kernel": "H|psi> at N=27 complex128 (high passes + low pass)",
                     "bytes_per_amplitude": 40,
                     # the state in and out only: E_b is formed on chip from small tables
                     "compulsory_bytes_per_amplitude": 32,
                     "achieved_compulsory": round(gbs128 * 32 / 40, 1),
                     "frac_compulsory": round(gbs128 * 32 / 40 / PEAK_HBM_GBS, 4),
                     # two passes move >= 80 B/amplitude: frac <= 0.5 at peak, 0.39 at the
                     # best measured copy (6.2 TB/s); the 0.70 target needs one pass
                     "frac_target": 0.70, "frac_ceiling_two_pass": 0.5,
                     "traffic": pmc_traffic("c128")},
        "register_build_ms": round(evolve_timed.register_ms, 3),
        "occupations_sum": round(float(occ.sum()), 6), "n_shots": len(shots),
        "device_copy_gbps": round(cp_gbs, 1),
    }

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
            "krylov_iters_per_step": round(st64['krylov_iters'] / K, 3),
            "traffic": pmc_traffic("c64"),
        }
        rsv.rsv_register_destroy(reg64)
        del psi64
    if args.next_rows:
        out["observables"] = observables_leg(rsv, ctx, w, reg128, psi128, min(W + K, w.n_steps - 10))
    rsv.rsv_register_destroy(reg128)
    del psi128
    torch.cuda.empty_cache()
    if args.n30_steps > 0:
        out["n30_c64"] = capacity_leg(rsv, wl, ctx, args.n30_steps)
    if args.next_rows:
        out["lindblad"] = lindblad_leg(rsv, wl, ctx, 12, 3)
        out["gradient"] = gradient_leg(rsv, wl, ctx, 20, 10)
    if args.serve_jobs > 0:
        out["serving"] = serving_leg(rsv, wl, ctx, args.serve_jobs, args.lanes)
        out["serving"]["small_jobs"] = small_job_leg(rsv, wl, ctx, 160, args.lanes)
        out["serving"]["noise_ensemble"] = ensemble_leg(rsv, wl, ctx, 512, args.lanes)
    rsv.rsv_ctx_destroy(ctx)

    if not args.no_cpu:
        log("cpu baseline: one oracle step at N=20 ...")
        out["cpu_baseline"] = cpu_baseline(wl, round(iters_per_step, 2))
    log(f"total {time.perf_counter() - t0:.1f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
