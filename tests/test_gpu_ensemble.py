"""Shot-to-shot noise ensembles through the server (Sec. III.A): every member against the
oracle evolved with the oracle's own draws of the member's parameters, alone == in the
ensemble bit for bit, and zero noise == the noiseless job bit for bit."""
import numpy as np
import pytest

from oracle import evolve, noise, observables
from paper_2510_09813_amd import rsv
from paper_2510_09813_amd import workloads as wl
from tests.gpu_util import assert_valid_samples

pytestmark = pytest.mark.gpu
INFID = {"c128": 1e-10, "c64": 1e-6}
NOISE = (0.05, 2 * np.pi * 0.25, 0.15)  # 5 % amplitude, 0.25 MHz detuning, 150 nm


@pytest.fixture(scope="module")
def ctx():
    import torch
    torch.cuda.set_device(0)
    c = rsv.rsv_ctx_create(0)
    yield c
    rsv.rsv_ctx_destroy(c)


def job(n, prec, t_ns, seed):
    w = wl.serving_job(np.random.default_rng(seed), n_min=n, n_max=n, precision=prec)
    w.t_ns, w.omega, w.delta = t_ns, w.omega[:t_ns + 1], w.delta[:t_ns + 1]
    return w


def run(ctx, submit, n_expected, pack):
    srv = rsv.rsv_server_create(ctx, n_lanes=2, arena_bytes=1 << 30, pack_max_atoms=pack)
    try:
        submit(srv)
        done = []
        while len(done) < n_expected:
            done += rsv.rsv_server_poll(srv, 64, 1000)
    finally:
        rsv.rsv_server_destroy(srv)
    assert all(c["status"] == rsv.RSV_OK for c in done), [c["error"] for c in done]
    return {c["tag"]: c for c in done}


def submit_ensemble(w, prec, members, nz=NOISE, noise_seed=9):
    def f(srv):
        ids = rsv.rsv_server_submit_ensemble(
            srv, w.xyz, w.c6, rsv.PulseArrays(w.omega, w.delta), rsv.evolve_opts(w.dt_ns, w.tol, w.kmax, 12),
            nz, noise_seed, members, prec, n_shots=300, seed=5, return_state=True, tag=100)
        assert len(ids) == members and len(set(ids)) == members
    return f


@pytest.mark.parametrize("prec,n,members,pack", [("c64", 8, 12, 13), ("c128", 11, 4, 0),
                                                 ("c128", 6, 6, 12)])
def test_members_match_oracle(ctx, prec, n, members, pack):
    w = job(n, prec, 300, seed=n)
    got = run(ctx, submit_ensemble(w, prec, members), members, pack)
    for s in range(members):
        c = got[100 + s]
        f, off, pos = noise.member(9, s, n, *NOISE, w.xyz)
        om, de = noise.member_pulses(w.omega, w.delta, f, off)
        method = "dense" if n <= 10 else "lanczos"
        ref = evolve.evolve(pos, w.c6, om, de, None, w.t_ns, w.dt_ns, method=method)
        loss = observables.fidelity_loss(ref, c["state"])
        assert loss <= INFID[prec], (s, loss)
        np.testing.assert_allclose(c["occupations"], observables.occupations(ref),
                                   atol=1e-8 if prec == "c128" else 1e-5)
        assert_valid_samples(c["samples"], c["state"], 5 + s, 298)
    # the members differ from each other (the noise acts)
    assert observables.fidelity_loss(got[100]["state"], got[101]["state"]) > 1e-8


def test_per_site_members_with_phase(ctx):
    """A job with per-site pulses and a phase: members keep their per-site rows, scaled and
    offset atom by atom, against the oracle with the same draws."""
    n, members = 7, 5
    rng = np.random.default_rng(77)
    w = job(n, "c128", 200, seed=7)
    om = np.outer(rng.uniform(0.5, 1.5, n), w.omega)
    de = np.outer(rng.uniform(0.5, 1.5, n), w.delta)
    ph = np.outer(rng.uniform(-1, 1, n), np.linspace(0, 1, w.t_ns + 1))

    def f(srv):
        rsv.rsv_server_submit_ensemble(srv, w.xyz, w.c6, rsv.PulseArrays(om, de, ph),
                                       rsv.evolve_opts(w.dt_ns, w.tol, w.kmax, 12), NOISE, 3,
                                       members, "c128", return_state=True, tag=100)
    got = run(ctx, f, members, 12)
    for s in range(members):
        fac, off, pos = noise.member(3, s, n, *NOISE, w.xyz)
        mom, mde = noise.member_pulses(om, de, fac, off)
        ref = evolve.evolve(pos, w.c6, mom, mde, ph, w.t_ns, w.dt_ns, method="dense")
        assert observables.fidelity_loss(ref, got[100 + s]["state"]) <= INFID["c128"], s


@pytest.mark.parametrize("prec,pack", [("c64", 13), ("c128", 0)])
def test_member_alone_equals_in_ensemble(ctx, prec, pack):
    n, members, s = 9, 8, 5
    w = job(n, prec, 200, seed=3)
    ens = run(ctx, submit_ensemble(w, prec, members), members, pack)
    f, off, pos = rsv.rsv_noise_member(NOISE, 9, w.xyz, s)
    om = f * np.broadcast_to(w.omega, (n, w.omega.size))
    de = np.broadcast_to(w.delta, (n, w.delta.size)) + off[:, None]

    def one(srv):
        rsv.rsv_server_submit(srv, pos, w.c6, rsv.PulseArrays(om, de),
                              rsv.evolve_opts(w.dt_ns, w.tol, w.kmax, 12), prec, n_shots=300,
                              seed=5 + s, return_state=True, tag=100 + s)
    alone = run(ctx, one, 1, pack)[100 + s]
    c = ens[100 + s]
    assert np.array_equal(alone["state"], c["state"])
    assert np.array_equal(alone["occupations"], c["occupations"])
    assert np.array_equal(alone["samples"], c["samples"])


def test_zero_noise_equals_noiseless_job(ctx):
    n, members = 10, 5
    w = job(n, "c64", 200, seed=4)
    ens = run(ctx, submit_ensemble(w, "c64", members, nz=(0.0, 0.0, 0.0)), members, 13)

    def one(srv):
        rsv.rsv_server_submit(srv, w.xyz, w.c6, rsv.PulseArrays(w.omega, w.delta),
                              rsv.evolve_opts(w.dt_ns, w.tol, w.kmax, 12), "c64", n_shots=300,
                              seed=5, return_state=True, tag=100)
    base = run(ctx, one, 1, 13)[100]
    for s in range(members):
        assert np.array_equal(ens[100 + s]["state"], base["state"])


def test_ensemble_rejections(ctx):
    w = job(6, "c64", 100, seed=1)
    srv = rsv.rsv_server_create(ctx, n_lanes=1, arena_bytes=1 << 28, max_queue=3)
    try:
        with pytest.raises(rsv.RsvError) as e:  # all or none: 4 members do not fit a queue of 3
            submit_ensemble(w, "c64", 4)(srv)
        assert e.value.code in (rsv.RSV_EBUSY,)
        with pytest.raises(rsv.RsvError):
            submit_ensemble(w, "c64", 0)(srv)
        with pytest.raises(rsv.RsvError):
            submit_ensemble(w, "c64", 2, nz=(0.1, -1.0, 0.0))(srv)
    finally:
        rsv.rsv_server_destroy(srv)
