"""Shot-to-shot parameter noise (Sec. III.A), host side, CPU only: the oracle's generator
against SplitMix64's published outputs and the normal distribution, the member
perturbation's structure, and the library's rsv_noise_member against the oracle's draws."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import noise, observables
from paper_2510_09813_amd import rsv
from paper_2510_09813_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "splitmix64.txt")


def test_counter_form_matches_published_outputs():
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        seed, k, out = (int(v) for v in line.split())
        assert noise.splitmix64_at(seed, k) == out
    # and the sequential generator of the sampler
    assert [noise.splitmix64_at(99, k) for k in range(5)] == observables.splitmix64(99, 5)


def test_gaussians_are_standard_normal():
    g = np.array([noise.gaussian(7, c) for c in range(20000)])
    assert abs(g.mean()) < 4 / np.sqrt(g.size)
    assert abs(g.var() - 1) < 4 * np.sqrt(2 / g.size)
    assert stats.kstest(g, "norm").pvalue > 1e-3
    # independent streams for different seeds, no correlation between neighbours
    h = np.array([noise.gaussian(8, c) for c in range(20000)])
    assert abs(np.corrcoef(g, h)[0, 1]) < 4 / np.sqrt(g.size)
    assert abs(np.corrcoef(g[:-1], g[1:])[0, 1]) < 4 / np.sqrt(g.size)


def test_member_structure():
    xyz = wl.chain(5, 6.0)
    f, off, pos = noise.member(3, 2, 5, 0.0, 0.0, 0.0, xyz)
    assert f == 1.0 and np.all(off == 0) and np.array_equal(pos, xyz)
    f1, off1, pos1 = noise.member(3, 2, 5, 0.1, 2.0, 0.05, xyz)
    f2, off2, pos2 = noise.member(3, 2, 5, 0.2, 4.0, 0.10, xyz)
    # the same variates scaled: doubling every sigma doubles every perturbation
    assert np.isclose(f2 - 1, 2 * (f1 - 1)) and np.allclose(off2, 2 * off1)
    assert np.allclose(pos2 - xyz, 2 * (pos1 - xyz))
    # member s uses variates s (4N + 1) .. s (4N + 1) + 4N
    per = 4 * 5 + 1
    assert np.isclose(f1, 1 + 0.1 * noise.gaussian(3, 2 * per))
    assert np.isclose(off1[4], 2.0 * noise.gaussian(3, 2 * per + 5))
    assert np.isclose(pos1[1, 2] - xyz[1, 2], 0.05 * noise.gaussian(3, 2 * per + 1 + 5 + 3 + 2))
    om, de = noise.member_pulses(np.ones(4), np.zeros(4), f1, off1)
    assert om.shape == de.shape == (5, 4) and np.allclose(de[:, 2], off1)


@pytest.mark.parametrize("member", [0, 1, 17, 123456])
def test_library_draws_match_oracle(member):
    rng = np.random.default_rng(member)
    xyz = wl.random_register(9, 30.0, 5.0, rng)
    nz = (0.05, 2 * np.pi * 0.3, 0.1)
    f, off, pos = rsv.rsv_noise_member(nz, 42, xyz, member)
    fo, offo, poso = noise.member(42, member, 9, *nz, xyz)
    assert abs(f - fo) <= 1e-15 * abs(fo)
    np.testing.assert_allclose(off, offo, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(pos, poso, rtol=1e-15, atol=1e-15)


def test_library_rejects_bad_noise():
    with pytest.raises(rsv.RsvError):
        rsv.rsv_noise_member((-0.1, 0.0, 0.0), 1, wl.chain(3, 5.0), 0)
    with pytest.raises(rsv.RsvError):
        rsv.rsv_noise_member((0.1, float("nan"), 0.0), 1, wl.chain(3, 5.0), 0)
    with pytest.raises(rsv.RsvError):
        rsv.rsv_noise_member((0.1, 0.0, 0.0), 1, wl.chain(3, 5.0), -1)
