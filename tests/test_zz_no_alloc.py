"""The allocation-free sampler (rsv_sample_device_static) against rsv_sample_device.

Both run the same kernels; the static form keeps its block sums, scan and indices in a
device array inside the library instead of context memory.  Indices are integers: bit-exact
agreement is required, on two calls in a row (the second on a smaller state with fewer
shots, so stale contents of the shared array would show), in both precisions.
"""
import numpy as np
import pytest

from paper_2510_09813_amd import rsv
from paper_2510_09813_amd import workloads as wl
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    torch.cuda.set_device(0)
    c = rsv.rsv_ctx_create(0)
    yield c
    rsv.rsv_ctx_destroy(c)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_static_sampler_matches_allocating_one(ctx, prec):
    rng = np.random.default_rng(5)
    # large then small: 2^21 amplitudes (512 blocks), then 2^13 (2 blocks) with fewer shots
    for n, shots, seed in ((21, 5000, 11), (13, 700, 12), (7, 3, 13)):
        psi = wl.random_state(n, rng)
        psi[: 1 << (n - 2)] = 0  # a zero-mass quarter: the search must skip whole blocks
        d = to_dev(psi, prec)
        want = rsv.rsv_sample_device(ctx, n, d, seed, shots, prec)
        got = rsv.rsv_sample_device_static(ctx, n, d, seed, shots, prec)
        np.testing.assert_array_equal(got, want)
        assert np.all(got >= (1 << (n - 2))) and np.all(got < (1 << n))


def test_static_sampler_limits(ctx):
    d = to_dev(wl.random_state(10, np.random.default_rng(0)), "c128")
    assert rsv.rsv_sample_device_static(ctx, 10, d, 0, 0, "c128").size == 0
    with pytest.raises(rsv.RsvError):
        rsv.rsv_sample_device_static(ctx, 10, d, 0, 65537, "c128")
    got = rsv.rsv_sample_device_static(ctx, 10, d, 3, 65536, "c128")
    np.testing.assert_array_equal(got, rsv.rsv_sample_device(ctx, 10, d, 3, 65536, "c128"))
