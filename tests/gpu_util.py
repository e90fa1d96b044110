"""Helpers shared by the GPU tests: device buffers and a session context."""
import numpy as np

from paper_2510_09813_amd import rsv

DTYPES = {"c128": "complex128", "c64": "complex64"}
REAL = {"c128": "float64", "c64": "float32"}


def to_dev(x, prec):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x).astype(DTYPES[prec])).to("cuda:0")


def empty_dev(n, prec):
    import torch
    return torch.empty(1 << n, dtype=getattr(torch, DTYPES[prec]), device="cuda:0")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def rel_err(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def assert_valid_samples(got, psi, seed, min_agree):
    """Shots drawn by the library from psi against the oracle's sampler (the definition of
    reading R16: shot s is the smallest b with CDF(b) > u_s CDF_total).  At least min_agree
    shots must be the oracle's index; every other shot must be a correct answer too: the
    oracle's index and the library's are neighbours among the indices with nonzero mass, and
    u_s CDF_total lies within FP64 rounding of the prefix sum that separates them (each side
    sums at most 2^N terms, so the two sums and the two targets differ by at most
    4 * 2^N * eps * total)."""
    from oracle import observables
    got = np.asarray(got, dtype=np.uint64)
    want = observables.sample(psi, seed, got.size)
    p = observables.probabilities(psi)
    cdf = np.cumsum(p)
    total = cdf[-1]
    u = observables.uniforms(seed, got.size)
    bound = 4.0 * p.size * np.finfo(np.float64).eps * total
    bad = np.flatnonzero(got != want)
    assert got.size - bad.size >= min_agree, (got.size - bad.size, min_agree)
    for s in bad:
        a, b = sorted((int(got[s]), int(want[s])))
        assert b < p.size and p[a] > 0 and p[b] > 0, (s, a, b)
        assert not np.any(p[a + 1:b] > 0), (s, a, b)  # adjacent among indices with mass
        assert abs(cdf[a] - u[s] * total) <= bound, (s, a, b, cdf[a] - u[s] * total, bound)
    return got.size - bad.size
