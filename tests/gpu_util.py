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
