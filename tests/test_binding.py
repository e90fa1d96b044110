"""The Python binding checks every buffer before librsv sees it (CPU only): a tensor of the
wrong dtype, length, layout or device, a host state of the wrong length and per-site pulses
with the wrong number of rows raise ValueError without calling the library, which would
otherwise read or write past the end of the buffer."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2510_09813_amd import rsv

N = 5


def fake(prec):
    # a handle that is never dereferenced: every call below fails its checks first
    return rsv.Register(C.c_void_p(None), N, rsv.PRECISIONS[prec])


def pulses(rows=None):
    shape = (11,) if rows is None else (rows, 11)
    return rsv.PulseArrays(np.ones(shape), np.zeros(shape))


BAD_STATES = [
    ("dtype", lambda p: torch.zeros(1 << N, dtype=torch.complex64 if p == "c128" else torch.complex128)),
    ("elements", lambda p: torch.zeros((1 << N) - 1, dtype=getattr(torch, rsv.DTYPES[p]))),
    ("elements", lambda p: torch.zeros(1 << (N + 1), dtype=getattr(torch, rsv.DTYPES[p]))),
    ("contiguous", lambda p: torch.zeros(2 << N, dtype=getattr(torch, rsv.DTYPES[p]))[::2]),
    ("GPU", lambda p: torch.zeros(1 << N, dtype=getattr(torch, rsv.DTYPES[p]))),  # host tensor
    ("torch tensor", lambda p: 12345),  # a raw address is not accepted
]


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("why,make", BAD_STATES)
def test_state_buffers_are_checked(prec, why, make):
    reg = fake(prec)
    bad = make(prec)
    with pytest.raises(ValueError, match=why):
        rsv.rsv_apply_hamiltonian(reg, pulses(), 0, 10, bad, bad)
    with pytest.raises(ValueError, match=why):
        rsv.rsv_evolve_device(reg, pulses(), rsv.evolve_opts(10), bad)
    with pytest.raises(ValueError, match=why):
        rsv.rsv_occupations_device(None, N, bad, prec)
    with pytest.raises(ValueError, match=why):
        rsv.rsv_sample_device(None, N, bad, 0, 10, prec)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_diagonal_buffer_is_checked(prec):
    reg = fake(prec)
    wrong = torch.float32 if prec == "c128" else torch.float64
    with pytest.raises(ValueError, match="dtype"):
        rsv.rsv_register_diagonal(reg, torch.zeros(1 << N, dtype=wrong))
    right = torch.float64 if prec == "c128" else torch.float32
    with pytest.raises(ValueError, match="elements"):
        rsv.rsv_register_diagonal(reg, torch.zeros(1 << (N - 1), dtype=right))


def test_host_inputs_are_checked():
    reg = fake("c128")
    with pytest.raises(ValueError, match="amplitudes"):
        rsv.rsv_evolve(reg, pulses(), rsv.evolve_opts(10), psi0=np.zeros(1 << (N - 1)))
    with pytest.raises(ValueError, match="rows"):
        rsv.rsv_evolve(reg, pulses(rows=N + 1), rsv.evolve_opts(10))
    with pytest.raises(ValueError, match="rows"):
        rsv.rsv_apply_hamiltonian(reg, pulses(rows=N - 1), 0, 10, None, None)
    with pytest.raises(ValueError, match="amplitudes"):
        rsv.rsv_server_submit(None, np.zeros((N, 3)), 1.0, pulses(), rsv.evolve_opts(10),
                              psi0=np.zeros(3))
    with pytest.raises(ValueError, match="rows"):
        rsv.rsv_server_submit(None, np.zeros((N, 3)), 1.0, pulses(rows=2), rsv.evolve_opts(10))
    with pytest.raises(ValueError):
        rsv.PulseArrays(np.ones((2, 3, 4)), np.ones((2, 3, 4)))
    with pytest.raises(ValueError):
        rsv.rsv_occupations_device(None, 31, torch.zeros(4), "c128")
    with pytest.raises(ValueError):
        rsv.rsv_sample_device(None, N, None, 0, -1, "c128")
    with pytest.raises(ValueError):
        rsv.rsv_register_create(None, np.zeros((2, 3)), 1.0, "c32")
