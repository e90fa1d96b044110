"""Host-side checks of the C ABI (no GPU): every declared symbol is exported, the host FP64
tridiagonal exponential matches an independent exponential, input validation that needs no
device, and the workspace formula."""
import os
import re

import numpy as np
import pytest
import scipy.linalg

from paper_2510_09813_amd import rsv

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "rsv.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsv_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = rsv.lib()
    decl = declared_functions()
    assert decl, "no declarations parsed"
    assert sorted(rsv.EXPORTED) == decl
    for name in decl:
        assert hasattr(lib, name), name
    assert "gfx950" in rsv.rsv_version()


@pytest.mark.parametrize("m", [1, 2, 3, 7, 16, 30, 64])
def test_tridiag_expm_matches_expm(m):
    rng = np.random.default_rng(m)
    a = rng.normal(size=m) * 50
    b = np.abs(rng.normal(size=m - 1)) * 8
    t = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    for tau in (0.0, 0.01, 0.2):
        e1 = np.zeros(m)
        e1[0] = 1
        ref = scipy.linalg.expm(-1j * tau * t) @ e1
        got = rsv.rsv_tridiag_expm(a, b, tau)
        assert np.abs(got - ref).max() < 1e-12


def test_tridiag_expm_degenerate_and_decoupled():
    # zero off-diagonal: T is diagonal, y = e^{-i tau a_0} e_1
    a = np.array([3.0, -1.0, 2.0, 2.0])
    got = rsv.rsv_tridiag_expm(a, np.zeros(3), 0.7)
    assert abs(got[0] - np.exp(-0.7j * 3.0)) < 1e-15 and np.abs(got[1:]).max() < 1e-15
    # repeated eigenvalues
    a = np.full(6, 2.5)
    b = np.ones(5)
    t = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    ref = scipy.linalg.expm(-1j * 1.3 * t)[:, 0]
    assert np.abs(rsv.rsv_tridiag_expm(a, b, 1.3) - ref).max() < 1e-13


def test_tridiag_expm_rejects_bad_input():
    with pytest.raises(rsv.RsvError) as e:
        rsv.rsv_tridiag_expm(np.zeros(65), np.zeros(64), 0.1)
    assert e.value.code == rsv.RSV_EINVAL
    with pytest.raises(rsv.RsvError):
        rsv.rsv_tridiag_expm(np.array([1.0, np.nan]), np.array([1.0]), 0.1)


def test_workspace_formula():
    # (kmax + 3) vectors + diagonal + state: grows by 2^N amplitudes per Krylov vector
    a = rsv.rsv_workspace_bytes(27, 30, "c128")
    b = rsv.rsv_workspace_bytes(27, 31, "c128")
    assert b - a == 16 << 27
    c = rsv.rsv_workspace_bytes(30, 20, "c64")
    assert 180 * 2 ** 30 < c < 200 * 2 ** 30  # N = 30 in complex64 fits 288 GB
    assert rsv.rsv_workspace_bytes(31, 20, "c64") == 0
    assert rsv.rsv_workspace_bytes(10, 1, "c64") == 0
