"""Host logic of the H|psi> tile plans (CPU only): for every register size and both
precisions, the low pass (with its extension of the top bits) and the high passes flip
every bit exactly once, each tile stays inside the index with its contiguous run below its
high bits, every pass's tiles cover the index space exactly once (checked element by element
up to 20 atoms), and the plan has the fewest passes that 12-bit high tiles with runs of at
least 2^3 amplitudes and an extension of at most 7 bits allow."""
import ctypes as C

import pytest

from paper_2510_09813_amd import rsv

N_MAX = 30


class TilePlan(C.Structure):
    _fields_ = [("n", C.c_int), ("lo_bits", C.c_int), ("hi_bits", C.c_int),
                ("n_hi_passes", C.c_int), ("flip_lo", C.c_int * N_MAX),
                ("flip_hi", C.c_int * N_MAX), ("tile_a", C.c_int * N_MAX),
                ("run_bits", C.c_int * N_MAX), ("lo_ext", C.c_int),
                ("lo_ext_bit", C.c_int)]


def plan(prec, n):
    """rsv::make_tile_plan(prec, n) through its C++ symbol."""
    f = rsv.lib()._ZN3rsv14make_tile_planEii  # rsv::make_tile_plan(int, int), host code
    f.restype = TilePlan
    f.argtypes = [C.c_int, C.c_int]
    return f(prec, n)


@pytest.mark.parametrize("prec", [0, 1])
def test_plans_partition_the_bits_and_the_index(prec):
    for n in range(1, N_MAX + 1):
        p = plan(prec, n)
        assert p.n == n and 1 <= p.lo_bits <= n
        # complex64 takes 12-bit low tiles where the extension leaves one high pass
        assert p.lo_bits == min(n, 12 if prec == 0 or 22 <= n <= 28 else 13)
        covered = []
        for i in range(p.n_hi_passes):
            r, a, f0, f1 = p.run_bits[i], p.tile_a[i], p.flip_lo[i], p.flip_hi[i]
            g = p.hi_bits - r
            assert 3 <= r <= 6 and r <= a and a + g <= n and a <= f0 < f1 <= a + g
            covered += list(range(f0, f1))
            if n <= 20:
                gap, seen = a - r, set()
                for blk in range(1 << (n - p.hi_bits)):
                    obase = ((blk & ((1 << gap) - 1)) << r) | ((blk >> gap) << (a + g))
                    for e in range(1 << p.hi_bits):
                        seen.add(obase | (e & ((1 << r) - 1)) | ((e >> r) << a))
                assert seen == set(range(1 << n))
        assert 0 <= p.lo_ext <= 7 and p.lo_bits + p.lo_ext <= n
        # the high passes flip the bits between the low tile and the extension (the top bits)
        assert covered == list(range(p.lo_bits, n - p.lo_ext))
        if p.lo_ext:
            assert p.lo_ext_bit == n - p.lo_ext
        # the passes are as few as the shortest run and the extension allow; the extension
        # only where it saves a high pass, and then never below one high pass
        rest = n - p.lo_bits
        per = p.hi_bits - 3
        plain = -(-rest // per) if rest > 0 else 0
        fewest = -(-max(rest - 7, 0) // per)
        if plain >= 2 and fewest < plain:
            assert p.lo_ext > 0 and p.n_hi_passes == fewest >= 1
        else:
            assert p.lo_ext == 0 and p.n_hi_passes == plain
