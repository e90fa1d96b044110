"""ctypes binding of librsv (include/rsv.h): argument marshalling only.

Every function has the name of the C call it wraps; status codes other than RSV_OK raise
``RsvError`` with the library's message.  Device buffers are torch tensors (complex128 for
RSV_C128, complex64 for RSV_C64) or raw device addresses; torch only provides memory and
streams, all arithmetic runs in librsv's HIP kernels.  There is no fallback: if librsv.so is
missing or cannot be loaded, ``lib()`` raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librsv.so")

RSV_OK, RSV_EINVAL, RSV_ENOMEM, RSV_EDEVICE, RSV_ENOTCONV, RSV_ENUMERIC, RSV_EBUSY, \
    RSV_ECANCELLED = range(8)
RSV_C128, RSV_C64 = 0, 1
PRECISIONS = {"c128": RSV_C128, "c64": RSV_C64}

# Every symbol include/rsv.h declares; the CPU test suite checks that the library exports them.
EXPORTED = [
    "rsv_version", "rsv_last_error", "rsv_ctx_create", "rsv_ctx_destroy", "rsv_ctx_bytes_in_use",
    "rsv_register_create", "rsv_register_destroy", "rsv_register_diagonal", "rsv_workspace_bytes",
    "rsv_apply_hamiltonian", "rsv_evolve_device", "rsv_evolve", "rsv_result_state",
    "rsv_result_occupations", "rsv_result_sample", "rsv_result_stats", "rsv_result_destroy",
    "rsv_occupations_device", "rsv_sample_device", "rsv_sample_device_static",
    "rsv_tridiag_expm", "rsv_evolve_device_observed", "rsv_energy_device",
    "rsv_correlations_device", "rsv_lindblad_apply", "rsv_lindblad_evolve_device",
    "rsv_lindblad_occupations", "rsv_gradient_occupations",
]


class Lindblad(C.Structure):
    _fields_ = [("relax_rate", C.c_double), ("dephasing_rate", C.c_double)]


class RsvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"librsv error {code}: {msg}")
        self.code = code


class Pulses(C.Structure):
    _fields_ = [("n_samples", C.c_int64), ("per_site", C.c_int),
                ("omega", C.POINTER(C.c_double)), ("delta", C.POINTER(C.c_double)),
                ("phi", C.POINTER(C.c_double))]


class EvolveOpts(C.Structure):
    _fields_ = [("dt_ns", C.c_int), ("tol", C.c_double), ("kmax", C.c_int),
                ("max_substep_depth", C.c_int), ("first_step", C.c_int64),
                ("n_steps", C.c_int64), ("reorth", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("krylov_iters", C.c_int64), ("krylov_max", C.c_int64),
                ("substeps", C.c_int64), ("norm_final", C.c_double), ("seconds", C.c_double),
                ("bytes_hpsi", C.c_double), ("ortho_loss", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Loads librsv.so (torch first, so that one HIP runtime serves both)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    try:
        import torch  # noqa: F401
    except Exception:  # pragma: no cover - torch is optional for host-only calls
        pass
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u64, dbl, sz = C.c_void_p, C.c_int, C.c_int64, C.c_uint64, C.c_double, C.c_size_t
    pd = C.POINTER(C.c_double)
    sig = {
        "rsv_version": (C.c_char_p, []),
        "rsv_last_error": (C.c_char_p, []),
        "rsv_ctx_create": (i32, [i32, sz, C.POINTER(vp)]),
        "rsv_ctx_destroy": (None, [vp]),
        "rsv_ctx_bytes_in_use": (sz, [vp]),
        "rsv_register_create": (i32, [vp, i32, pd, dbl, i32, C.POINTER(vp)]),
        "rsv_register_destroy": (None, [vp]),
        "rsv_register_diagonal": (i32, [vp, vp, vp]),
        "rsv_workspace_bytes": (sz, [i32, i32, i32]),
        "rsv_apply_hamiltonian": (i32, [vp, C.POINTER(Pulses), i64, i32, vp, vp, vp]),
        "rsv_evolve_device": (i32, [vp, C.POINTER(Pulses), C.POINTER(EvolveOpts), vp, vp,
                                    C.POINTER(Stats)]),
        "rsv_evolve": (i32, [vp, C.POINTER(Pulses), C.POINTER(EvolveOpts), vp, C.POINTER(vp)]),
        "rsv_result_state": (i32, [vp, vp]),
        "rsv_result_occupations": (i32, [vp, pd]),
        "rsv_result_sample": (i32, [vp, u64, i32, C.POINTER(C.c_uint64)]),
        "rsv_result_stats": (i32, [vp, C.POINTER(Stats)]),
        "rsv_result_destroy": (None, [vp]),
        "rsv_occupations_device": (i32, [vp, i32, i32, vp, pd, vp]),
        "rsv_sample_device": (i32, [vp, i32, i32, vp, u64, i32, C.POINTER(C.c_uint64), vp]),
        "rsv_sample_device_static": (i32, [vp, i32, i32, vp, u64, i32, C.POINTER(C.c_uint64),
                                           vp]),
        "rsv_tridiag_expm": (i32, [i32, pd, pd, dbl, pd, pd]),
        "rsv_evolve_device_observed": (i32, [vp, C.POINTER(Pulses), C.POINTER(EvolveOpts), vp,
                                             vp, i32, pd, C.POINTER(Stats)]),
        "rsv_energy_device": (i32, [vp, C.POINTER(Pulses), i64, i32, vp, pd, vp]),
        "rsv_correlations_device": (i32, [vp, i32, i32, vp, pd, vp]),
        "rsv_lindblad_apply": (i32, [vp, C.POINTER(Pulses), i64, i32, C.POINTER(Lindblad), vp,
                                     vp, vp]),
        "rsv_lindblad_evolve_device": (i32, [vp, C.POINTER(Pulses), C.POINTER(EvolveOpts),
                                             C.POINTER(Lindblad), vp, vp, C.POINTER(Stats)]),
        "rsv_lindblad_occupations": (i32, [vp, i32, i32, vp, pd, pd, vp]),
        "rsv_gradient_occupations": (i32, [vp, C.POINTER(Pulses), C.POINTER(EvolveOpts), pd, vp,
                                           pd, pd, pd, C.POINTER(Stats)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(rc: int):
    if rc != RSV_OK:
        raise RsvError(rc, lib().rsv_last_error().decode())


class Register:
    """Handle of an rsv_register together with its size and precision, so that buffers
    handed to the library can be checked before the call (ctypes passes _as_parameter_)."""

    def __init__(self, handle: C.c_void_p, n_atoms: int, precision: int):
        self._as_parameter_ = handle
        self.n_atoms = int(n_atoms)
        self.precision = int(precision)

    @property
    def value(self):
        return self._as_parameter_.value


COMPLEX_DTYPE = {RSV_C128: "complex128", RSV_C64: "complex64"}
DTYPES = {"c128": "complex128", "c64": "complex64"}
REAL_DTYPE = {RSV_C128: "float64", RSV_C64: "float32"}


def _prec(precision) -> int:
    p = PRECISIONS.get(precision, precision)
    if p not in (RSV_C128, RSV_C64):
        raise ValueError(f"unknown precision {precision!r}")
    return p


def _dptr(buf, numel: int, dtype: str, what: str) -> int:
    """Device address of a contiguous torch tensor on a GPU holding exactly ``numel``
    elements of ``dtype`` (the library reads and writes that many); anything else raises
    ValueError before the library is called."""
    import torch
    if not isinstance(buf, torch.Tensor):
        raise ValueError(f"{what}: expected a torch tensor, got {type(buf).__name__}")
    want = getattr(torch, dtype)
    if buf.dtype != want:
        raise ValueError(f"{what}: dtype {buf.dtype} does not match the register ({want})")
    if buf.numel() != numel:
        raise ValueError(f"{what}: {buf.numel()} elements, the register needs {numel}")
    if not buf.is_contiguous():
        raise ValueError(f"{what}: tensor must be contiguous")
    if not buf.is_cuda:
        raise ValueError(f"{what}: tensor must be on a GPU, not {buf.device}")
    return int(buf.data_ptr())


def _state_ptr(buf, n_atoms: int, precision: int, what: str) -> int:
    return _dptr(buf, 1 << n_atoms, COMPLEX_DTYPE[precision], what)


def _check_pulses(pulses: "PulseArrays", n_atoms: int):
    if pulses.omega.ndim == 2 and pulses.omega.shape[0] != n_atoms:
        raise ValueError(f"per-site pulses have {pulses.omega.shape[0]} rows, the register "
                         f"has {n_atoms} atoms")


def _host_state(psi0, n_atoms: int):
    buf = np.ascontiguousarray(np.asarray(psi0, dtype=np.complex128)).reshape(-1)
    if buf.size != 1 << n_atoms:
        raise ValueError(f"initial state has {buf.size} amplitudes, need 2^{n_atoms}")
    return buf


def _stream(stream) -> Optional[int]:
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return int(torch.cuda.current_stream().cuda_stream) or None
        except Exception:  # pragma: no cover
            pass
        return None
    return int(stream)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class PulseArrays:
    """Keeps the sample arrays alive while librsv reads them."""

    def __init__(self, omega, delta, phi=None):
        self.omega, self.delta = _f64(omega), _f64(delta)
        self.phi = None if phi is None else _f64(phi)
        if self.omega.shape != self.delta.shape or (self.phi is not None and self.phi.shape != self.omega.shape):
            raise ValueError("omega, delta and phi must have the same shape")
        if self.omega.ndim not in (1, 2) or self.omega.shape[-1] < 1:
            raise ValueError("pulse arrays are [n_samples] or [n_atoms][n_samples]")
        pd = C.POINTER(C.c_double)
        self.struct = Pulses(self.omega.shape[-1], 1 if self.omega.ndim == 2 else 0,
                             self.omega.ctypes.data_as(pd), self.delta.ctypes.data_as(pd),
                             self.phi.ctypes.data_as(pd) if self.phi is not None else None)


def evolve_opts(dt_ns: int, tol: float = 1e-10, kmax: int = 30, max_substep_depth: int = 12,
                first_step: int = 0, n_steps: int = -1, reorth: int = 0) -> EvolveOpts:
    return EvolveOpts(dt_ns, tol, kmax, max_substep_depth, first_step, n_steps, reorth)


# ------------------------------------------------------------------------- C calls
def rsv_version() -> str:
    return lib().rsv_version().decode()


def rsv_ctx_create(device: int = 0, budget: int = 0):
    h = C.c_void_p()
    _check(lib().rsv_ctx_create(device, budget, C.byref(h)))
    return h


def rsv_ctx_destroy(ctx):
    lib().rsv_ctx_destroy(ctx)


def rsv_ctx_bytes_in_use(ctx) -> int:
    return int(lib().rsv_ctx_bytes_in_use(ctx))


def rsv_register_create(ctx, xyz, c6: float, precision="c128") -> Register:
    xyz = _f64(xyz).reshape(-1, 3)
    h = C.c_void_p()
    prec = _prec(precision)
    _check(lib().rsv_register_create(ctx, xyz.shape[0], xyz.ctypes.data_as(C.POINTER(C.c_double)),
                                     float(c6), prec, C.byref(h)))
    return Register(h, xyz.shape[0], prec)


def rsv_register_destroy(reg):
    lib().rsv_register_destroy(reg)


def rsv_register_diagonal(reg: Register, d_out, stream=None):
    ptr = _dptr(d_out, 1 << reg.n_atoms, REAL_DTYPE[reg.precision], "diagonal")
    _check(lib().rsv_register_diagonal(reg, ptr, _stream(stream)))


def rsv_workspace_bytes(n_atoms: int, kmax: int, precision="c128") -> int:
    return int(lib().rsv_workspace_bytes(n_atoms, kmax, PRECISIONS.get(precision, precision)))


def rsv_apply_hamiltonian(reg: Register, pulses: PulseArrays, step: int, dt_ns: int, d_in, d_out,
                          stream=None):
    _check_pulses(pulses, reg.n_atoms)
    pin = _state_ptr(d_in, reg.n_atoms, reg.precision, "input state")
    pout = _state_ptr(d_out, reg.n_atoms, reg.precision, "output state")
    _check(lib().rsv_apply_hamiltonian(reg, C.byref(pulses.struct), step, dt_ns, pin, pout,
                                       _stream(stream)))


def rsv_evolve_device(reg: Register, pulses: PulseArrays, opts: EvolveOpts, d_psi,
                      stream=None) -> Stats:
    _check_pulses(pulses, reg.n_atoms)
    ptr = _state_ptr(d_psi, reg.n_atoms, reg.precision, "state")
    st = Stats()
    _check(lib().rsv_evolve_device(reg, C.byref(pulses.struct), C.byref(opts), ptr,
                                   _stream(stream), C.byref(st)))
    return st


def rsv_evolve_device_observed(reg: Register, pulses: PulseArrays, opts: EvolveOpts, d_psi,
                               every: int, stream=None):
    """Evolves d_psi in place; returns (stats, occupations [steps // every, N]) where row r
    holds <n_i> after step (r + 1) * every of the call."""
    _check_pulses(pulses, reg.n_atoms)
    if every < 1:
        raise ValueError("every must be >= 1")
    ptr = _state_ptr(d_psi, reg.n_atoms, reg.precision, "state")
    total = (pulses.omega.shape[-1] - 1) // opts.dt_ns
    first = opts.first_step
    steps = total - first if opts.n_steps < 0 else min(opts.n_steps, total - first)
    occ = np.zeros((max(steps, 0) // every, reg.n_atoms))
    st = Stats()
    _check(lib().rsv_evolve_device_observed(reg, C.byref(pulses.struct), C.byref(opts), ptr,
                                            _stream(stream), every,
                                            occ.ctypes.data_as(C.POINTER(C.c_double)), C.byref(st)))
    return st, occ


def rsv_energy_device(reg: Register, pulses: PulseArrays, step: int, dt_ns: int, d_psi,
                      stream=None) -> float:
    _check_pulses(pulses, reg.n_atoms)
    ptr = _state_ptr(d_psi, reg.n_atoms, reg.precision, "state")
    e = C.c_double()
    _check(lib().rsv_energy_device(reg, C.byref(pulses.struct), step, dt_ns, ptr, C.byref(e),
                                   _stream(stream)))
    return e.value


def rsv_evolve(reg: Register, pulses: PulseArrays, opts: EvolveOpts, psi0=None):
    _check_pulses(pulses, reg.n_atoms)
    h = C.c_void_p()
    buf = None if psi0 is None else _host_state(psi0, reg.n_atoms)
    _check(lib().rsv_evolve(reg, C.byref(pulses.struct), C.byref(opts),
                            buf.ctypes.data if buf is not None else None, C.byref(h)))
    return h


def rsv_result_state(res, n_atoms: int) -> np.ndarray:
    out = np.empty(1 << n_atoms, dtype=np.complex128)
    _check(lib().rsv_result_state(res, out.ctypes.data))
    return out


def rsv_result_occupations(res, n_atoms: int) -> np.ndarray:
    out = np.empty(n_atoms, dtype=np.float64)
    _check(lib().rsv_result_occupations(res, out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def rsv_result_sample(res, seed: int, n_shots: int) -> np.ndarray:
    out = np.empty(n_shots, dtype=np.uint64)
    _check(lib().rsv_result_sample(res, seed, n_shots, out.ctypes.data_as(C.POINTER(C.c_uint64))))
    return out


def rsv_result_stats(res) -> Stats:
    st = Stats()
    _check(lib().rsv_result_stats(res, C.byref(st)))
    return st


def rsv_result_destroy(res):
    lib().rsv_result_destroy(res)


def _atoms(n_atoms: int) -> int:
    if not 1 <= int(n_atoms) <= 30:
        raise ValueError("n_atoms must be in 1..30")
    return int(n_atoms)


def rsv_occupations_device(ctx, n_atoms: int, d_psi, precision="c128", stream=None) -> np.ndarray:
    prec, n = _prec(precision), _atoms(n_atoms)
    ptr = _state_ptr(d_psi, n, prec, "state")
    out = np.empty(n, dtype=np.float64)
    _check(lib().rsv_occupations_device(ctx, n, prec, ptr,
                                        out.ctypes.data_as(C.POINTER(C.c_double)),
                                        _stream(stream)))
    return out


def rsv_sample_device(ctx, n_atoms: int, d_psi, seed: int, n_shots: int, precision="c128",
                      stream=None) -> np.ndarray:
    prec, n = _prec(precision), _atoms(n_atoms)
    if n_shots < 0:
        raise ValueError("n_shots must be >= 0")
    ptr = _state_ptr(d_psi, n, prec, "state")
    out = np.empty(n_shots, dtype=np.uint64)
    _check(lib().rsv_sample_device(ctx, n, prec, ptr, seed, n_shots,
                                   out.ctypes.data_as(C.POINTER(C.c_uint64)), _stream(stream)))
    return out


def rsv_sample_device_static(ctx, n_atoms: int, d_psi, seed: int, n_shots: int,
                             precision="c128", stream=None) -> np.ndarray:
    prec, n = _prec(precision), _atoms(n_atoms)
    if n_shots < 0:
        raise ValueError("n_shots must be >= 0")
    ptr = _state_ptr(d_psi, n, prec, "state")
    out = np.empty(n_shots, dtype=np.uint64)
    _check(lib().rsv_sample_device_static(ctx, n, prec, ptr, seed, n_shots,
                                          out.ctypes.data_as(C.POINTER(C.c_uint64)),
                                          _stream(stream)))
    return out


def rsv_correlations_device(ctx, n_atoms: int, d_psi, precision="c128", stream=None) -> np.ndarray:
    prec, n = _prec(precision), _atoms(n_atoms)
    ptr = _state_ptr(d_psi, n, prec, "state")
    out = np.empty((n, n), dtype=np.float64)
    _check(lib().rsv_correlations_device(ctx, n, prec, ptr,
                                         out.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream)))
    return out


def _rho_ptr(buf, n_atoms: int, precision: int, what: str) -> int:
    return _dptr(buf, 1 << (2 * n_atoms), COMPLEX_DTYPE[precision], what)


def rsv_lindblad_apply(reg: Register, pulses: PulseArrays, step: int, dt_ns: int, rates, d_in,
                       d_out, stream=None):
    """d_out = L_step d_in; rates = (relax_rate, dephasing_rate) in 1/us."""
    _check_pulses(pulses, reg.n_atoms)
    pin = _rho_ptr(d_in, reg.n_atoms, reg.precision, "input density matrix")
    pout = _rho_ptr(d_out, reg.n_atoms, reg.precision, "output density matrix")
    _check(lib().rsv_lindblad_apply(reg, C.byref(pulses.struct), step, dt_ns,
                                    C.byref(Lindblad(*rates)), pin, pout, _stream(stream)))


def rsv_lindblad_evolve_device(reg: Register, pulses: PulseArrays, opts: EvolveOpts, rates, d_rho,
                               stream=None) -> Stats:
    _check_pulses(pulses, reg.n_atoms)
    ptr = _rho_ptr(d_rho, reg.n_atoms, reg.precision, "density matrix")
    st = Stats()
    _check(lib().rsv_lindblad_evolve_device(reg, C.byref(pulses.struct), C.byref(opts),
                                            C.byref(Lindblad(*rates)), ptr, _stream(stream),
                                            C.byref(st)))
    return st


def rsv_lindblad_occupations(ctx, n_atoms: int, d_rho, precision="c128", stream=None):
    """(<n_i> [N], trace) of a device density matrix."""
    prec, n = _prec(precision), _atoms(n_atoms)
    ptr = _rho_ptr(d_rho, n, prec, "density matrix")
    out, tr = np.empty(n), C.c_double()
    _check(lib().rsv_lindblad_occupations(ctx, n, prec, ptr, out.ctypes.data_as(C.POINTER(C.c_double)),
                                          C.byref(tr), _stream(stream)))
    return out, tr.value


def rsv_gradient_occupations(reg: Register, pulses: PulseArrays, opts: EvolveOpts, weights,
                             psi0=None):
    """(C, dC/dOmega [n_samples], dC/ddelta [n_samples], stats) for C = sum_i w_i <n_i>
    after the evolution, global pulses only."""
    _check_pulses(pulses, reg.n_atoms)
    if pulses.omega.ndim != 1:
        raise ValueError("gradients are taken for global pulses")
    w = _f64(weights).reshape(-1)
    if w.size != reg.n_atoms:
        raise ValueError(f"{w.size} weights for {reg.n_atoms} atoms")
    buf = None if psi0 is None else _host_state(psi0, reg.n_atoms)
    ns = pulses.omega.shape[-1]
    go, gd = np.zeros(ns), np.zeros(ns)
    val, st = C.c_double(), Stats()
    pd = C.POINTER(C.c_double)
    _check(lib().rsv_gradient_occupations(reg, C.byref(pulses.struct), C.byref(opts),
                                          w.ctypes.data_as(pd),
                                          buf.ctypes.data if buf is not None else None,
                                          C.byref(val), go.ctypes.data_as(pd), gd.ctypes.data_as(pd),
                                          C.byref(st)))
    return val.value, go, gd, st


def rsv_tridiag_expm(alpha, beta, tau: float):
    a, b = _f64(alpha), _f64(beta)
    m = a.size
    if b.size != max(m - 1, 0):
        raise ValueError("beta must have m - 1 entries")
    yr, yi = np.empty(m), np.empty(m)
    pd = C.POINTER(C.c_double)
    _check(lib().rsv_tridiag_expm(m, a.ctypes.data_as(pd), b.ctypes.data_as(pd) if m > 1 else None,
                                  float(tau), yr.ctypes.data_as(pd), yi.ctypes.data_as(pd)))
    return yr + 1j * yi


# ------------------------------------------------------------------------- serving
class ServerOpts(C.Structure):
    _fields_ = [("n_lanes", C.c_int), ("arena_bytes", C.c_size_t), ("max_queue", C.c_int),
                ("pack_max_atoms", C.c_int), ("pack_max_jobs", C.c_int)]


class JobDesc(C.Structure):
    _fields_ = [("n_atoms", C.c_int), ("xyz_um", C.POINTER(C.c_double)), ("c6", C.c_double),
                ("prec", C.c_int), ("pulses", Pulses), ("opts", EvolveOpts),
                ("psi0_host", C.c_void_p), ("n_shots", C.c_int), ("seed", C.c_uint64),
                ("return_state", C.c_int), ("tag", C.c_uint64), ("verify_fp64", C.c_int)]


class Completion(C.Structure):
    _fields_ = [("job_id", C.c_uint64), ("tag", C.c_uint64), ("status", C.c_int),
                ("n_atoms", C.c_int), ("n_shots", C.c_int), ("t_submit", C.c_double),
                ("t_start", C.c_double), ("t_end", C.c_double), ("stats", Stats),
                ("occupations", C.POINTER(C.c_double)), ("samples", C.POINTER(C.c_uint64)),
                ("state", C.c_void_p), ("error", C.c_char * 160),
                ("infidelity_fp64", C.c_double), ("max_occ_err_fp64", C.c_double)]


def _server_sigs(L):
    vp = C.c_void_p
    sig = {
        "rsv_server_create": (C.c_int, [vp, C.POINTER(ServerOpts), C.POINTER(vp)]),
        "rsv_server_job_bytes": (C.c_size_t, [C.c_int, C.c_int, C.c_int, C.c_int]),
        "rsv_server_submit": (C.c_int, [vp, C.POINTER(JobDesc), C.POINTER(C.c_uint64)]),
        "rsv_server_poll": (C.c_int, [vp, C.POINTER(Completion), C.c_int, C.POINTER(C.c_int),
                                      C.c_int]),
        "rsv_server_release": (None, [vp, C.POINTER(Completion)]),
        "rsv_server_cancel": (C.c_int, [vp, C.c_uint64]),
        "rsv_server_status": (C.c_int, [vp, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                        C.POINTER(C.c_int), C.POINTER(C.c_size_t)]),
        "rsv_server_destroy": (None, [vp]),
        "rsv_noise_member": (C.c_int, [C.POINTER(Noise), C.c_uint64, C.c_int, C.c_int64,
                                       C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "rsv_server_submit_ensemble": (C.c_int, [vp, C.POINTER(JobDesc), C.POINTER(Noise),
                                                 C.c_uint64, C.c_int, C.POINTER(C.c_uint64)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args


EXPORTED += ["rsv_server_create", "rsv_server_job_bytes", "rsv_server_submit", "rsv_server_poll",
             "rsv_server_release", "rsv_server_cancel", "rsv_server_status", "rsv_server_destroy",
             "rsv_noise_member", "rsv_server_submit_ensemble"]


class Noise(C.Structure):
    _fields_ = [("omega_rel_sigma", C.c_double), ("delta_sigma", C.c_double),
                ("position_sigma_um", C.c_double)]


def _slib():
    L = lib()
    if not getattr(L, "_server_sigs", False):
        _server_sigs(L)
        L._server_sigs = True
    return L


def rsv_server_create(ctx, n_lanes: int = 4, arena_bytes: int = 0, max_queue: int = 0,
                      pack_max_atoms: int = 0, pack_max_jobs: int = 0):
    h = C.c_void_p()
    opts = ServerOpts(n_lanes, arena_bytes, max_queue, pack_max_atoms, pack_max_jobs)
    _check(_slib().rsv_server_create(ctx, C.byref(opts), C.byref(h)))
    return h


def rsv_server_job_bytes(n_atoms: int, kmax: int, precision="c64", n_shots: int = 0) -> int:
    return int(_slib().rsv_server_job_bytes(n_atoms, kmax, PRECISIONS.get(precision, precision),
                                            n_shots))


def rsv_server_submit(srv, xyz, c6, pulses: PulseArrays, opts: EvolveOpts, precision="c64",
                      psi0=None, n_shots: int = 0, seed: int = 0, return_state: bool = False,
                      tag: int = 0, verify_fp64: bool = False) -> int:
    xyz = _f64(xyz).reshape(-1, 3)
    _check_pulses(pulses, xyz.shape[0])
    buf = None if psi0 is None else _host_state(psi0, xyz.shape[0])
    jd = JobDesc(xyz.shape[0], xyz.ctypes.data_as(C.POINTER(C.c_double)), float(c6),
                 PRECISIONS.get(precision, precision), pulses.struct, opts,
                 buf.ctypes.data if buf is not None else None, n_shots, seed, int(return_state), tag,
                 int(verify_fp64))
    jid = C.c_uint64()
    _check(_slib().rsv_server_submit(srv, C.byref(jd), C.byref(jid)))
    return int(jid.value)


def rsv_noise_member(noise, noise_seed: int, xyz, member: int):
    """(omega factor, delta offsets [N], displaced positions [N, 3]) of ensemble member
    `member`; noise is (omega_rel_sigma, delta_sigma, position_sigma_um)."""
    xyz = _f64(xyz).reshape(-1, 3)
    n = xyz.shape[0]
    f = C.c_double()
    off, pos = np.empty(n), np.empty((n, 3))
    pd = C.POINTER(C.c_double)
    _check(_slib().rsv_noise_member(C.byref(Noise(*noise)), noise_seed, n, member,
                                    xyz.ctypes.data_as(pd), C.byref(f), off.ctypes.data_as(pd),
                                    pos.ctypes.data_as(pd)))
    return f.value, off, pos


def rsv_server_submit_ensemble(srv, xyz, c6, pulses: PulseArrays, opts: EvolveOpts, noise,
                               noise_seed: int, n_members: int, precision="c64", psi0=None,
                               n_shots: int = 0, seed: int = 0, return_state: bool = False,
                               tag: int = 0):
    """Queues n_members noisy copies of a job; returns their ids (member order)."""
    xyz = _f64(xyz).reshape(-1, 3)
    _check_pulses(pulses, xyz.shape[0])
    buf = None if psi0 is None else _host_state(psi0, xyz.shape[0])
    jd = JobDesc(xyz.shape[0], xyz.ctypes.data_as(C.POINTER(C.c_double)), float(c6),
                 PRECISIONS.get(precision, precision), pulses.struct, opts,
                 buf.ctypes.data if buf is not None else None, n_shots, seed, int(return_state), tag)
    ids = np.zeros(max(int(n_members), 0), dtype=np.uint64)
    _check(_slib().rsv_server_submit_ensemble(srv, C.byref(jd), C.byref(Noise(*noise)), noise_seed,
                                              int(n_members),
                                              ids.ctypes.data_as(C.POINTER(C.c_uint64))))
    return [int(i) for i in ids]


def rsv_server_poll(srv, max_n: int = 64, timeout_ms: int = -1):
    """Completed jobs as dicts (arrays copied out; the server's copies are released)."""
    arr = (Completion * max_n)()
    got = C.c_int()
    _check(_slib().rsv_server_poll(srv, arr, max_n, C.byref(got), timeout_ms))
    out = []
    for i in range(got.value):
        c = arr[i]
        d = {"job_id": int(c.job_id), "tag": int(c.tag), "status": int(c.status),
             "n_atoms": int(c.n_atoms), "t_submit": c.t_submit, "t_start": c.t_start,
             "t_end": c.t_end, "stats": c.stats.as_dict(), "error": c.error.decode(errors="replace"),
             "infidelity_fp64": c.infidelity_fp64, "max_occ_err_fp64": c.max_occ_err_fp64,
             "occupations": None, "samples": None, "state": None}
        if c.occupations:
            d["occupations"] = np.ctypeslib.as_array(c.occupations, (c.n_atoms,)).copy()
        if c.samples and c.n_shots > 0:
            d["samples"] = np.ctypeslib.as_array(c.samples, (c.n_shots,)).copy()
        if c.state:
            dim = 1 << c.n_atoms
            raw = np.ctypeslib.as_array(C.cast(c.state, C.POINTER(C.c_double)), (2 * dim,))
            d["state"] = raw.view(np.complex128).copy()
        _slib().rsv_server_release(srv, C.byref(arr[i]))
        out.append(d)
    return out


def rsv_server_cancel(srv, job_id: int):
    _check(_slib().rsv_server_cancel(srv, job_id))


def rsv_server_status(srv):
    q, r, d, used = C.c_int(), C.c_int(), C.c_int(), C.c_size_t()
    _check(_slib().rsv_server_status(srv, C.byref(q), C.byref(r), C.byref(d), C.byref(used)))
    return {"queued": q.value, "running": r.value, "done": d.value, "arena_used": used.value}


def rsv_server_destroy(srv):
    _slib().rsv_server_destroy(srv)
