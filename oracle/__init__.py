"""FP64 CPU oracle for the error-injecting state-vector simulator.

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import this package; the GPU library and its
Python binding never do.  The arithmetic lives in ``qsim_oracle.c`` (plain C,
complex double, one gate at a time over the whole vector); this module only
compiles it with gcc and marshals numpy arrays through ctypes.

States are numpy float64 arrays of length 2 * 2**M, interleaved re/im, index
bit q = qubit q (Sec. 1.2, Fig. 1 of the paper).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

from circuitgen import GATE_DTYPE

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qsim_oracle.c")
_SRC3 = os.path.join(_HERE, "qtrit_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, OpenMP pair loops)."""
    stale = not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(_SRC), os.path.getmtime(_SRC3))
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-fopenmp", "-Wall", "-o", tmp, _SRC, _SRC3, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Errors(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("p_bitflip", ctypes.c_double),
                ("p_phaseflip", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("trial", ctypes.c_uint64)]


@dataclass
class Errors:
    """Error model: per-gate angle error N(0, sigma^2) and per-qubit-per-step
    bit/phase flip probabilities, keyed by (seed, trial)."""
    sigma: float = 0.0
    p_bitflip: float = 0.0
    p_phaseflip: float = 0.0
    seed: int = 0
    trial: int = 0

    def _c(self) -> _Errors:
        return _Errors(self.sigma, self.p_bitflip, self.p_phaseflip, self.seed, self.trial)


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        ep = ctypes.POINTER(_Errors)
        L.oq_philox4x64_10.argtypes = [u64p, u64p, u64p]
        L.oq_gauss.argtypes = [ep, ctypes.c_uint64]
        L.oq_gauss.restype = ctypes.c_double
        L.oq_angle_error.argtypes = [ep, ctypes.c_uint64]
        L.oq_angle_error.restype = ctypes.c_double
        L.oq_flip_events.argtypes = [ep, ctypes.c_uint64, ctypes.c_int]
        L.oq_flip_events.restype = ctypes.c_int
        L.oq_gate_matrix.argtypes = [ctypes.c_uint32, ctypes.c_double, ctypes.c_double, dp]
        L.oq_gate_matrix.restype = ctypes.c_int
        L.oq_apply_matrix.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, dp]
        L.oq_apply_swap.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_uint64]
        L.oq_apply_negate.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_uint64]
        L.oq_init.argtypes = [dp, ctypes.c_int, ctypes.c_uint64]
        L.oq_run.argtypes = [dp, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ep,
                             ctypes.c_uint64]
        L.oq_run.restype = ctypes.c_int
        L.oq_overlap.argtypes = [dp, dp, ctypes.c_int, dp]
        L.oq_fidelity.argtypes = [dp, dp, ctypes.c_int]
        L.oq_fidelity.restype = ctypes.c_double
        L.oq_probs.argtypes = [dp, ctypes.c_int, ctypes.c_uint64, dp]
        L.oq_run_trials.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ep,
                                    ctypes.c_uint64, dp]
        L.oq_run_trials.restype = ctypes.c_int
        L.oq_num_threads.restype = ctypes.c_int
        L.oq_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _gates(g) -> np.ndarray:
    return np.ascontiguousarray(g, dtype=GATE_DTYPE)


def philox4x64_10(counter, key) -> np.ndarray:
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    p = ctypes.POINTER(ctypes.c_uint64)
    lib().oq_philox4x64_10(c.ctypes.data_as(p), k.ctypes.data_as(p), out.ctypes.data_as(p))
    return out


def gauss(errors: Errors, step: int) -> float:
    e = errors._c()
    return lib().oq_gauss(ctypes.byref(e), step)


def angle_error(errors: Errors | None, step: int) -> float:
    if errors is None:
        return 0.0
    e = errors._c()
    return lib().oq_angle_error(ctypes.byref(e), step)


def flip_events(errors: Errors | None, step: int, qubit: int) -> int:
    if errors is None:
        return 0
    e = errors._c()
    return lib().oq_flip_events(ctypes.byref(e), step, qubit)


def gate_matrix(kind: int, theta: float = 0.0, eps: float = 0.0):
    """(form, U) with U a 2x2 complex array; form 0 = general, 1 = exact swap,
    2 = exact sign flip of |1>."""
    u = np.zeros(8)
    form = lib().oq_gate_matrix(kind, theta, eps, _dp(u))
    if form < 0:
        raise ValueError("unknown gate kind %d" % kind)
    U = (u[0::2] + 1j * u[1::2]).reshape(2, 2)
    return form, U


def init(M: int, k: int = 0) -> np.ndarray:
    psi = np.empty(2 << M, dtype=np.float64)
    lib().oq_init(_dp(psi), M, k)
    return psi


def apply_matrix(psi, M, target, cmask, U):
    u = np.empty(8)
    u[0::2] = np.real(np.asarray(U).ravel())
    u[1::2] = np.imag(np.asarray(U).ravel())
    lib().oq_apply_matrix(_dp(psi), M, target, cmask, _dp(u))
    return psi


def apply_swap(psi, M, target, cmask=0):
    lib().oq_apply_swap(_dp(psi), M, target, cmask)
    return psi


def apply_negate(psi, M, target, cmask=0):
    lib().oq_apply_negate(_dp(psi), M, target, cmask)
    return psi


def run(psi: np.ndarray, M: int, gates, errors: Errors | None = None, step0: int = 0) -> np.ndarray:
    g = _gates(gates)
    e = errors._c() if errors is not None else None
    rc = lib().oq_run(_dp(psi), M, g.ctypes.data, len(g),
                      ctypes.byref(e) if e is not None else None, step0)
    if rc != 0:
        raise ValueError("oracle rejected the circuit or error model")
    return psi


def simulate(M: int, gates, errors: Errors | None = None, k: int = 0) -> np.ndarray:
    return run(init(M, k), M, gates, errors)


def overlap(a, b, M):
    out = np.zeros(4)
    lib().oq_overlap(_dp(a), _dp(b), M, _dp(out))
    return complex(out[0], out[1]), float(out[2]), float(out[3])


def fidelity(a, b, M) -> float:
    return float(lib().oq_fidelity(_dp(a), _dp(b), M))


def probs(psi, M, mask=None) -> np.ndarray:
    if mask is None:
        mask = (1 << M) - 1
    m = bin(mask).count("1")
    out = np.zeros(1 << m)
    lib().oq_probs(_dp(psi), M, mask, _dp(out))
    return out


def run_trials(gates, M, errors: Errors, n_trials: int) -> np.ndarray:
    g = _gates(gates)
    out = np.zeros(n_trials)
    e = errors._c()
    rc = lib().oq_run_trials(g.ctypes.data, len(g), M, ctypes.byref(e), n_trials, _dp(out))
    if rc != 0:
        raise ValueError("oracle rejected the trials")
    return out


def num_threads() -> int:
    return int(lib().oq_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the pair loops from now on (timing only; results do not
    depend on it)."""
    lib().oq_set_num_threads(int(n))


def as_complex(psi: np.ndarray) -> np.ndarray:
    return psi[0::2] + 1j * psi[1::2]


# ------------------------------------------------------- three-state model

class _Pulse3(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("ion", ctypes.c_int32), ("a", ctypes.c_int32),
                ("b", ctypes.c_int32), ("cond_ion", ctypes.c_int32),
                ("cond_level", ctypes.c_int32), ("theta", ctypes.c_double),
                ("phi", ctypes.c_double)]


PULSE_ROT, PULSE_PHASE = 0, 1


def _lib3():
    L = lib()
    if not hasattr(L, "_q3_ready"):
        dp = ctypes.POINTER(ctypes.c_double)
        ep = ctypes.POINTER(_Errors)
        pp = ctypes.POINTER(_Pulse3)
        L.oq3_lower_gate.argtypes = [ctypes.c_void_p, pp, ctypes.c_size_t]
        L.oq3_lower_gate.restype = ctypes.c_size_t
        L.oq3_pulse_matrix.argtypes = [pp, ctypes.c_double, dp]
        L.oq3_apply_pulse.argtypes = [dp, ctypes.c_int, pp, ctypes.c_double]
        L.oq3_init.argtypes = [dp, ctypes.c_int, ctypes.c_uint64]
        L.oq3_run.argtypes = [dp, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ep,
                              ctypes.c_uint64]
        L.oq3_run.restype = ctypes.c_int
        L.oq3_probs.argtypes = [dp, ctypes.c_int, ctypes.c_uint64, dp]
        L._q3_ready = True
    return L


def _pulse(p) -> _Pulse3:
    return _Pulse3(int(p["kind"]), int(p["ion"]), int(p.get("a", 0)), int(p.get("b", 1)),
                   int(p.get("cond_ion", -1)), int(p.get("cond_level", 0)),
                   float(p.get("theta", 0.0)), float(p.get("phi", 0.0)))


def lower3(gate) -> list:
    """The three-state model's transformations of one gate (list of dicts)."""
    g = np.ascontiguousarray(np.array([gate], dtype=GATE_DTYPE))
    buf = (_Pulse3 * 64)()
    n = _lib3().oq3_lower_gate(g.ctypes.data, buf, 64)
    return [{f: getattr(buf[i], f) for f, _ in _Pulse3._fields_} for i in range(n)]


def pulse_matrix3(pulse, eps: float = 0.0) -> np.ndarray:
    u = np.zeros(8)
    p = _pulse(pulse)
    _lib3().oq3_pulse_matrix(ctypes.byref(p), eps, _dp(u))
    return (u[0::2] + 1j * u[1::2]).reshape(2, 2)


def init3(M: int, k: int = 0) -> np.ndarray:
    psi = np.empty(2 * 3 ** M, dtype=np.float64)
    _lib3().oq3_init(_dp(psi), M, k)
    return psi


def apply_pulse3(psi, M, pulse, eps: float = 0.0):
    p = _pulse(pulse)
    _lib3().oq3_apply_pulse(_dp(psi), M, ctypes.byref(p), eps)
    return psi


def run3(psi, M, gates, errors: Errors | None = None, step0: int = 0):
    g = _gates(gates)
    e = errors._c() if errors is not None else None
    rc = _lib3().oq3_run(_dp(psi), M, g.ctypes.data, len(g),
                         ctypes.byref(e) if e is not None else None, step0)
    if rc != 0:
        raise ValueError("three-state oracle rejected the circuit or error model")
    return psi


def simulate3(M: int, gates, errors: Errors | None = None, k: int = 0) -> np.ndarray:
    return run3(init3(M, k), M, gates, errors)


def probs3(psi, M, mask=None) -> np.ndarray:
    if mask is None:
        mask = (1 << M) - 1
    out = np.zeros(3 ** bin(mask).count("1"))
    _lib3().oq3_probs(_dp(psi), M, mask, _dp(out))
    return out
