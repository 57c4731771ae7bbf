"""Python binding of the qsim HIP library (libqsim.so, C-ABI in include/qsim.h).

Argument marshalling only: every step of the simulation runs in the library's
HIP kernels on the GPU.  The functions keep the C names (``qsim_create``,
``qsim_apply_circuit``, ``qsim_inject_errors``, ``qsim_fidelity``,
``qsim_probs`` ...) and raise ``QsimError`` on a negative status.  ``State`` is
a small convenience wrapper over a handle.  If the library has not been built
(``python -m paper_quant_ph_9804039_amd._build``) loading fails loudly: there
is no CPU fallback.

PyTorch is only plumbing here: ``torch_options`` lets a state live in a torch
tensor's memory and run on a torch stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from circuitgen import GATE_DTYPE

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsim.so")

QSIM_OK, QSIM_EINVAL, QSIM_ENOMEM, QSIM_EDEVICE, QSIM_ERANGE = 0, -1, -2, -3, -4
QSIM_C64, QSIM_C128 = 0, 1
QSIM_H, QSIM_RZ, QSIM_X, QSIM_CNOT, QSIM_TOFFOLI, QSIM_Z, QSIM_CPHASE = 0, 1, 2, 3, 4, 5, 6
QSIM_MAX_QUBITS = 34

EXPORTED = [
    "qsim_create", "qsim_destroy", "qsim_reset", "qsim_apply_circuit", "qsim_apply_inverse",
    "qsim_inject_errors", "qsim_fidelity", "qsim_overlap", "qsim_norm", "qsim_probs",
    "qsim_get_amplitudes", "qsim_set_amplitudes", "qsim_run_trials", "qsim_synchronize",
    "qsim_info", "qsim_profile", "qsim_get_stats", "qsim_last_error", "qsim_plan", "qsim_serve",
    "qsim_trial_plan", "qsim_overlap_noalloc", "qsim_touched_qubits",
    "qsim3_create", "qsim3_destroy", "qsim3_reset", "qsim3_inject_errors", "qsim3_apply_circuit",
    "qsim3_apply_pulses", "qsim3_lower", "qsim3_overlap", "qsim3_fidelity", "qsim3_probs",
    "qsim3_get_amplitudes", "qsim3_synchronize", "qsim3_info",
]


class QsimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"qsim status {code}: {msg}")
        self.code = code


class qsim_error_model(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("p_bitflip", ctypes.c_double),
                ("p_phaseflip", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("trial", ctypes.c_uint64)]


class qsim_options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("hip_stream", ctypes.c_void_p),
                ("ext_buffer", ctypes.c_void_p), ("ext_bytes", ctypes.c_size_t),
                ("renorm_period", ctypes.c_int), ("exec_mode", ctypes.c_int),
                ("tile_bits", ctypes.c_int), ("low_bits", ctypes.c_int),
                ("group_bits", ctypes.c_int), ("lazy_qubits", ctypes.c_int),
                ("remap_qubits", ctypes.c_int)]


class qsim_stats(ctypes.Structure):
    _fields_ = [("gates", ctypes.c_uint64), ("flips", ctypes.c_uint64),
                ("passes", ctypes.c_uint64), ("fused_passes", ctypes.c_uint64),
                ("renorms", ctypes.c_uint64), ("pass_ms", ctypes.c_double),
                ("pass_bytes", ctypes.c_double), ("fused_ms", ctypes.c_double),
                ("fused_bytes", ctypes.c_double), ("other_ms", ctypes.c_double),
                ("fused_flops", ctypes.c_double), ("remaps", ctypes.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class qsim_pass_info(ctypes.Structure):
    _fields_ = [("fused", ctypes.c_uint32), ("first_op", ctypes.c_uint32),
                ("n_ops", ctypes.c_uint32), ("n_groups", ctypes.c_uint32),
                ("norm_after", ctypes.c_uint32), ("span_qubits", ctypes.c_uint32),
                ("tile_mask", ctypes.c_uint64), ("flops", ctypes.c_double),
                ("tiles", ctypes.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class qsim3_pulse(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("ion", ctypes.c_int32), ("a", ctypes.c_int32),
                ("b", ctypes.c_int32), ("cond_ion", ctypes.c_int32),
                ("cond_level", ctypes.c_int32), ("theta", ctypes.c_double),
                ("phi", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class qsim_request(ctypes.Structure):
    _fields_ = [("num_qubits", ctypes.c_int), ("dtype", ctypes.c_int),
                ("gates", ctypes.c_void_p), ("n_gates", ctypes.c_size_t),
                ("errors", qsim_error_model), ("arrival_s", ctypes.c_double)]


class qsim_result(ctypes.Structure):
    _fields_ = [("fidelity", ctypes.c_double), ("admit_s", ctypes.c_double),
                ("done_s", ctypes.c_double), ("status", ctypes.c_int), ("slot", ctypes.c_int)]


class qsim_serve_options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("max_slots", ctypes.c_int),
                ("hbm_budget", ctypes.c_size_t), ("strict_fifo", ctypes.c_int),
                ("max_heavy", ctypes.c_int), ("heavy_bytes", ctypes.c_size_t)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libqsim.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_quant_ph_9804039_amd._build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, sz, dp = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_size_t, ctypes.POINTER(ctypes.c_double)
    sig = {
        "qsim_create": [ctypes.c_int, ctypes.c_int, ctypes.POINTER(qsim_options), ctypes.POINTER(vp)],
        "qsim_destroy": [vp],
        "qsim_reset": [vp, u64],
        "qsim_apply_circuit": [vp, vp, sz],
        "qsim_apply_inverse": [vp, vp, sz],
        "qsim_inject_errors": [vp, ctypes.POINTER(qsim_error_model)],
        "qsim_fidelity": [vp, vp, dp],
        "qsim_overlap": [vp, vp, dp],
        "qsim_norm": [vp, dp],
        "qsim_probs": [vp, u64, dp, sz],
        "qsim_get_amplitudes": [vp, u64, u64, dp],
        "qsim_set_amplitudes": [vp, u64, u64, dp],
        "qsim_run_trials": [vp, sz, ctypes.c_int, ctypes.c_int, ctypes.POINTER(qsim_error_model),
                            u64, dp],
        "qsim_synchronize": [vp],
        "qsim_info": [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                      ctypes.POINTER(u64), ctypes.POINTER(vp), ctypes.POINTER(sz)],
        "qsim_profile": [vp, ctypes.c_int],
        "qsim_get_stats": [vp, ctypes.POINTER(qsim_stats)],
        "qsim_plan": [ctypes.c_int, ctypes.c_int, ctypes.POINTER(qsim_options), vp, sz,
                      ctypes.POINTER(qsim_error_model), u64, ctypes.POINTER(qsim_pass_info), sz,
                      ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(ctypes.c_uint32), sz],
        "qsim_serve": [ctypes.POINTER(qsim_request), sz, ctypes.POINTER(qsim_serve_options),
                       ctypes.POINTER(qsim_result)],
        "qsim_trial_plan": [vp, sz, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_uint32),
                            sz, ctypes.POINTER(sz)],
        "qsim_overlap_noalloc": [vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 vp, dp],
        "qsim_touched_qubits": [vp, ctypes.POINTER(u64)],
        "qsim3_create": [ctypes.c_int, ctypes.c_int, ctypes.POINTER(qsim_options), ctypes.POINTER(vp)],
        "qsim3_destroy": [vp],
        "qsim3_reset": [vp, u64],
        "qsim3_inject_errors": [vp, ctypes.POINTER(qsim_error_model)],
        "qsim3_apply_circuit": [vp, vp, sz],
        "qsim3_apply_pulses": [vp, ctypes.POINTER(qsim3_pulse), sz],
        "qsim3_lower": [vp, sz, ctypes.c_int, ctypes.POINTER(qsim3_pulse), sz, ctypes.POINTER(sz)],
        "qsim3_overlap": [vp, vp, dp],
        "qsim3_fidelity": [vp, vp, dp],
        "qsim3_probs": [vp, u64, dp, sz],
        "qsim3_get_amplitudes": [vp, u64, u64, dp],
        "qsim3_synchronize": [vp],
        "qsim3_info": [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                       ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u64)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.qsim_last_error.argtypes = []
    L.qsim_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc: int) -> int:
    if rc != QSIM_OK:
        msg = lib().qsim_last_error().decode(errors="replace")
        raise QsimError(rc, msg)
    return rc


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _gates(g) -> np.ndarray:
    return np.ascontiguousarray(g, dtype=GATE_DTYPE)


def _em(sigma=0.0, p_bitflip=0.0, p_phaseflip=0.0, seed=0, trial=0) -> qsim_error_model:
    return qsim_error_model(float(sigma), float(p_bitflip), float(p_phaseflip), int(seed), int(trial))


# ------------------------------------------------------------ C-ABI wrappers

def qsim_create(num_qubits: int, dtype: int = QSIM_C64, options: qsim_options | None = None):
    h = ctypes.c_void_p()
    _check(lib().qsim_create(num_qubits, dtype, ctypes.byref(options) if options else None,
                             ctypes.byref(h)))
    return h


def qsim_destroy(h) -> None:
    _check(lib().qsim_destroy(h))


def qsim_reset(h, basis_index: int = 0) -> None:
    _check(lib().qsim_reset(h, basis_index))


def qsim_apply_circuit(h, gates) -> None:
    g = _gates(gates)
    _check(lib().qsim_apply_circuit(h, g.ctypes.data, len(g)))


def qsim_apply_inverse(h, gates) -> None:
    g = _gates(gates)
    _check(lib().qsim_apply_inverse(h, g.ctypes.data, len(g)))


def qsim_inject_errors(h, sigma=None, p_bitflip=0.0, p_phaseflip=0.0, seed=0, trial=0) -> None:
    """Arm the error model; ``sigma=None`` disarms it."""
    if sigma is None:
        _check(lib().qsim_inject_errors(h, None))
    else:
        em = _em(sigma, p_bitflip, p_phaseflip, seed, trial)
        _check(lib().qsim_inject_errors(h, ctypes.byref(em)))


def qsim_fidelity(a, b) -> float:
    out = ctypes.c_double()
    _check(lib().qsim_fidelity(a, b, ctypes.byref(out)))
    return out.value


def qsim_overlap(a, b):
    out = np.zeros(4)
    _check(lib().qsim_overlap(a, b, _dp(out)))
    return complex(out[0], out[1]), float(out[2]), float(out[3])


def qsim_overlap_noalloc(ptr_a: int, dtype_a: int, ptr_b: int, dtype_b: int, num_qubits: int,
                         device: int = 0, hip_stream=None):
    """Overlap of two caller-owned device registers (raw device addresses);
    allocates nothing.  Returns (<a|b>, <a|a>, <b|b>)."""
    out = np.zeros(4)
    _check(lib().qsim_overlap_noalloc(ptr_a, dtype_a, ptr_b, dtype_b, num_qubits, device,
                                      hip_stream, _dp(out)))
    return complex(out[0], out[1]), float(out[2]), float(out[3])


def qsim_norm(h) -> float:
    out = ctypes.c_double()
    _check(lib().qsim_norm(h, ctypes.byref(out)))
    return out.value


def qsim_probs(h, qubit_mask: int | None = None) -> np.ndarray:
    M = qsim_info(h)["num_qubits"]
    if qubit_mask is None:
        qubit_mask = (1 << M) - 1
    n = 1 << bin(qubit_mask).count("1")
    out = np.zeros(n)
    _check(lib().qsim_probs(h, qubit_mask, _dp(out), n))
    return out


def qsim_get_amplitudes(h, offset: int = 0, count: int | None = None) -> np.ndarray:
    """Amplitudes [offset, offset+count) as a complex128 numpy array."""
    M = qsim_info(h)["num_qubits"]
    if count is None:
        count = (1 << M) - offset
    out = np.zeros(2 * count)
    _check(lib().qsim_get_amplitudes(h, offset, count, _dp(out)))
    return out[0::2] + 1j * out[1::2]


def qsim_set_amplitudes(h, values, offset: int = 0) -> None:
    v = np.asarray(values)
    if np.iscomplexobj(v):
        buf = np.empty(2 * len(v))
        buf[0::2], buf[1::2] = v.real, v.imag
    else:
        buf = np.ascontiguousarray(v, dtype=np.float64)
    _check(lib().qsim_set_amplitudes(h, offset, len(buf) // 2, _dp(buf)))


def qsim_run_trials(gates, num_qubits: int, dtype: int, sigma=0.0, p_bitflip=0.0,
                    p_phaseflip=0.0, seed=0, trial=0, n_trials: int = 1) -> np.ndarray:
    g = _gates(gates)
    em = _em(sigma, p_bitflip, p_phaseflip, seed, trial)
    out = np.zeros(n_trials)
    _check(lib().qsim_run_trials(g.ctypes.data, len(g), num_qubits, dtype, ctypes.byref(em),
                                 n_trials, _dp(out)))
    return out


def qsim_synchronize(h) -> None:
    _check(lib().qsim_synchronize(h))


def qsim_info(h) -> dict:
    M, dt, step, ptr, nb = (ctypes.c_int(), ctypes.c_int(), ctypes.c_uint64(), ctypes.c_void_p(),
                            ctypes.c_size_t())
    _check(lib().qsim_info(h, ctypes.byref(M), ctypes.byref(dt), ctypes.byref(step),
                           ctypes.byref(ptr), ctypes.byref(nb)))
    return {"num_qubits": M.value, "dtype": dt.value, "step": step.value,
            "device_ptr": ptr.value, "bytes": nb.value}


def qsim_touched_qubits(h) -> int:
    m = ctypes.c_uint64()
    _check(lib().qsim_touched_qubits(h, ctypes.byref(m)))
    return m.value


def qsim_profile(h, enable: bool) -> None:
    _check(lib().qsim_profile(h, 1 if enable else 0))


def qsim_get_stats(h) -> dict:
    st = qsim_stats()
    _check(lib().qsim_get_stats(h, ctypes.byref(st)))
    return st.as_dict()


def qsim_plan(num_qubits: int, dtype: int, gates, options: qsim_options | None = None,
              sigma=None, p_bitflip=0.0, p_phaseflip=0.0, seed=0, trial=0, step0: int = 0,
              return_order: bool = False):
    """Host-only dry run of the pass schedule: (list of pass dicts, op count),
    plus the execution order (stream index of each executed operation) when
    return_order is set."""
    g = _gates(gates)
    em = None if sigma is None else _em(sigma, p_bitflip, p_phaseflip, seed, trial)
    npass, nops = ctypes.c_size_t(), ctypes.c_size_t()
    L = lib()
    opt = ctypes.byref(options) if options else None
    emp = ctypes.byref(em) if em else None
    _check(L.qsim_plan(num_qubits, dtype, opt, g.ctypes.data, len(g), emp, step0, None, 0,
                       ctypes.byref(npass), ctypes.byref(nops), None, 0))
    out = (qsim_pass_info * max(1, npass.value))()
    order = np.zeros(max(1, nops.value), dtype=np.uint32)
    _check(L.qsim_plan(num_qubits, dtype, opt, g.ctypes.data, len(g), emp, step0, out,
                       npass.value, ctypes.byref(npass), ctypes.byref(nops),
                       order.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), nops.value))
    passes = [out[i].as_dict() for i in range(npass.value)]
    if return_order:
        return passes, nops.value, order[:nops.value]
    return passes, nops.value


def qsim_trial_plan(gates, num_qubits: int, group_bits: int) -> np.ndarray:
    """Host-only dry run of the Monte Carlo register-group schedule: one row
    per group, (first gate, gate count, qubit mask, uncontrolled Hadamards)."""
    g = _gates(gates)
    n = ctypes.c_size_t()
    L = lib()
    _check(L.qsim_trial_plan(g.ctypes.data, len(g), num_qubits, group_bits, None, 0,
                             ctypes.byref(n)))
    out = np.zeros((max(1, n.value), 4), dtype=np.uint32)
    _check(L.qsim_trial_plan(g.ctypes.data, len(g), num_qubits, group_bits,
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), n.value,
                             ctypes.byref(n)))
    return out[:n.value]


def qsim_serve(requests, max_slots: int = 8, hbm_budget: int = 0, strict_fifo: bool = False,
               device: int = 0, max_heavy: int = 0, heavy_bytes: int = 0):
    """Serve a list of requests (dicts with keys M, dtype, gates, sigma,
    p_bitflip, p_phaseflip, seed, trial, arrival_s) with continuous batching;
    returns one result dict per request (fidelity, admit_s, done_s, status,
    slot)."""
    n = len(requests)
    arr = (qsim_request * max(1, n))()
    keep = []
    for i, r in enumerate(requests):
        g = _gates(r["gates"])
        keep.append(g)
        arr[i] = qsim_request(int(r["M"]), int(r.get("dtype", QSIM_C64)), g.ctypes.data, len(g),
                              _em(r.get("sigma", 0.0), r.get("p_bitflip", 0.0),
                                  r.get("p_phaseflip", 0.0), r.get("seed", 0), r.get("trial", 0)),
                              float(r.get("arrival_s", 0.0)))
    out = (qsim_result * max(1, n))()
    opt = qsim_serve_options(device, max_slots, hbm_budget, 1 if strict_fifo else 0, max_heavy,
                             heavy_bytes)
    _check(lib().qsim_serve(arr, n, ctypes.byref(opt), out))
    return [{f: getattr(out[i], f) for f, _ in qsim_result._fields_} for i in range(n)]


def qsim_last_error() -> str:
    return lib().qsim_last_error().decode(errors="replace")


# --------------------------------------------------------------- helpers

def make_options(device=0, hip_stream=None, ext_buffer=None, ext_bytes=0, renorm_period=0,
                 exec_mode=0, tile_bits=0, low_bits=0, group_bits=0,
                 lazy_qubits=0, remap_qubits=0) -> qsim_options:
    return qsim_options(device, hip_stream, ext_buffer, ext_bytes, renorm_period, exec_mode,
                        tile_bits, low_bits, group_bits, lazy_qubits, remap_qubits)


def torch_options(tensor=None, stream=None, **kw) -> qsim_options:
    """Options that place the state in ``tensor``'s device memory (borrowed; the
    tensor must outlive the state) and/or queue its work on a torch stream."""
    ext, nbytes, dev = None, 0, kw.pop("device", None)
    if tensor is not None:
        ext, nbytes = tensor.data_ptr(), tensor.numel() * tensor.element_size()
        if dev is None:
            dev = tensor.device.index or 0
    hs = stream.cuda_stream if stream is not None else None
    return make_options(device=dev or 0, hip_stream=hs, ext_buffer=ext, ext_bytes=nbytes, **kw)


class State:
    """Owning wrapper of one register."""

    def __init__(self, num_qubits: int, dtype: int = QSIM_C64, options: qsim_options | None = None):
        self.num_qubits = num_qubits
        self.dtype = dtype
        self._opt = options  # keep alive
        self.h = qsim_create(num_qubits, dtype, options)

    def close(self):
        if self.h is not None:
            qsim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def reset(self, basis_index: int = 0):
        qsim_reset(self.h, basis_index)
        return self

    def apply(self, gates):
        qsim_apply_circuit(self.h, gates)
        return self

    def apply_inverse(self, gates):
        qsim_apply_inverse(self.h, gates)
        return self

    def inject_errors(self, sigma=None, p_bitflip=0.0, p_phaseflip=0.0, seed=0, trial=0):
        qsim_inject_errors(self.h, sigma, p_bitflip, p_phaseflip, seed, trial)
        return self

    def fidelity(self, other: "State") -> float:
        return qsim_fidelity(self.h, other.h)

    def overlap(self, other: "State"):
        return qsim_overlap(self.h, other.h)

    def norm(self) -> float:
        return qsim_norm(self.h)

    def probs(self, qubit_mask: int | None = None) -> np.ndarray:
        return qsim_probs(self.h, qubit_mask)

    def amplitudes(self, offset: int = 0, count: int | None = None) -> np.ndarray:
        return qsim_get_amplitudes(self.h, offset, count)

    def set_amplitudes(self, values, offset: int = 0):
        qsim_set_amplitudes(self.h, values, offset)
        return self

    def synchronize(self):
        qsim_synchronize(self.h)
        return self

    def info(self) -> dict:
        return qsim_info(self.h)

    def touched_qubits(self) -> int:
        return qsim_touched_qubits(self.h)

    def profile(self, enable: bool = True):
        qsim_profile(self.h, enable)
        return self

    def stats(self) -> dict:
        return qsim_get_stats(self.h)


# ------------------------------------------------------ three-state model

def qsim3_lower(gates, num_ions: int) -> list:
    """Host-only: the transformations of the three-state model the gates
    lower to, as dicts."""
    g = _gates(gates)
    n = ctypes.c_size_t()
    L = lib()
    _check(L.qsim3_lower(g.ctypes.data, len(g), num_ions, None, 0, ctypes.byref(n)))
    out = (qsim3_pulse * max(1, n.value))()
    _check(L.qsim3_lower(g.ctypes.data, len(g), num_ions, out, n.value, ctypes.byref(n)))
    return [out[i].as_dict() for i in range(n.value)]


class State3:
    """Owning wrapper of one three-state register (3^M amplitudes)."""

    def __init__(self, num_ions: int, dtype: int = QSIM_C64, options: qsim_options | None = None):
        self.num_ions = num_ions
        self._opt = options
        h = ctypes.c_void_p()
        _check(lib().qsim3_create(num_ions, dtype, ctypes.byref(options) if options else None,
                                  ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h is not None:
            _check(lib().qsim3_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def reset(self, basis_index: int = 0):
        _check(lib().qsim3_reset(self.h, basis_index))
        return self

    def inject_errors(self, sigma=None, p_bitflip=0.0, p_phaseflip=0.0, seed=0, trial=0):
        if sigma is None:
            _check(lib().qsim3_inject_errors(self.h, None))
        else:
            em = _em(sigma, p_bitflip, p_phaseflip, seed, trial)
            _check(lib().qsim3_inject_errors(self.h, ctypes.byref(em)))
        return self

    def apply(self, gates):
        g = _gates(gates)
        _check(lib().qsim3_apply_circuit(self.h, g.ctypes.data, len(g)))
        return self

    def apply_pulses(self, pulses):
        arr = (qsim3_pulse * max(1, len(pulses)))()
        for i, p in enumerate(pulses):
            arr[i] = qsim3_pulse(int(p["kind"]), int(p["ion"]), int(p.get("a", 0)),
                                 int(p.get("b", 1)), int(p.get("cond_ion", -1)),
                                 int(p.get("cond_level", 0)), float(p.get("theta", 0.0)),
                                 float(p.get("phi", 0.0)))
        _check(lib().qsim3_apply_pulses(self.h, arr, len(pulses)))
        return self

    def overlap(self, other: "State3"):
        out = np.zeros(4)
        _check(lib().qsim3_overlap(self.h, other.h, _dp(out)))
        return complex(out[0], out[1]), float(out[2]), float(out[3])

    def fidelity(self, other: "State3") -> float:
        out = ctypes.c_double()
        _check(lib().qsim3_fidelity(self.h, other.h, ctypes.byref(out)))
        return out.value

    def probs(self, ion_mask: int) -> np.ndarray:
        out = np.zeros(3 ** bin(ion_mask).count("1"))
        _check(lib().qsim3_probs(self.h, ion_mask, _dp(out), len(out)))
        return out

    def amplitudes(self, offset: int = 0, count: int | None = None) -> np.ndarray:
        if count is None:
            count = 3 ** self.num_ions - offset
        out = np.zeros(2 * count)
        _check(lib().qsim3_get_amplitudes(self.h, offset, count, _dp(out)))
        return out[0::2] + 1j * out[1::2]

    def synchronize(self):
        _check(lib().qsim3_synchronize(self.h))
        return self

    def info(self) -> dict:
        M, dt, step = ctypes.c_int(), ctypes.c_int(), ctypes.c_uint64()
        nt, nl = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().qsim3_info(self.h, ctypes.byref(M), ctypes.byref(dt), ctypes.byref(step),
                                ctypes.byref(nt), ctypes.byref(nl)))
        return {"num_ions": M.value, "dtype": dt.value, "step": step.value,
                "transformations": nt.value, "launches": nl.value}
