"""Brute-force dense checker for small registers (M <= 10).

TEST INFRASTRUCTURE ONLY.  It follows Sec. 1.3 of the paper literally: every
transformation is a 2^M x 2^M matrix multiplied into the 2^M state vector.
The full matrix of a gate is assembled from Kronecker products (qubit q is
index bit 2^q, so the leftmost factor is qubit M-1) with a projector onto
"all controls set":  U_full = (I - P) + P K,  K = I x .. x U_t x .. x I.

It deliberately shares nothing with the pair-loop oracle in qsim_oracle.c:
the perturbed one-qubit gates are built here with scipy's matrix exponential,
i * expm(-i (pi + eps)/2 A) for a gate whose own rotation axis is A
(A = H, X or Z), expm(-i (theta + eps)/2 Z) for Rz and expm(i (theta + eps)
|1><1|) for the controlled phase; the random draws come
from numpy's own Philox4x64-10 generator.  The draw recipe (key = (seed,
trial), counter = (step, qubit, stream, 0), Box-Muller on the high halves of
words 0 and 1 for the angle, high halves below floor(p 2^32) for the flips)
is the same specification the oracle implements, written out again here.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from circuitgen import CNOT, CPHASE, H, RZ, TOFFOLI, X, Z

I2 = np.eye(2, dtype=complex)
PAULI_X = np.array([[0, 1], [1, 0]], dtype=complex)
PAULI_Z = np.array([[1, 0], [0, -1]], dtype=complex)
HADAMARD = (PAULI_X + PAULI_Z) / np.sqrt(2.0)
PROJ1 = np.array([[0, 0], [0, 1]], dtype=complex)


def one_qubit_matrix(kind: int, theta: float, eps: float) -> np.ndarray:
    if kind == RZ:
        return scipy.linalg.expm(-0.5j * (theta + eps) * PAULI_Z)
    if kind == CPHASE:  # e^{i phi} on |1> of the target (the control is a projector)
        return scipy.linalg.expm(1j * (theta + eps) * PROJ1)
    axis = {H: HADAMARD, X: PAULI_X, CNOT: PAULI_X, TOFFOLI: PAULI_X, Z: PAULI_Z}[kind]
    if eps == 0.0:
        return axis.copy()
    return 1j * scipy.linalg.expm(-0.5j * (np.pi + eps) * axis)


def _kron_all(factors):
    out = np.ones((1, 1), dtype=complex)
    for f in factors:
        out = np.kron(out, f)
    return out


def full_matrix(M: int, U2: np.ndarray, target: int, controls=()) -> np.ndarray:
    K = _kron_all([U2 if q == target else I2 for q in reversed(range(M))])
    if not controls:
        return K
    P = _kron_all([PROJ1 if q in controls else I2 for q in reversed(range(M))])
    return (np.eye(1 << M, dtype=complex) - P) + P @ K


def _block(seed: int, trial: int, step: int, qubit: int, stream: int) -> np.ndarray:
    # numpy's Philox advances its 256-bit counter before each block, so start
    # one below the wanted counter.
    words = [step, qubit, stream, 0]
    for n in range(4):
        if words[n] > 0:
            words[n] -= 1
            break
        words[n] = (1 << 64) - 1
    bg = np.random.Philox(key=np.array([seed, trial], dtype=np.uint64),
                          counter=np.array(words, dtype=np.uint64))
    return bg.random_raw(4)


def angle_error(errors, step: int) -> float:
    if errors is None or errors.sigma == 0.0:
        return 0.0
    w = _block(errors.seed, errors.trial, step, 0, 1)
    u1 = (float(int(w[0]) >> 32) + 0.5) * 2.0 ** -32
    u2 = (float(int(w[1]) >> 32) + 0.5) * 2.0 ** -32
    return errors.sigma * np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def flip_events(errors, step: int, qubit: int):
    if errors is None or (errors.p_bitflip == 0.0 and errors.p_phaseflip == 0.0):
        return False, False
    w = _block(errors.seed, errors.trial, step, qubit, 2)
    thr_b = int(np.floor(errors.p_bitflip * 2.0 ** 32))
    thr_p = int(np.floor(errors.p_phaseflip * 2.0 ** 32))
    return (int(w[0]) >> 32) < thr_b, (int(w[1]) >> 32) < thr_p


def simulate(M: int, gates, errors=None, k: int = 0, step0: int = 0) -> np.ndarray:
    """Complex state vector after the circuit, by dense matrix products."""
    if M > 10:
        raise ValueError("dense checker is limited to M <= 10")
    psi = np.zeros(1 << M, dtype=complex)
    psi[k] = 1.0
    for n, g in enumerate(gates):
        step = step0 + n
        kind, tgt = int(g["kind"]), int(g["target"])
        ctrls = tuple(int(c) for c in (g["ctrl0"], g["ctrl1"]) if int(c) >= 0)
        eps = angle_error(errors, step)
        psi = full_matrix(M, one_qubit_matrix(kind, float(g["theta"]), eps), tgt, ctrls) @ psi
        for q in range(M):
            bit, phase = flip_events(errors, step, q)
            if bit:
                psi = full_matrix(M, PAULI_X, q) @ psi
            if phase:
                psi = full_matrix(M, PAULI_Z, q) @ psi
    return psi


# ------------------------------------------------------- three-state model

def pulse_matrix3_dense(M: int, pulse, eps: float = 0.0) -> np.ndarray:
    """3^M x 3^M matrix of one transformation of the three-state model, built
    from its generator: expm(-i (theta+eps)/2 (e^{i phi}|a><b| + h.c.)) on
    the ion's three levels (a phase transformation: expm(-i (theta+eps)/2
    (|a><a| - |b><b|))), Kronecker products over the ions (ion q has place
    value 3^q, so the leftmost factor is ion M-1), and a projector onto the
    condition ion's level when the transformation is conditional."""
    th = float(pulse["theta"]) + eps
    Gm = np.zeros((3, 3), dtype=complex)
    a, b = int(pulse.get("a", 0)), int(pulse.get("b", 1))
    if int(pulse["kind"]) == 1:
        Gm[a, a], Gm[b, b] = 1.0, -1.0
    else:
        ph = float(pulse["phi"])
        Gm[a, b] = np.exp(1j * ph)
        Gm[b, a] = np.exp(-1j * ph)
    U3 = scipy.linalg.expm(-0.5j * th * Gm)
    I3 = np.eye(3, dtype=complex)
    ion = int(pulse["ion"])
    K = _kron_all([U3 if q == ion else I3 for q in reversed(range(M))])
    ci = int(pulse.get("cond_ion", -1))
    if ci < 0:
        return K
    Pv = np.zeros((3, 3), dtype=complex)
    Pv[int(pulse["cond_level"]), int(pulse["cond_level"])] = 1.0
    P = _kron_all([Pv if q == ci else I3 for q in reversed(range(M))])
    return (np.eye(3 ** M, dtype=complex) - P) + P @ K
