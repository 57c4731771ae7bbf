"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws inputs: random gate lists, the GHZ preparation list,
Poisson request traces. It holds none of the simulator's arithmetic (no gate
matrices, no error draws, no state updates), so both the FP64 oracle and the
GPU library can be fed from it without sharing any of the method.

The paper's own benchmark circuits (its Shor-factoring circuits, Table 2) are
not printed in the paper, so random circuits over the paper's gate set
(Section 2.0: one-, two- and three-bit controlled-NOTs plus rotation gates)
stand in for them.

Gate record layout (24 bytes, little endian), the interface both sides read:
    uint32 kind, int32 target, int32 ctrl0, int32 ctrl1, float64 theta
with ctrl = -1 when unused.  Qubit q is index bit 2**q of the state vector.
"""
from __future__ import annotations

import numpy as np

H, RZ, X, CNOT, TOFFOLI, Z, CPHASE = 0, 1, 2, 3, 4, 5, 6
KIND_NAMES = {H: "H", RZ: "RZ", X: "X", CNOT: "CNOT", TOFFOLI: "TOFFOLI", Z: "Z",
              CPHASE: "CPHASE"}
ARITY = {H: 1, RZ: 1, X: 1, CNOT: 2, TOFFOLI: 3, Z: 1, CPHASE: 2}
ANGLED = (RZ, CPHASE)  # kinds whose theta is an angle

GATE_DTYPE = np.dtype(
    [("kind", "<u4"), ("target", "<i4"), ("ctrl0", "<i4"), ("ctrl1", "<i4"), ("theta", "<f8")],
    align=False,
)
assert GATE_DTYPE.itemsize == 24


def gates_from_list(items) -> np.ndarray:
    """Build a gate array from tuples (kind, target, ctrl0=-1, ctrl1=-1, theta=0.0)."""
    out = np.zeros(len(items), dtype=GATE_DTYPE)
    for n, it in enumerate(items):
        it = list(it)
        kind, tgt = int(it[0]), int(it[1])
        c0 = int(it[2]) if len(it) > 2 else -1
        c1 = int(it[3]) if len(it) > 3 else -1
        theta = float(it[4]) if len(it) > 4 else 0.0
        out[n] = (kind, tgt, c0, c1, theta)
    return out


def random_circuit(num_qubits: int, num_gates: int, seed: int,
                   kinds=(H, RZ, CNOT, TOFFOLI), top_bias: float = 0.0,
                   top_count: int = 4) -> np.ndarray:
    """Uniform random circuit over ``kinds`` on distinct random qubits.

    Per gate: kind uniform over ``kinds``; qubits drawn without replacement,
    the last one is the target and the rest are controls; RZ and CPHASE
    angles uniform on [0, 2*pi).  With ``top_bias`` > 0 the target is, with
    that probability, uniform over the top ``top_count`` qubits, otherwise
    uniform over all qubits; controls are then uniform over the remaining
    qubits.
    """
    M = int(num_qubits)
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.zeros(num_gates, dtype=GATE_DTYPE)
    kinds = list(kinds)
    for g in range(num_gates):
        kind = kinds[int(rng.integers(len(kinds)))]
        ar = ARITY[kind]
        if ar > M:
            raise ValueError(f"{KIND_NAMES[kind]} needs {ar} qubits, register has {M}")
        if top_bias > 0.0:
            if rng.random() < top_bias:
                tgt = int(M - top_count + rng.integers(top_count))
            else:
                tgt = int(rng.integers(M))
            rest = [q for q in range(M) if q != tgt]
            ctrls = [int(c) for c in rng.choice(rest, ar - 1, replace=False)] if ar > 1 else []
        else:
            qs = [int(q) for q in rng.choice(M, ar, replace=False)]
            tgt, ctrls = qs[-1], qs[:-1]
        theta = float(rng.uniform(0.0, 2.0 * np.pi)) if kind in ANGLED else 0.0
        c0 = ctrls[0] if len(ctrls) > 0 else -1
        c1 = ctrls[1] if len(ctrls) > 1 else -1
        out[g] = (kind, tgt, c0, c1, theta)
    return out


def ghz_circuit(num_qubits: int) -> np.ndarray:
    """H on qubit 0, then CNOT(control q-1, target q) for q = 1..M-1."""
    items = [(H, 0)] + [(CNOT, q, q - 1) for q in range(1, num_qubits)]
    return gates_from_list(items)


def modexp15_circuit(a_qubits: int = 4, qubit_map=None) -> np.ndarray:
    """f(A) = 7^A mod 15 (Sec. 2.2, Fig. 4) on a register A of `a_qubits`
    qubits (0 .. a_qubits-1) in uniform superposition and a 4-qubit register
    y (qubits a_qubits .. a_qubits+3) prepared to 1, by repeated squaring
    (EQ 1): bit l of A multiplies y by 7^(2^l) mod 15, which is 7, 4, then 1.

    On 4-bit y in 1..14, multiplying by 2 mod 15 is a left rotation of the
    bits (2^4 = 16 = 1 mod 15), so 4 = a rotation by two places (two swaps),
    and 7 = -8 is a rotation by three places followed by the complement
    (15 - y = NOT y).  A controlled swap is CNOT, Toffoli, CNOT; a controlled
    complement is a CNOT per bit.  Gates: H, X, CNOT and Toffoli only.
    qubit_map[i], if given, is the register qubit that logical qubit i uses."""
    y = [a_qubits + i for i in range(4)]
    items = [(H, q) for q in range(a_qubits)] + [(X, y[0])]

    def cswap(c, p, q):
        items.extend([(CNOT, p, q), (TOFFOLI, q, c, p), (CNOT, p, q)])

    for l in range(a_qubits):
        factor = pow(7, 1 << l, 15)
        if factor == 7:  # rotate by three places (= right by one), then complement
            cswap(l, y[0], y[1])
            cswap(l, y[1], y[2])
            cswap(l, y[2], y[3])
            items.extend((CNOT, yi, l) for yi in y)
        elif factor == 4:  # rotate by two places
            cswap(l, y[0], y[2])
            cswap(l, y[1], y[3])
        # factor 1: nothing to do
    if qubit_map is not None:
        qm = [int(x) for x in qubit_map]
        if len(qm) != a_qubits + 4 or len(set(qm)) != len(qm):
            raise ValueError("qubit_map needs a_qubits + 4 distinct qubits")
        items = [(it[0],) + tuple(qm[x] for x in it[1:]) for it in items]
    return gates_from_list(items)


def qft_circuit(qubits, swaps: bool = True) -> np.ndarray:
    """Quantum Fourier transform (the quantum FFT of Sec. 2.2) on the listed
    qubits, qubits[0] the least significant bit of the register value x:
    |x> -> 2^(-n/2) sum_y e^(2 pi i x y / 2^n) |y>.

    Most significant bit first: H on it, then a controlled phase of
    pi / 2^(j-k) from each lower bit k; the result then holds y with its bits
    in reverse order, which the closing swaps (three CNOTs each) undo.  Gates:
    H, CPHASE and CNOT."""
    q = [int(x) for x in qubits]
    if len(set(q)) != len(q):
        raise ValueError("qft_circuit needs distinct qubits")
    n = len(q)
    items = []
    for j in range(n - 1, -1, -1):
        items.append((H, q[j]))
        for k in range(j - 1, -1, -1):
            items.append((CPHASE, q[j], q[k], -1, np.pi / float(1 << (j - k))))
    if swaps:
        for i in range(n // 2):
            a, b = q[i], q[n - 1 - i]
            items.extend([(CNOT, a, b), (CNOT, b, a), (CNOT, a, b)])
    return gates_from_list(items)


def modexp_circuit(base: int, modulus: int, a_qubits: int):
    """f(A) = base^A mod modulus for a general modulus (Sec. 2.2, EQ 1 and
    Fig. 6), from X, CNOT and Toffoli gates, with A (a_qubits qubits) put in
    uniform superposition by Hadamards first.  Returns (gates, layout).

    Repeated squaring (EQ 1): bit l of A multiplies the running product P
    (L = bits of modulus - 1, starts at 1) by m = base^(2^l) mod modulus.
    As in Fig. 6, a multiplication is a sequence of modulo additions, one
    per bit j of P, of the constant m 2^j mod modulus into a running sum S,
    each controlled by bit l of A and bit j of P (their AND is formed in one
    qubit by a Toffoli).  A modulo addition of a constant c < modulus into
    S < modulus (S has L + 1 bits, the top one taking the sign) is: add c,
    subtract the modulus, copy the sign into a flag, add the modulus back
    where the flag is set, subtract c, clear the flag from the sign of that
    result, add c again.  Additions of constants load the constant into a
    register B (one CNOT per set bit, from the control) and run a ripple-
    carry adder S += B built from MAJ / UMA blocks (Cuccaro et al., 2004)
    with one carry qubit; a subtraction is the adder run backwards.  Where
    bit l of A is 0 the multiplication copies P into S instead; P and S are
    then swapped, and S is cleared by running, backwards, the multiplication
    by the inverse of m.  On every basis input |A>|1>|0..0> the circuit
    leaves |A>|base^A mod modulus>|0..0>.

    Layout (qubits in order): A, P (L), S (L + 1), B (L + 1), the adder's
    carry qubit, the flag, the AND qubit: a_qubits + 3L + 5 qubits.  This is
    not the paper's own 4L + 4-qubit circuit (unpublished), but the same
    function by the same decomposition."""
    base, modulus, a_qubits = int(base), int(modulus), int(a_qubits)
    if modulus < 3 or not (0 < base < modulus) or np.gcd(base, modulus) != 1 or a_qubits < 1:
        raise ValueError("modexp_circuit needs 0 < base < modulus, gcd(base, modulus) = 1")
    L = (modulus - 1).bit_length()
    n = L + 1
    A = list(range(a_qubits))
    P = list(range(a_qubits, a_qubits + L))
    S = list(range(P[-1] + 1, P[-1] + 1 + n))
    B = list(range(S[-1] + 1, S[-1] + 1 + n))
    carry, flag, both = B[-1] + 1, B[-1] + 2, B[-1] + 3
    items = []

    def adder():  # S += B (mod 2^n)
        prev = [carry] + B[:-1]
        for i in range(n):  # MAJ(prev, S_i, B_i)
            items.extend([(CNOT, S[i], B[i]), (CNOT, prev[i], B[i]), (TOFFOLI, B[i], prev[i], S[i])])
        for i in reversed(range(n)):  # UMA(prev, S_i, B_i)
            items.extend([(TOFFOLI, B[i], prev[i], S[i]), (CNOT, prev[i], B[i]), (CNOT, S[i], prev[i])])

    def backwards(emit):
        start = len(items)
        emit()
        seg = items[start:]
        del items[start:]
        items.extend(reversed(seg))

    def load(value, ctrl):  # B ^= value, under ctrl (None: unconditional)
        for i in range(n):
            if (value >> i) & 1:
                items.append((CNOT, B[i], ctrl) if ctrl is not None else (X, B[i]))

    def add_const(value, ctrl, sign):
        load(value, ctrl)
        adder() if sign > 0 else backwards(adder)
        load(value, ctrl)

    def mod_add(c):  # S = S + c mod modulus, where `both` is set
        add_const(c, both, +1)
        add_const(modulus, None, -1)
        items.append((CNOT, flag, S[-1]))
        add_const(modulus, flag, +1)
        add_const(c, both, -1)
        items.extend([(X, S[-1]), (CNOT, flag, S[-1]), (X, S[-1])])
        add_const(c, both, +1)

    def multiply(m, a_bit):  # S = a_bit ? m P mod modulus : P   (S = 0 before)
        for j in range(L):
            items.append((TOFFOLI, both, a_bit, P[j]))
            mod_add((m << j) % modulus)
            items.append((TOFFOLI, both, a_bit, P[j]))
        items.append((X, a_bit))
        for j in range(L):
            items.append((TOFFOLI, S[j], a_bit, P[j]))
        items.append((X, a_bit))

    items.extend((H, q) for q in A)
    items.append((X, P[0]))
    for l in range(a_qubits):
        m = pow(base, 1 << l, modulus)
        multiply(m, A[l])
        for j in range(L):  # swap P and S
            items.extend([(CNOT, S[j], P[j]), (CNOT, P[j], S[j]), (CNOT, S[j], P[j])])
        minv = pow(m, -1, modulus)
        backwards(lambda: multiply(minv, A[l]))
    layout = {"A": A, "P": P, "S": S, "B": B, "carry": carry, "flag": flag, "and": both,
              "num_qubits": both + 1}
    return gates_from_list(items), layout


def save_gates(path, gates: np.ndarray) -> None:
    np.ascontiguousarray(gates, dtype=GATE_DTYPE).tofile(path)


def load_gates(path) -> np.ndarray:
    return np.fromfile(path, dtype=GATE_DTYPE)


def random_state(num_qubits: int, seed: int) -> np.ndarray:
    """Random complex vector (not normalised), interleaved as float64 pairs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(2 * (1 << num_qubits))


def poisson_trace(n_requests: int, rate_hz: float, seed: int,
                  m_range=(10, 28), g_range=(100, 2000),
                  sigmas=(1e-4, 1e-3, 1e-2)):
    """Poisson request stream: arrival time, register size, gate count, sigma.

    Returns a list of dicts with keys ``t`` (seconds from start), ``M``,
    ``G``, ``sigma``, ``circuit_seed`` and ``error_seed``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    reqs = []
    for r in range(n_requests):
        t += float(rng.exponential(1.0 / rate_hz)) if rate_hz > 0 else 0.0
        reqs.append({
            "t": t,
            "M": int(rng.integers(m_range[0], m_range[1] + 1)),
            "G": int(rng.integers(g_range[0], g_range[1] + 1)),
            "sigma": float(sigmas[int(rng.integers(len(sigmas)))]),
            "circuit_seed": int(seed) + r,
            "error_seed": int(seed) + 1000 + r,
        })
    return reqs
