"""The general f(A) = X^A mod N circuit (Sec. 2.2, EQ 1, Fig. 6), CPU only.

Pinned against arithmetic, not against the simulator: a classical reversible
run of its X / CNOT / Toffoli gates on every basis input (a bit vector, no
amplitudes) must give |A>|X^A mod N>|0..0>; then the FP64 oracle on a small
instance must give the same distribution, and after the quantum FFT on A the
period's peaks (Fig. 4)."""
import numpy as np
import pytest

import circuitgen as cg
import oracle


def classical(gates, k):
    x = k
    for g in gates:
        kind, t, c0, c1 = int(g["kind"]), int(g["target"]), int(g["ctrl0"]), int(g["ctrl1"])
        assert kind in (cg.X, cg.CNOT, cg.TOFFOLI)
        if (c0 < 0 or (x >> c0) & 1) and (c1 < 0 or (x >> c1) & 1):
            x ^= 1 << t
    return x


@pytest.mark.parametrize("base,N,a", [(7, 15, 4), (2, 15, 3), (11, 15, 2), (2, 21, 3), (4, 5, 3),
                                      (3, 7, 3)])
def test_every_basis_input_gives_the_power(base, N, a):
    gates, lay = cg.modexp_circuit(base, N, a)
    assert lay["num_qubits"] == a + 3 * (N - 1).bit_length() + 5
    body = gates[a:]  # the Hadamards on A come first
    assert np.all(gates["kind"][:a] == cg.H)
    for A in range(1 << a):
        assert classical(body, A) == A | (pow(base, A, N) << a), A


def test_oracle_distribution_and_period_after_qft():
    base, N, a = 4, 5, 2  # 4^A mod 5 = 1, 4, 1, 4: period two
    gates, lay = cg.modexp_circuit(base, N, a)
    M = lay["num_qubits"]
    psi = oracle.simulate(M, gates)
    p = oracle.probs(psi, M)
    want = np.zeros(1 << M)
    for A in range(1 << a):
        want[A | (pow(base, A, N) << a)] = 1.0 / (1 << a)
    assert np.max(np.abs(p - want)) < 1e-14
    oracle.run(psi, M, cg.qft_circuit(range(a)))
    pA = oracle.probs(psi, M, (1 << a) - 1)
    assert np.max(np.abs(pA - [0.5, 0.0, 0.5, 0.0])) < 1e-14


def test_rejects_non_coprime_and_bad_sizes():
    for args in [(5, 15, 2), (0, 7, 2), (3, 2, 2), (2, 9, 0)]:
        with pytest.raises(ValueError):
            cg.modexp_circuit(*args)
