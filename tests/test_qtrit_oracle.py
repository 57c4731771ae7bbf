"""Pins of the three-state (detailed Cirac-Zoller) oracle, CPU only.

Each ion has its two QU-bit levels plus a temporary third one (Sec. 2.0),
M ions take 3^M states and one transformation is 3^(M-1) independent
operations (Sec. 3.1).  Pinned against: the transformation's generator
(scipy expm), dense 3^M x 3^M products for small M, the CNOT truth table
(Table 1) reproduced by its five transformations, Fig. 1(b), the two-state
oracle (every error-free circuit agrees with it up to a global phase, with
nothing left in the temporary levels), closed forms of single angle errors,
and norm conservation."""
import numpy as np
import pytest
import scipy.linalg

import circuitgen as cg
import oracle
from oracle import dense

KINDS = (cg.H, cg.RZ, cg.X, cg.Z, cg.CNOT, cg.TOFFOLI, cg.CPHASE)


def binary_indices(M):
    return np.array([sum(((i >> q) & 1) * 3 ** q for q in range(M)) for i in range(1 << M)])


@pytest.mark.parametrize("a,b", [(0, 1), (0, 2), (1, 2)])
def test_pulse_matrix_is_the_generator_exponential(a, b):
    rng = np.random.default_rng(a + 3 * b)
    for _ in range(5):
        th, ph, eps = rng.uniform(-7, 7), rng.uniform(-4, 4), rng.normal() * 0.1
        p = {"kind": oracle.PULSE_ROT, "ion": 0, "a": a, "b": b, "theta": th, "phi": ph}
        Gm = np.zeros((2, 2), complex)
        Gm[0, 1], Gm[1, 0] = np.exp(1j * ph), np.exp(-1j * ph)
        want = scipy.linalg.expm(-0.5j * (th + eps) * Gm)
        assert np.max(np.abs(oracle.pulse_matrix3(p, eps) - want)) < 2e-15
    ph = {"kind": oracle.PULSE_PHASE, "ion": 0, "theta": 0.7}
    assert np.allclose(oracle.pulse_matrix3(ph), np.diag(np.exp([-0.35j, 0.35j])), atol=1e-16)


@pytest.mark.parametrize("M,seed", [(1, 1), (2, 2), (3, 3), (4, 4)])
def test_pulses_match_dense_products(M, seed):
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal(2 * 3 ** M)
    want = oracle.as_complex(psi).copy()
    for _ in range(30):
        a, b = sorted(rng.choice(3, 2, replace=False).tolist())
        ion = int(rng.integers(M))
        p = {"kind": int(rng.integers(2)), "ion": ion, "a": a, "b": b,
             "theta": rng.uniform(0, 7), "phi": rng.uniform(-3, 3), "cond_ion": -1}
        if M > 1 and rng.random() < 0.5:
            p["cond_ion"] = int(rng.choice([q for q in range(M) if q != ion]))
            p["cond_level"] = int(rng.integers(3))
        eps = rng.normal() * 0.05
        oracle.apply_pulse3(psi, M, p, eps)
        want = dense.pulse_matrix3_dense(M, p, eps) @ want
    assert np.max(np.abs(oracle.as_complex(psi) - want)) < 1e-13


def test_five_transformation_cnot_reproduces_table1():
    """Table 1 / Fig. 2 in the detailed model: on the four basis states of
    the QU-bit levels the CNOT's five transformations give exactly |c, t xor
    c>, amplitude 1 within rounding, nothing in the temporary levels."""
    for c, t in [(1, 0), (0, 1), (2, 0), (0, 2)]:
        M = 3
        for bc in (0, 1):
            for bt in (0, 1):
                k = bc * 3 ** c + bt * 3 ** t
                a = oracle.as_complex(oracle.simulate3(M, cg.gates_from_list([(cg.CNOT, t, c)]),
                                                       k=k))
                want = bc * 3 ** c + (bt ^ bc) * 3 ** t
                assert abs(a[want] - 1.0) < 1e-15
                assert np.sum(np.abs(np.delete(a, want)) ** 2) < 1e-30
    assert len(oracle.lower3(cg.gates_from_list([(cg.CNOT, 0, 1)])[0])) == 5


def test_fig1b_hadamard_in_the_detailed_model():
    a = oracle.as_complex(oracle.simulate3(1, cg.gates_from_list([(cg.H, 0)])))
    assert np.max(np.abs(np.abs(a[:2]) ** 2 - 0.5)) < 1e-15 and a[2] == 0.0


@pytest.mark.parametrize("M,seed", [(3, 5), (5, 6), (7, 7)])
def test_error_free_runs_equal_the_two_state_model(M, seed):
    g = cg.random_circuit(M, 120, seed, kinds=KINDS)
    p3 = oracle.as_complex(oracle.simulate3(M, g))
    p2 = oracle.as_complex(oracle.simulate(M, g))
    r = p3[binary_indices(M)]
    assert 1.0 - abs(np.vdot(p2, r)) ** 2 < 1e-12
    assert 1.0 - np.sum(np.abs(r) ** 2) < 1e-12  # no population left in level 2


def test_single_angle_errors_closed_forms():
    e = 0.03
    # X = rot(01, pi): with pi + eps the |1> population is cos^2(eps/2)
    psi = oracle.init3(1, 0)
    oracle.apply_pulse3(psi, 1, {"kind": 0, "ion": 0, "a": 0, "b": 1, "theta": np.pi}, e)
    assert abs(np.abs(oracle.as_complex(psi)[1]) ** 2 - np.cos(e / 2) ** 2) < 1e-15
    # the CNOT's conditional 2 pi rotation with 2 pi + eps on |1>_c |1>_t:
    # the first transformation turns the target into (|0> + |1>)/sqrt(2), the
    # faulty rotation moves sin^2(eps/2) of the |1> half into the temporary
    # level, and the last transformation leaves that level alone: 1/2 sin^2
    M, c, t = 2, 1, 0
    psi = oracle.init3(M, 1 * 3 ** c + 1 * 3 ** t)
    pulses = oracle.lower3(cg.gates_from_list([(cg.CNOT, t, c)])[0])
    for j, p in enumerate(pulses):
        oracle.apply_pulse3(psi, M, p, e if j == 2 else 0.0)
    pr = oracle.probs3(psi, M, 1 << t)
    assert abs(pr[2] - 0.5 * np.sin(e / 2) ** 2) < 1e-15


def test_norm_conserved_with_errors_and_flips_and_marginals():
    M = 6
    g = cg.random_circuit(M, 200, 66, kinds=KINDS)
    em = oracle.Errors(sigma=0.05, p_bitflip=0.01, p_phaseflip=0.01, seed=6, trial=6)
    psi = oracle.simulate3(M, g, em)
    assert abs(np.sum(psi * psi) - 1.0) < 1e-12
    full = oracle.probs3(psi, M)
    assert np.allclose(full, psi[0::2] ** 2 + psi[1::2] ** 2, atol=0, rtol=1e-15)
    m = oracle.probs3(psi, M, 0b100101)
    assert abs(m.sum() - 1.0) < 1e-12 and len(m) == 27
    leak = 1.0 - full[binary_indices(M)].sum()
    assert 0.0 < leak < 0.5  # angle errors leave population in the temporary levels


def test_flips_exchange_levels_exactly():
    M = 2
    rng = np.random.default_rng(9)
    v = rng.standard_normal(2 * 9)
    em = oracle.Errors(sigma=0.0, p_bitflip=1.0, p_phaseflip=0.0, seed=1, trial=1)
    got = oracle.as_complex(oracle.run3(v.copy(), M, cg.gates_from_list([(cg.RZ, 0, -1, -1, 0.0)]),
                                         em))
    x = oracle.as_complex(v).reshape(3, 3)  # [level of ion 1, level of ion 0]
    # Rz(0) is the identity; then both ions' levels 0 and 1 exchange
    perm = [1, 0, 2]
    want = x[np.ix_(perm, perm)].ravel()
    assert np.array_equal(got, want)
