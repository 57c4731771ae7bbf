"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: the paper's
printed values (fixtures under tests/golden/), textbook truth tables, closed
forms, numpy/scipy library routines (Philox4x64-10, the matrix exponential,
Kronecker products), invariants, and a brute-force dense 2^M x 2^M product.
"""
import math
import os

import numpy as np
import pytest
import scipy.stats

import circuitgen as cg
import oracle
from oracle import dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
H_EXACT = float.fromhex("0x1.6a09e667f3bcdp-1")  # sqrt(1/2), correctly rounded


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


# ------------------------------------------------------------------ Fig. 1

def test_fig1a_zero_state():
    rows = [r for r in _rows("fig1_qubit_vectors.txt") if r[0] == "a"]
    psi = oracle.init(1, 0)
    amps = oracle.as_complex(psi)
    p = oracle.probs(psi, 1)
    for _, idx, amp, prob in rows:
        assert amps[int(idx)] == float(amp)
        assert p[int(idx)] == float(prob)


def test_fig1b_superposition_from_h():
    rows = [r for r in _rows("fig1_qubit_vectors.txt") if r[0] == "b"]
    psi = oracle.simulate(1, cg.gates_from_list([(cg.H, 0)]))
    amps = oracle.as_complex(psi)
    p = oracle.probs(psi, 1)
    for _, idx, amp, prob in rows:
        assert amp == "1/sqrt(2)" and prob == "1/2"
        # amplitude is sqrt(1/2) rounded once; probability within 1 ulp of 1/2
        assert amps[int(idx)].real == H_EXACT and amps[int(idx)].imag == 0.0
        assert abs(p[int(idx)] - 0.5) <= math.ulp(0.5)
    # 1/sqrt(2) of Fig. 1(b): the correctly rounded square root of 1/2
    assert amps[0].real == math.sqrt(0.5)


# ------------------------------------------------------------ Table 1 / Fig. 2

def test_table1_cnot_truth_table_on_basis_states():
    # index = 2A + B: A (control) is qubit 1, B (target) is qubit 0
    g = cg.gates_from_list([(cg.CNOT, 0, 1)])
    for A, B, A2, B2 in (map(int, r) for r in _rows("table1_cnot_truth_table.txt")):
        psi = oracle.simulate(2, g, k=2 * A + B)
        out = oracle.as_complex(psi)
        want = np.zeros(4, complex)
        want[2 * A2 + B2] = 1.0
        assert np.array_equal(out, want)


def test_fig2_cnot_matrix_swaps_a2_a3():
    Mfig = np.array([[int(x) for x in r] for r in _rows("fig2_cnot_matrix.txt")], dtype=float)
    a = cg.random_state(2, 7)
    ref = Mfig @ oracle.as_complex(a)
    psi = a.copy()
    oracle.run(psi, 2, cg.gates_from_list([(cg.CNOT, 0, 1)]))
    out = oracle.as_complex(psi)
    assert np.array_equal(out, ref)
    assert out[2] == oracle.as_complex(a)[3] and out[3] == oracle.as_complex(a)[2]


# ----------------------------------------------- permutation gates, basis states

@pytest.mark.parametrize("M", [3, 5, 7])
def test_permutation_gates_on_every_basis_state(M):
    rng = np.random.default_rng(M)
    for _ in range(6):
        t, c0, c1 = (int(x) for x in rng.choice(M, 3, replace=False))
        cases = [
            ((cg.X, t), lambda k: k ^ (1 << t)),
            ((cg.CNOT, t, c0), lambda k: k ^ (((k >> c0) & 1) << t)),
            ((cg.TOFFOLI, t, c0, c1), lambda k: k ^ ((((k >> c0) & (k >> c1)) & 1) << t)),
        ]
        for gate, f in cases:
            g = cg.gates_from_list([gate])
            for k in range(1 << M):
                out = oracle.simulate(M, g, k=k)
                want = np.zeros(2 << M)
                want[2 * f(k)] = 1.0
                assert np.array_equal(out, want), (gate, k)


def test_swap_moves_bits_exactly_including_signed_zero():
    M = 4
    psi = cg.random_state(M, 3)
    psi[5] = -0.0
    ref = psi.copy()
    oracle.run(psi, M, cg.gates_from_list([(cg.CNOT, 2, 0)]))
    c = oracle.as_complex
    for i in range(1 << M):
        j = i ^ (1 << 2) if (i & 1) else i
        assert psi[2 * i].tobytes() == ref[2 * j].tobytes()
        assert psi[2 * i + 1].tobytes() == ref[2 * j + 1].tobytes()
    assert c(psi).shape == (1 << M,)


# ---------------------------------------------------------- gate matrices

def _expm_gate(kind, theta, eps):
    import scipy.linalg
    Xp = np.array([[0, 1], [1, 0]], complex)
    Zp = np.diag([1.0, -1.0]).astype(complex)
    if kind == cg.RZ:
        return scipy.linalg.expm(-0.5j * (theta + eps) * Zp)
    A = {cg.H: (Xp + Zp) / np.sqrt(2), cg.X: Xp, cg.CNOT: Xp, cg.TOFFOLI: Xp, cg.Z: Zp}[kind]
    return 1j * scipy.linalg.expm(-0.5j * (np.pi + eps) * A)


@pytest.mark.parametrize("kind", [cg.H, cg.RZ, cg.X, cg.CNOT, cg.TOFFOLI, cg.Z])
def test_gate_matrix_equals_rotation_exponential(kind):
    rng = np.random.default_rng(kind + 11)
    for eps in [0.0, 1e-3, -0.02, 0.7, float(rng.normal())]:
        theta = float(rng.uniform(0, 2 * np.pi)) if kind == cg.RZ else 0.0
        form, U = oracle.gate_matrix(kind, theta, eps)
        ref = _expm_gate(kind, theta, eps)
        assert np.max(np.abs(U - ref)) < 2e-15, (kind, eps)
        assert np.max(np.abs(U.conj().T @ U - np.eye(2))) < 1e-15


def test_unperturbed_gates_are_textbook():
    for kind, want, form_want in [
        (cg.H, np.array([[H_EXACT, H_EXACT], [H_EXACT, -H_EXACT]]), 0),
        (cg.X, np.array([[0, 1], [1, 0]]), 1),
        (cg.CNOT, np.array([[0, 1], [1, 0]]), 1),
        (cg.TOFFOLI, np.array([[0, 1], [1, 0]]), 1),
        (cg.Z, np.array([[1, 0], [0, -1]]), 2),
    ]:
        form, U = oracle.gate_matrix(kind, 0.0, 0.0)
        assert form == form_want
        assert np.array_equal(U, want.astype(complex))
    _, U = oracle.gate_matrix(cg.RZ, 0.3, 0.0)
    assert np.allclose(np.diag(U), [np.exp(-0.15j), np.exp(0.15j)], atol=1e-16, rtol=0)


# ------------------------------------------------------------ random draws

@pytest.mark.parametrize("key", [(0, 0), (1030, 7), (2**63 + 5, 2**40)])
def test_philox_matches_numpy(key):
    rng = np.random.default_rng(1)
    for _ in range(20):
        ctr = [int(x) for x in rng.integers(0, 2**63, size=4, dtype=np.int64)]
        ctr[3] = int(rng.integers(0, 3))
        words = list(ctr)
        for n in range(4):
            if words[n] > 0:
                words[n] -= 1
                break
            words[n] = 2**64 - 1
        want = np.random.Philox(key=np.array(key, dtype=np.uint64),
                                counter=np.array(words, dtype=np.uint64)).random_raw(4)
        assert np.array_equal(oracle.philox4x64_10(ctr, key), want)


def test_gaussian_draws_are_standard_normal():
    em = oracle.Errors(sigma=1.0, seed=1014, trial=3)
    z = np.array([oracle.gauss(em, s) for s in range(20000)])
    assert abs(z.mean()) < 5 / math.sqrt(len(z))
    assert abs(z.var() - 1.0) < 0.05
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3


def test_gaussian_draw_matches_dense_checker_recipe():
    em = oracle.Errors(sigma=0.01, seed=12, trial=1012)
    for s in range(50):
        assert abs(oracle.angle_error(em, s) - dense.angle_error(em, s)) <= 4e-18


def test_flip_frequencies_and_limits():
    em = oracle.Errors(p_bitflip=0.1, p_phaseflip=0.02, seed=5)
    ev = np.array([oracle.flip_events(em, s, q) for s in range(4000) for q in range(10)])
    n = len(ev)
    fb, fp = np.mean(ev & 1), np.mean((ev >> 1) & 1)
    assert abs(fb - 0.1) < 5 * math.sqrt(0.1 * 0.9 / n)
    assert abs(fp - 0.02) < 5 * math.sqrt(0.02 * 0.98 / n)
    # bit and phase flips of one qubit are independent
    both = np.mean(ev == 3)
    assert abs(both - 0.002) < 5 * math.sqrt(0.002 / n)
    never = oracle.Errors(p_bitflip=0.0, p_phaseflip=0.0, seed=5)
    always = oracle.Errors(p_bitflip=1.0, p_phaseflip=1.0, seed=5)
    for s in range(100):
        assert oracle.flip_events(never, s, s % 7) == 0
        assert oracle.flip_events(always, s, s % 7) == 3
    for s in range(200):
        for q in range(4):
            b, p = dense.flip_events(em, s, q)
            assert oracle.flip_events(em, s, q) == int(b) | (int(p) << 1)


# --------------------------------------------------- dense brute force, M <= 10

@pytest.mark.parametrize("M,G,seed", [(1, 30, 1), (2, 40, 2), (3, 60, 3), (5, 60, 5),
                                      (8, 40, 8), (10, 25, 10)])
def test_pair_loops_match_dense_matrices(M, G, seed):
    kinds = (cg.H, cg.RZ, cg.X, cg.Z) if M < 2 else \
        (cg.H, cg.RZ, cg.X, cg.Z, cg.CNOT) if M < 3 else \
        (cg.H, cg.RZ, cg.X, cg.Z, cg.CNOT, cg.TOFFOLI)
    gates = cg.random_circuit(M, G, seed, kinds=kinds)
    for em in [None,
               oracle.Errors(sigma=0.3, seed=seed, trial=1),
               oracle.Errors(sigma=0.05, p_bitflip=0.05, p_phaseflip=0.05, seed=seed, trial=2)]:
        got = oracle.as_complex(oracle.simulate(M, gates, em))
        want = dense.simulate(M, gates, em)
        assert np.max(np.abs(got - want)) < 1e-12, (M, em)


def test_dense_checker_controls_and_bit_order_small_case():
    # M=3, Toffoli(controls 0 and 2, target 1) swaps |101> <-> |111> only
    g = cg.gates_from_list([(cg.TOFFOLI, 1, 0, 2)])
    a = cg.random_state(3, 9)
    got = oracle.as_complex(oracle.run(a.copy(), 3, g))
    want = oracle.as_complex(a).copy()
    want[[5, 7]] = want[[7, 5]]
    assert np.array_equal(got, want)
    assert np.allclose(dense.full_matrix(3, dense.PAULI_X, 1, (0, 2)) @ oracle.as_complex(a), want)


# --------------------------------------------------------------- invariants

def test_norm_conserved():
    M = 12
    gates = cg.random_circuit(M, 200, 12)
    for em in [None, oracle.Errors(sigma=0.01, p_bitflip=1e-3, p_phaseflip=1e-3, seed=1012)]:
        psi = oracle.simulate(M, gates, em)
        assert abs(np.sum(psi * psi) - 1.0) < 1e-12


def _inverse(gates):
    inv = gates[::-1].copy()
    angled = (inv["kind"] == cg.RZ) | (inv["kind"] == cg.CPHASE)
    inv["theta"] = np.where(angled, -inv["theta"], inv["theta"])
    return inv


def test_gate_then_inverse_is_identity():
    M = 10
    gates = cg.random_circuit(M, 300, 4)
    psi = oracle.simulate(M, gates)
    oracle.run(psi, M, _inverse(gates))
    want = oracle.init(M, 0)
    assert np.max(np.abs(psi - want)) < 1e-12


@pytest.mark.parametrize("M", [2, 9, 16])
def test_ghz_exact(M):
    psi = oracle.simulate(M, cg.ghz_circuit(M))
    c = oracle.as_complex(psi)
    assert c[0] == H_EXACT and c[-1] == H_EXACT
    assert np.count_nonzero(c) == 2


def test_fidelity_self_and_orthogonal():
    a = cg.random_state(8, 1)
    assert abs(oracle.fidelity(a, a, 8) - 1.0) < 1e-15
    assert oracle.fidelity(oracle.init(8, 0), oracle.init(8, 1), 8) == 0.0
    # invariant to scaling and global phase
    b = cg.random_state(8, 2)
    cb = oracle.as_complex(b) * (0.5 * np.exp(0.7j))
    b2 = np.empty_like(b)
    b2[0::2], b2[1::2] = cb.real, cb.imag
    assert abs(oracle.fidelity(a, b, 8) - oracle.fidelity(a, b2, 8)) < 1e-15
    # against numpy's vdot
    ca, cb0 = oracle.as_complex(a), oracle.as_complex(b)
    ref = abs(np.vdot(ca, cb0)) ** 2 / (np.vdot(ca, ca).real * np.vdot(cb0, cb0).real)
    assert abs(oracle.fidelity(a, b, 8) - ref) < 1e-14


# ------------------------------------------------ closed forms of the error model

def test_rz_angle_error_on_plus_state():
    em = oracle.Errors(sigma=0.05, seed=77)
    g = cg.gates_from_list([(cg.H, 0), (cg.RZ, 0, -1, -1, 0.0)])
    ideal = oracle.simulate(1, g)
    for trial in range(20):
        em.trial = trial
        # only the Rz step (step 1) is perturbed here: arm the model from step 1
        psi = oracle.simulate(1, g[:1])
        oracle.run(psi, 1, g[1:], em, step0=1)
        eps = oracle.angle_error(em, 1)
        assert abs(oracle.fidelity(ideal, psi, 1) - math.cos(eps / 2) ** 2) < 1e-15


def test_perturbed_x_and_h_on_zero_state():
    for kind, closed in [(cg.X, lambda e: math.cos(e / 2) ** 2),
                         (cg.H, lambda e: math.cos(e / 2) ** 2 + 0.5 * math.sin(e / 2) ** 2)]:
        g = cg.gates_from_list([(kind, 0)])
        ideal = oracle.simulate(1, g)
        for trial in range(20):
            em = oracle.Errors(sigma=0.2, seed=3, trial=trial)
            psi = oracle.simulate(1, g, em)
            eps = oracle.angle_error(em, 0)
            assert eps != 0.0
            assert abs(oracle.fidelity(ideal, psi, 1) - closed(eps)) < 1e-15


def test_flip_closed_forms():
    plus = cg.gates_from_list([(cg.H, 0)])
    ident = cg.gates_from_list([(cg.RZ, 0, -1, -1, 0.0)])
    bit = oracle.Errors(p_bitflip=1.0, seed=1)
    phase = oracle.Errors(p_phaseflip=1.0, seed=1)
    f = oracle.fidelity
    # X on |+>: F = 1; Z on |+>: F = 0
    assert abs(f(oracle.simulate(1, plus), oracle.simulate(1, plus, bit), 1) - 1.0) < 1e-15
    assert f(oracle.simulate(1, plus), oracle.simulate(1, plus, phase), 1) < 1e-30
    # X on |0>: F = 0; Z on |0>: F = 1
    assert f(oracle.simulate(1, ident), oracle.simulate(1, ident, bit), 1) == 0.0
    assert f(oracle.simulate(1, ident), oracle.simulate(1, ident, phase), 1) == 1.0


def test_error_free_model_is_bit_identical():
    M = 9
    gates = cg.random_circuit(M, 150, 21)
    a = oracle.simulate(M, gates, None)
    b = oracle.simulate(M, gates, oracle.Errors(sigma=0.0, p_bitflip=0.0, p_phaseflip=0.0,
                                                seed=99, trial=5))
    assert a.tobytes() == b.tobytes()


def test_split_circuit_equals_whole():
    M = 8
    gates = cg.random_circuit(M, 120, 31)
    em = oracle.Errors(sigma=0.02, p_bitflip=0.01, p_phaseflip=0.01, seed=31, trial=4)
    whole = oracle.simulate(M, gates, em)
    part = oracle.simulate(M, gates[:50], em)
    oracle.run(part, M, gates[50:], em, step0=50)
    assert whole.tobytes() == part.tobytes()


def test_angle_only_drift_first_order():
    # E[1 - F] ~ G sigma^2 / 4 for small sigma (each gate loses ~ eps^2/4 on average)
    M, G, sigma = 6, 200, 0.02
    gates = cg.random_circuit(M, G, 8, kinds=(cg.H, cg.RZ, cg.CNOT, cg.TOFFOLI))
    F = oracle.run_trials(gates, M, oracle.Errors(sigma=sigma, seed=8), 200)
    infid = 1.0 - F.mean()
    assert 0.3 * G * sigma ** 2 / 4 < infid < 1.5 * G * sigma ** 2 / 4


def test_flip_free_fraction_binomial():
    M, G, p = 4, 50, 2e-3
    gates = cg.random_circuit(M, G, 2)
    em = oracle.Errors(p_bitflip=p, p_phaseflip=p, seed=2)
    n = 0
    T = 400
    for t in range(T):
        em.trial = t
        if all(oracle.flip_events(em, s, q) == 0 for s in range(G) for q in range(M)):
            n += 1
    pf = (1 - p) ** (2 * M * G)
    assert abs(n / T - pf) < 5 * math.sqrt(pf * (1 - pf) / T)


# ------------------------------------------------------------- probabilities

def test_probs_full_and_marginal():
    M = 7
    psi = oracle.simulate(M, cg.random_circuit(M, 80, 5))
    full = oracle.probs(psi, M)
    c = oracle.as_complex(psi)
    assert np.max(np.abs(full - np.abs(c) ** 2)) < 1e-16
    assert abs(full.sum() - 1.0) < 1e-13
    mask = 0b1010010
    marg = oracle.probs(psi, M, mask)
    idx = np.arange(1 << M)
    key = ((idx >> 1) & 1) | (((idx >> 4) & 1) << 1) | (((idx >> 6) & 1) << 2)
    ref = np.bincount(key, weights=np.abs(c) ** 2, minlength=8)
    assert np.max(np.abs(marg - ref)) < 1e-15


def test_ghz_marginals():
    M = 10
    psi = oracle.simulate(M, cg.ghz_circuit(M))
    for q in range(M):
        p = oracle.probs(psi, M, 1 << q)
        assert abs(p[0] - 0.5) <= 2 * math.ulp(0.5) and abs(p[1] - 0.5) <= 2 * math.ulp(0.5)


def test_run_trials_equals_single_runs():
    M = 5
    gates = cg.random_circuit(M, 40, 9)
    base = oracle.Errors(sigma=0.05, p_bitflip=0.01, p_phaseflip=0.01, seed=9, trial=100)
    F = oracle.run_trials(gates, M, base, 8)
    ideal = oracle.simulate(M, gates)
    for t in range(8):
        em = oracle.Errors(0.05, 0.01, 0.01, 9, 100 + t)
        assert F[t] == oracle.fidelity(ideal, oracle.simulate(M, gates, em), M)


def test_invalid_inputs_rejected():
    bad = [
        [(cg.CNOT, 0, 0)],          # control == target
        [(cg.H, 5)],                # target out of range
        [(cg.TOFFOLI, 0, 1, 1)],    # duplicate controls
        [(cg.CNOT, 0)],             # missing control
        [(cg.H, 0, 1)],             # H takes no control
    ]
    for items in bad:
        with pytest.raises(ValueError):
            oracle.simulate(3, cg.gates_from_list(items))
    with pytest.raises(ValueError):
        oracle.simulate(3, cg.gates_from_list([(cg.H, 0)]), oracle.Errors(p_bitflip=1.5))


@pytest.mark.parametrize("a_qubits", [4, 5])
def test_fig4_modexp_7_mod_15_has_period_four(a_qubits):
    """Sec. 2.2 / Fig. 4 / EQ 1: the f(A) circuit (repeated squaring, X = 7,
    N = 15) on A in uniform superposition leaves |A>|7^A mod 15> with
    probability 2^-a for every A, and f repeats with period four (L + 1 = 5
    bits of A as in Sec. 2.2.1, or 4)."""
    M = a_qubits + 4
    gates = cg.modexp15_circuit(a_qubits)
    assert set(int(k) for k in gates["kind"]) <= {cg.H, cg.X, cg.CNOT, cg.TOFFOLI}
    p = np.abs(oracle.as_complex(oracle.simulate(M, gates))) ** 2
    want = np.zeros(1 << M)
    for A in range(1 << a_qubits):
        want[A | (pow(7, A, 15) << a_qubits)] = 1.0 / (1 << a_qubits)
    assert np.max(np.abs(p - want)) < 1e-15
    f = [pow(7, A, 15) for A in range(1 << a_qubits)]
    assert f[:4] == [1, 7, 4, 13] and all(f[A] == f[A % 4] for A in range(len(f)))


# ------------------------------------------- controlled phase and quantum FFT

def test_cphase_matrix_is_phase_exponential():
    import scipy.linalg
    P1 = np.diag([0.0, 1.0]).astype(complex)
    for theta, eps in [(0.0, 0.0), (np.pi, 0.0), (np.pi / 8, 1e-3), (2.5, -0.3)]:
        form, U = oracle.gate_matrix(cg.CPHASE, theta, eps)
        assert form == 0
        assert np.max(np.abs(U - scipy.linalg.expm(1j * (theta + eps) * P1))) < 2e-15
        assert U[0, 0] == 1.0 and U[0, 1] == 0.0 and U[1, 0] == 0.0


@pytest.mark.parametrize("M", [2, 3, 5])
def test_cphase_on_every_basis_state(M):
    """CPHASE(theta) on (control c, target t) multiplies |k> by e^{i theta}
    exactly when bits c and t of k are both 1, and leaves every other basis
    state untouched; it is symmetric in c and t."""
    theta = 0.8125
    for c in range(M):
        for t in range(M):
            if c == t:
                continue
            g = cg.gates_from_list([(cg.CPHASE, t, c, -1, theta)])
            g_sw = cg.gates_from_list([(cg.CPHASE, c, t, -1, theta)])
            for k in range(1 << M):
                out = oracle.as_complex(oracle.simulate(M, g, k=k))
                out_sw = oracle.as_complex(oracle.simulate(M, g_sw, k=k))
                want = np.zeros(1 << M, complex)
                both = (k >> c) & 1 and (k >> t) & 1
                want[k] = complex(np.cos(theta), np.sin(theta)) if both else 1.0
                assert np.array_equal(out, want), (c, t, k)
                assert np.array_equal(out_sw, want), (c, t, k)


@pytest.mark.parametrize("M,seed", [(2, 21), (4, 22), (7, 23), (9, 24)])
def test_pair_loops_match_dense_matrices_with_cphase(M, seed):
    kinds = (cg.H, cg.RZ, cg.CNOT, cg.CPHASE) + ((cg.TOFFOLI,) if M >= 3 else ())
    gates = cg.random_circuit(M, 50, seed, kinds=kinds)
    assert np.any(gates["kind"] == cg.CPHASE)
    for em in [None, oracle.Errors(sigma=0.2, p_bitflip=0.03, p_phaseflip=0.03, seed=seed,
                                   trial=4)]:
        got = oracle.as_complex(oracle.simulate(M, gates, em))
        want = dense.simulate(M, gates, em)
        assert np.max(np.abs(got - want)) < 1e-12, (M, em)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6])
def test_qft_of_basis_states_closed_form(n):
    """Sec. 2.2's quantum FFT: |x> -> 2^(-n/2) sum_y e^(2 pi i x y / 2^n) |y>,
    which is sqrt(2^n) times numpy's inverse FFT of the unit vector e_x."""
    N = 1 << n
    gates = cg.qft_circuit(range(n))
    y = np.arange(N)
    for x in range(N):
        got = oracle.as_complex(oracle.simulate(n, gates, k=x))
        closed = np.exp(2j * np.pi * x * y / N) / np.sqrt(N)
        e = np.zeros(N)
        e[x] = 1.0
        assert np.max(np.abs(got - closed)) < 1e-14, x
        assert np.max(np.abs(got - np.sqrt(N) * np.fft.ifft(e))) < 1e-14, x


def test_qft_on_scattered_qubits_of_a_larger_register():
    """The QFT acts on the value spelled by the listed qubits only: on
    qubits (5, 1, 3) of M = 7, with the other qubits holding a basis value."""
    M, qs = 7, [5, 1, 3]
    gates = cg.qft_circuit(qs)
    for x in range(8):
        rest = 0b1000100  # qubits 2 and 6 set
        k = rest | sum(((x >> i) & 1) << q for i, q in enumerate(qs))
        got = oracle.as_complex(oracle.simulate(M, gates, k=k))
        want = np.zeros(1 << M, complex)
        for yv in range(8):
            idx = rest | sum(((yv >> i) & 1) << q for i, q in enumerate(qs))
            want[idx] = np.exp(2j * np.pi * x * yv / 8) / np.sqrt(8)
        assert np.max(np.abs(got - want)) < 1e-14, x


@pytest.mark.parametrize("a_qubits", [4, 5])
def test_fig4_period_four_after_qft(a_qubits):
    """Fig. 4 / Sec. 2.2: f(A) = 7^A mod 15 repeats every four values of A,
    so after the quantum FFT on A (2^a values, a multiple of four) all of
    A's probability sits on the multiples of 2^a / 4, a quarter on each."""
    M = a_qubits + 4
    gates = np.concatenate([cg.modexp15_circuit(a_qubits), cg.qft_circuit(range(a_qubits))])
    psi = oracle.simulate(M, gates)
    pA = oracle.probs(psi, M, (1 << a_qubits) - 1)
    want = np.zeros(1 << a_qubits)
    want[:: (1 << a_qubits) // 4] = 0.25
    assert np.max(np.abs(pA - want)) < 1e-14
    assert abs(np.sum(psi * psi) - 1.0) < 1e-13


def test_cphase_inverse_and_invalid_forms():
    M = 8
    gates = cg.random_circuit(M, 200, 31, kinds=(cg.H, cg.RZ, cg.CNOT, cg.CPHASE))
    psi = oracle.simulate(M, gates)
    oracle.run(psi, M, _inverse(gates))
    assert np.max(np.abs(psi - oracle.init(M, 0))) < 1e-12
    for items in ([(cg.CPHASE, 0)], [(cg.CPHASE, 1, 1)], [(cg.CPHASE, 0, 1, 2)]):
        with pytest.raises(ValueError):
            oracle.simulate(3, cg.gates_from_list(items))
