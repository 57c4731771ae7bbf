"""Batched Monte Carlo trials (one persistent launch) against the oracle and
against the per-register path, through the C-ABI."""
import numpy as np
import pytest

import circuitgen as cg
import oracle
import paper_quant_ph_9804039_amd as q

pytestmark = pytest.mark.gpu


def _single(M, dtype, gates, sigma, p, seed, trial):
    with q.State(M, dtype, q.make_options(renorm_period=-1)) as ideal, \
            q.State(M, dtype, q.make_options(renorm_period=-1)) as noisy:
        ideal.apply(gates)
        noisy.inject_errors(sigma, p, p, seed=seed, trial=trial)
        noisy.apply(gates)
        return ideal.fidelity(noisy)


@pytest.mark.parametrize("dtype,tol", [(q.QSIM_C128, 1e-12), (q.QSIM_C64, 1e-6)])
def test_trials_match_oracle_with_many_flips(dtype, tol):
    M, G, T = 9, 120, 24
    gates = cg.random_circuit(M, G, 77, kinds=(cg.H, cg.RZ, cg.X, cg.Z, cg.CNOT, cg.TOFFOLI))
    em = oracle.Errors(sigma=0.05, p_bitflip=0.01, p_phaseflip=0.01, seed=91, trial=1000)
    want = oracle.run_trials(gates, M, em, T)
    got = q.qsim_run_trials(gates, M, dtype, em.sigma, em.p_bitflip, em.p_phaseflip, em.seed,
                            em.trial, T)
    assert np.max(np.abs(got - want)) < tol, np.max(np.abs(got - want))
    # the draws produced real flips in most trials (F far from the angle-only value)
    assert np.mean(want < 0.9) > 0.3


def test_trial_equals_per_register_path():
    M, G = 12, 200
    gates = cg.random_circuit(M, G, 12)
    got = q.qsim_run_trials(gates, M, q.QSIM_C128, 0.01, 2e-3, 2e-3, 5, 40, 6)
    for t in range(6):
        F = _single(M, q.QSIM_C128, gates, 0.01, 2e-3, 5, 40 + t)
        assert abs(got[t] - F) < 1e-12


def test_config3_shape_m14_c64_sample_against_oracle():
    """M=14, 500 gates, sigma=1e-3, p=1e-4 (complex64 state, FP64 reductions):
    the first 64 trials of a 4096-trial batch checked one by one against the
    FP64 oracle, every trial finite and in [0, 1]."""
    M, G, K = 14, 500, 64
    gates = cg.random_circuit(M, G, 14)
    em = oracle.Errors(sigma=1e-3, p_bitflip=1e-4, p_phaseflip=1e-4, seed=1014, trial=0)
    print("config3 M=14 c64 4096 trials, 64 against the oracle", flush=True)
    got = q.qsim_run_trials(gates, M, q.QSIM_C64, em.sigma, em.p_bitflip, em.p_phaseflip,
                            em.seed, 0, 4096)
    want = oracle.run_trials(gates, M, em, K)
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got[:K] - want)) < 1e-6
    assert np.all((got >= -1e-6) & (got <= 1 + 1e-6))
    # trials without any flip keep F close to 1 - O(G sigma^2)
    flip_free = [t for t in range(K)
                 if all(oracle.flip_events(oracle.Errors(1e-3, 1e-4, 1e-4, 1014, t), s, qb) == 0
                        for s in range(G) for qb in range(M))]
    assert flip_free
    for t in flip_free:
        assert got[t] > 0.99


def test_error_free_trials_have_unit_fidelity():
    M = 10
    gates = cg.random_circuit(M, 100, 3)
    F = q.qsim_run_trials(gates, M, q.QSIM_C64, 0.0, 0.0, 0.0, 1, 0, 300)
    assert np.max(np.abs(F - 1.0)) < 1e-6
    F = q.qsim_run_trials(gates, M, q.QSIM_C128, 0.0, 0.0, 0.0, 1, 0, 10)
    assert np.max(np.abs(F - 1.0)) < 1e-13


def test_trials_deterministic_and_small_registers():
    for M in (1, 2, 3, 5):
        kinds = (cg.H, cg.RZ, cg.X, cg.Z) + ((cg.CNOT,) if M >= 2 else ()) + \
            ((cg.TOFFOLI,) if M >= 3 else ())
        gates = cg.random_circuit(M, 50, M, kinds=kinds)
        em = oracle.Errors(sigma=0.1, p_bitflip=0.02, p_phaseflip=0.02, seed=M, trial=7)
        a = q.qsim_run_trials(gates, M, q.QSIM_C128, 0.1, 0.02, 0.02, M, 7, 20)
        b = q.qsim_run_trials(gates, M, q.QSIM_C128, 0.1, 0.02, 0.02, M, 7, 20)
        assert np.array_equal(a, b)
        want = oracle.run_trials(gates, M, em, 20)
        assert np.max(np.abs(a - want)) < 1e-12


def test_trials_reject_bad_input():
    g = cg.random_circuit(6, 10, 1)
    with pytest.raises(q.QsimError):
        q.qsim_run_trials(g, 15, q.QSIM_C64, 0.1, 0, 0, 0, 0, 4)
    with pytest.raises(q.QsimError):
        q.qsim_run_trials(g, 14, q.QSIM_C128, 0.1, 0, 0, 0, 0, 4)
    with pytest.raises(q.QsimError):
        q.qsim_run_trials(g, 6, q.QSIM_C64, -0.1, 0, 0, 0, 0, 4)
    with pytest.raises(q.QsimError):
        q.qsim_run_trials(cg.gates_from_list([(cg.CNOT, 1, 1)]), 6, q.QSIM_C64, 0.1, 0, 0, 0, 0, 4)
    assert len(q.qsim_run_trials(g, 6, q.QSIM_C64, 0.1, 0, 0, 0, 0, 0)) == 0


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("M", [11, 12])
@pytest.mark.parametrize("dtype,tol", [(q.QSIM_C128, 1e-12), (q.QSIM_C64, 1e-6)])
def test_every_kernel_variant_matches_oracle(monkeypatch, variant, M, dtype, tol):
    """Each variant the autotuner picks from (one LDS sweep per gate with 1024
    or 512 threads; the register in registers with 4 or 5 group qubits),
    forced in turn, against the oracle with dense flips and controls."""
    print(f"trials variant={variant} M={M} dtype={dtype}", flush=True)
    monkeypatch.setenv("QSIM_TRIAL_VARIANT", str(variant))
    gates = cg.random_circuit(M, 300, 40 + M,
                              kinds=(cg.H, cg.RZ, cg.X, cg.Z, cg.CNOT, cg.TOFFOLI))
    em = oracle.Errors(sigma=0.05, p_bitflip=0.004, p_phaseflip=0.004, seed=17 + M, trial=3)
    want = oracle.run_trials(gates, M, em, 12)
    got = q.qsim_run_trials(gates, M, dtype, em.sigma, em.p_bitflip, em.p_phaseflip, em.seed,
                            em.trial, 12)
    assert np.max(np.abs(got - want)) < tol, np.max(np.abs(got - want))
    assert np.mean(want < 0.9) > 0.3


def test_workspace_kept_between_calls_changes_no_result():
    """The per-device workspace (error-free register, buffers grown to the
    largest call) is reused across calls of different shapes and sizes: a
    call repeated after others gives the same fidelities bit for bit, and a
    larger batch starts with the smaller batch's trials."""
    ga = cg.random_circuit(12, 150, 3)
    gb = cg.random_circuit(13, 90, 4)
    print("workspace reuse: M=12 c64 / M=13 c128 / M=12 c64", flush=True)
    a1 = q.qsim_run_trials(ga, 12, q.QSIM_C64, 0.02, 1e-3, 1e-3, 8, 0, 48)
    b1 = q.qsim_run_trials(gb, 13, q.QSIM_C128, 0.02, 1e-3, 1e-3, 9, 0, 16)
    a2 = q.qsim_run_trials(ga, 12, q.QSIM_C64, 0.02, 1e-3, 1e-3, 8, 0, 48)
    assert np.array_equal(a1, a2)
    a3 = q.qsim_run_trials(ga, 12, q.QSIM_C64, 0.02, 1e-3, 1e-3, 8, 0, 1024)
    assert np.array_equal(a3[:48], a1)
    b2 = q.qsim_run_trials(gb, 13, q.QSIM_C128, 0.02, 1e-3, 1e-3, 9, 0, 16)
    assert np.array_equal(b1, b2)
    want = oracle.run_trials(gb, 13, oracle.Errors(0.02, 1e-3, 1e-3, 9, 0), 2)
    assert np.max(np.abs(b2[:2] - want)) < 1e-12


@pytest.mark.parametrize("variant", [2, 3])
@pytest.mark.parametrize("M,dtype,tol", [(14, q.QSIM_C64, 1e-6), (13, q.QSIM_C128, 1e-12)])
def test_register_group_variants_long_circuits(monkeypatch, variant, M, dtype, tol):
    """2000-gate circuits through the register-group variants (the ones the
    autotuner picks for config 3).  Regression: their butterfly form of the
    uncontrolled Hadamard once dropped its real scale, so the squared norm
    doubled with every H; a float32 emulation of this generator
    (random_circuit(14, 2000, 14)) overflowed at gate 1061, after 267 H, and
    complex128 overflowed near 2000 H.  The scale is now restored at the end
    of every register group, so the trials stay finite and match the
    oracle."""
    print(f"long trials variant={variant} M={M} dtype={dtype}", flush=True)
    monkeypatch.setenv("QSIM_TRIAL_VARIANT", str(variant))
    gates = cg.random_circuit(M, 2000, M)
    em = oracle.Errors(sigma=1e-3, p_bitflip=1e-4, p_phaseflip=1e-4, seed=2000 + M, trial=0)
    want = oracle.run_trials(gates, M, em, 16)
    got = q.qsim_run_trials(gates, M, dtype, em.sigma, em.p_bitflip, em.p_phaseflip, em.seed,
                            em.trial, 16)
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - want)) < tol, np.max(np.abs(got - want))


@pytest.mark.parametrize("variant", [2, 3])
@pytest.mark.parametrize("sigma", [0.05, 2.0])
@pytest.mark.parametrize("dtype,tol", [(q.QSIM_C64, 1e-6), (q.QSIM_C128, 1e-12)])
def test_register_group_variants_hadamard_heavy(monkeypatch, variant, sigma, dtype, tol):
    """Hadamard-only circuits (every gate a butterfly candidate, so groups are
    cut by the 32-butterfly bound alone) and, at sigma = 2, angle errors large
    enough that many Hadamards keep their full coefficients instead (|t| > 1)."""
    M = 11
    print(f"H-heavy trials variant={variant} sigma={sigma} dtype={dtype}", flush=True)
    monkeypatch.setenv("QSIM_TRIAL_VARIANT", str(variant))
    gates = cg.random_circuit(M, 600, 611, kinds=(cg.H,))
    em = oracle.Errors(sigma=sigma, p_bitflip=1e-3, p_phaseflip=1e-3, seed=611, trial=5)
    want = oracle.run_trials(gates, M, em, 16)
    got = q.qsim_run_trials(gates, M, dtype, em.sigma, em.p_bitflip, em.p_phaseflip, em.seed,
                            em.trial, 16)
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - want)) < tol, np.max(np.abs(got - want))
