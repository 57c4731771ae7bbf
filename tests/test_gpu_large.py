"""The paper's larger workloads at full size, through the C-ABI.

* M = 26, 1000 gates, sigma = 1e-3, p = 1e-4 (complex64 and complex128): the
  whole state and the fidelity against the FP64 oracle run in full.
* M = 33 complex64 and M = 32 complex128 (64 GiB registers), 500 gates with
  half of the targets on the top four qubits: too large for the oracle, so
  checked through properties that hold at any size -- the GHZ state, the echo
  of a circuit followed by its inverse (Sec. 1.0: the accumulated error is
  the overlap with the error-free run), and complex64 against complex128.
"""
import numpy as np
import pytest

import circuitgen as cg
import oracle
import paper_quant_ph_9804039_amd as q

pytestmark = pytest.mark.gpu

GiB = 1 << 30


def _say(msg):
    print(msg, flush=True)


def _free_hbm():
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    free, total = ctypes.c_size_t(), ctypes.c_size_t()
    assert hip.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    return free.value


def _need(nbytes):
    if _free_hbm() < nbytes + 4 * GiB:
        pytest.skip(f"needs {nbytes / GiB:.0f} GiB of free device memory")


# ------------------------------------------------------------ M = 26 vs oracle

@pytest.fixture(scope="module")
def m26_reference():
    M = 26
    gates = cg.random_circuit(M, 1000, 26)
    em = oracle.Errors(sigma=1e-3, p_bitflip=1e-4, p_phaseflip=1e-4, seed=1026, trial=0)
    _say("oracle: M=26, 1000 gates, error-free and noisy")
    ideal = oracle.simulate(M, gates)
    noisy = oracle.simulate(M, gates, em)
    F_ref = oracle.fidelity(ideal, noisy, M)
    return M, gates, em, oracle.as_complex(ideal), oracle.as_complex(noisy), F_ref


@pytest.mark.parametrize("dtype,tol_amp,tol_f", [(q.QSIM_C128, 1e-12, 1e-12),
                                                 (q.QSIM_C64, 2e-5, 1e-6)])
def test_config2_m26_state_and_fidelity_vs_oracle(m26_reference, dtype, tol_amp, tol_f):
    M, gates, em, ideal_ref, noisy_ref, F_ref = m26_reference
    _say(f"config2 M=26 dtype={dtype}")
    with q.State(M, dtype) as ideal, q.State(M, dtype) as noisy:
        ideal.apply(gates)
        noisy.inject_errors(em.sigma, em.p_bitflip, em.p_phaseflip, em.seed, em.trial)
        noisy.apply(gates)
        F = ideal.fidelity(noisy)
        assert abs(F - F_ref) <= tol_f, (F, F_ref)
        for st, ref in ((ideal, ideal_ref), (noisy, noisy_ref)):
            # raw amplitudes (no normalisation on this side): a global
            # scale error fails here
            a = st.amplitudes()
            assert np.all(np.isfinite(a))
            assert np.max(np.abs(a - ref)) <= tol_amp
            assert abs(np.vdot(a, a).real - np.vdot(ref, ref).real) <= 10 * tol_amp


# ------------------------------------------------- 64 GiB registers, invariants

LARGE = [(33, q.QSIM_C64, 1e-6), (32, q.QSIM_C128, 1e-13)]


@pytest.mark.parametrize("M,dtype,tol", LARGE)
def test_config5_ghz_at_full_size(M, dtype, tol):
    _need(64 * GiB)
    _say(f"config5 GHZ M={M} dtype={dtype}")
    with q.State(M, dtype) as s:
        s.apply(cg.ghz_circuit(M))
        h = np.sqrt(0.5)
        assert abs(s.amplitudes(0, 1)[0] - h) < tol
        assert abs(s.amplitudes((1 << M) - 1, 1)[0] - h) < tol
        rng = np.random.default_rng(M)
        for k in rng.integers(1, (1 << M) - 1, size=32):
            assert s.amplitudes(int(k), 1)[0] == 0.0
        mask = 1 | (1 << (M // 2)) | (1 << (M - 1))
        p = s.probs(mask)
        want = np.zeros(8)
        want[0] = want[7] = 0.5
        assert np.max(np.abs(p - want)) < 10 * tol
        assert abs(s.norm() - 1.0) < 10 * tol


@pytest.mark.parametrize("M,dtype,tol", LARGE)
def test_config5_echo_equals_two_register_fidelity(M, dtype, tol):
    """Trial run then the error-free circuit's inverse leaves |<0|psi>|^2 = F,
    the fidelity of the two-register method; the error-free run echoes to
    |0...0> exactly up to rounding."""
    _need(2 * 64 * GiB)
    gates = cg.random_circuit(M, 500, M, top_bias=0.5)
    em = oracle.Errors(sigma=1e-3, seed=1000 + M, trial=0)
    _say(f"config5 echo M={M} dtype={dtype}")
    with q.State(M, dtype) as ideal, q.State(M, dtype) as noisy:
        ideal.apply(gates)
        noisy.inject_errors(em.sigma, 0.0, 0.0, em.seed, em.trial)
        noisy.apply(gates)
        F = ideal.fidelity(noisy)
        # first-order drift of the angle errors: E[1 - F] ~ G sigma^2 / 4
        assert 0.9990 < F < 1.0
        noisy.apply_inverse(gates)
        ideal.apply_inverse(gates)
        a0 = noisy.amplitudes(0, 1)[0]
        echo = abs(a0) ** 2 / noisy.norm()
        assert abs(echo - F) < (1e-5 if dtype == q.QSIM_C64 else 1e-12), (echo, F)
        b0 = ideal.amplitudes(0, 1)[0]
        assert abs(abs(b0) ** 2 / ideal.norm() - 1.0) < (1e-5 if dtype == q.QSIM_C64 else 1e-12)


def test_config5_complex64_against_complex128_m33():
    """The error of the complex64 register at M = 33, measured against the
    complex128 register on the same device (64 + 128 GiB)."""
    M = 33
    _need(192 * GiB)
    gates = cg.random_circuit(M, 500, M, top_bias=0.5)
    _say("config5 c64 vs c128 M=33")
    with q.State(M, q.QSIM_C64) as a, q.State(M, q.QSIM_C128) as b:
        for s in (a, b):
            s.inject_errors(1e-3, 0.0, 0.0, seed=1033, trial=0)
            s.apply(gates)
        F = a.fidelity(b)
        assert 1.0 - F < 1e-6, F
        assert abs(a.norm() - 1.0) < 1e-5 and abs(b.norm() - 1.0) < 1e-12
