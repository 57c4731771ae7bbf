"""Edge cases of the C-ABI on the GPU: empty circuits, the one-qubit
register with every gate kind and errors, ragged amplitude windows, empty
Monte Carlo circuits, and the largest register the library takes."""
import numpy as np
import pytest

import circuitgen as cg
import oracle
import paper_quant_ph_9804039_amd as q

pytestmark = pytest.mark.gpu

GiB = 1 << 30


@pytest.mark.parametrize("dtype", [q.QSIM_C64, q.QSIM_C128])
@pytest.mark.parametrize("M", [1, 9, 13])
def test_empty_circuit_changes_nothing(dtype, M):
    print(f"empty circuit M={M} dtype={dtype}", flush=True)
    with q.State(M, dtype) as a, q.State(M, dtype) as b:
        a.apply(cg.random_circuit(M, 20, M, kinds=(cg.H, cg.RZ, cg.X)))
        before = a.amplitudes()
        step = a.info()["step"]
        a.inject_errors(0.1, 0.1, 0.1, seed=1, trial=0)
        a.apply(cg.gates_from_list([]))
        assert np.array_equal(a.amplitudes(), before) and a.info()["step"] == step
        b.apply(cg.gates_from_list([]))
        assert b.amplitudes()[0] == 1.0 and b.fidelity(b) == 1.0


@pytest.mark.parametrize("dtype,tol", [(q.QSIM_C128, 1e-13), (q.QSIM_C64, 1e-6)])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_one_qubit_register_every_kind_with_errors(dtype, tol, mode):
    print(f"one qubit dtype={dtype} mode={mode}", flush=True)
    gates = cg.random_circuit(1, 200, 5, kinds=(cg.H, cg.RZ, cg.X, cg.Z))
    em = oracle.Errors(sigma=0.1, p_bitflip=0.05, p_phaseflip=0.05, seed=9, trial=2)
    want = oracle.as_complex(oracle.simulate(1, gates, em))
    with q.State(1, dtype, q.make_options(exec_mode=mode, renorm_period=-1)) as s:
        s.inject_errors(em.sigma, em.p_bitflip, em.p_phaseflip, em.seed, em.trial)
        s.apply(gates)
        assert np.max(np.abs(s.amplitudes() - want)) < tol


@pytest.mark.parametrize("dtype", [q.QSIM_C64, q.QSIM_C128])
def test_ragged_amplitude_windows(dtype):
    M = 11
    print(f"amplitude windows dtype={dtype}", flush=True)
    r = cg.random_state(M, 21)  # interleaved re/im
    if dtype == q.QSIM_C64:
        r = r.astype(np.float32).astype(np.float64)
    v = r[0::2] + 1j * r[1::2]
    with q.State(M, dtype) as s:
        s.set_amplitudes(v)
        for off, cnt in [(0, 1), (3, 5), (1023, 3), ((1 << M) - 7, 7), ((1 << M) - 1, 1)]:
            assert np.array_equal(s.amplitudes(off, cnt), v[off: off + cnt])
        patch = np.arange(1, 6) * (0.25 + 0.5j)
        s.set_amplitudes(patch, offset=37)
        w = v.copy()
        w[37:42] = patch
        assert np.array_equal(s.amplitudes(), w)
        for off, cnt in [(1 << M, 1), ((1 << M) - 2, 3)]:
            with pytest.raises(q.QsimError) as e:
                s.amplitudes(off, cnt)
            assert e.value.code == q.QSIM_ERANGE


def test_trials_of_an_empty_circuit_are_perfect():
    print("trials of an empty circuit", flush=True)
    F = q.qsim_run_trials(cg.gates_from_list([]), 12, q.QSIM_C64, 0.1, 0.01, 0.01, 3, 0, 64)
    # no gate steps: no angle errors and no flip draws
    assert np.all(F == 1.0)


def test_largest_register_ghz_m34_complex64():
    """M = 34, the library's maximum: a 128 GiB complex64 register."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    free, total = ctypes.c_size_t(), ctypes.c_size_t()
    assert hip.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    if free.value < 132 * GiB:
        pytest.skip("needs 132 GiB of free device memory")
    M = q.QSIM_MAX_QUBITS
    print(f"GHZ M={M} complex64", flush=True)
    with q.State(M, q.QSIM_C64) as s:
        s.apply(cg.ghz_circuit(M))
        h = float(np.float32(np.sqrt(0.5)))
        assert s.amplitudes(0, 1)[0] == h and s.amplitudes((1 << M) - 1, 1)[0] == h
        assert s.amplitudes(1 << 33, 1)[0] == 0.0
        p = s.probs(1 | (1 << 33))
        assert np.max(np.abs(p - [0.5, 0.0, 0.0, 0.5])) < 1e-6
    with pytest.raises(q.QsimError):
        q.State(M + 1, q.QSIM_C64)
