"""Qubit remap (the one-GPU reorganisation of Sec. 3.1, 3.3, Fig. 8) on the
GPU, through the C-ABI: exchanging top qubits with low ones for the length of
a call and back changes nothing but the memory access pattern, so remapped
runs match the FP64 oracle, and exact permutation circuits are bit-identical
with and without the remap."""
import numpy as np
import pytest

import circuitgen as cg
import oracle
import paper_quant_ph_9804039_amd as q

pytestmark = pytest.mark.gpu

TOL = {q.QSIM_C128: 1e-12, q.QSIM_C64: 2e-5}


@pytest.mark.parametrize("mode,lazy", [(0, -1), (0, 1), (2, 1)])
@pytest.mark.parametrize("dtype", [q.QSIM_C128, q.QSIM_C64])
def test_remapped_runs_match_oracle(mode, lazy, dtype):
    M = 18
    print(f"remap vs oracle mode={mode} lazy={lazy} dtype={dtype}", flush=True)
    gates = cg.random_circuit(M, 300, 1818, top_bias=0.6,
                              kinds=(cg.H, cg.RZ, cg.CNOT, cg.TOFFOLI, cg.CPHASE))
    em = oracle.Errors(sigma=1e-3, p_bitflip=1e-3, p_phaseflip=1e-3, seed=818, trial=4)
    ref = oracle.as_complex(oracle.simulate(M, gates, em))
    opt = q.make_options(exec_mode=mode, lazy_qubits=lazy, remap_qubits=1)
    with q.State(M, dtype, opt) as s:
        s.inject_errors(em.sigma, em.p_bitflip, em.p_phaseflip, em.seed, em.trial)
        s.profile(True)
        for part in np.array_split(gates, 3):  # every call remaps and maps back
            s.apply(part)
        st = s.stats()
        a = s.amplitudes()
    assert st["remaps"] >= 3
    assert np.all(np.isfinite(a)) and np.max(np.abs(a - ref)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [q.QSIM_C128, q.QSIM_C64])
def test_permutation_circuit_bit_identical_with_and_without_remap(dtype):
    M = 16
    gates = cg.random_circuit(M, 240, 1616, top_bias=0.7, kinds=(cg.X, cg.CNOT, cg.TOFFOLI, cg.Z))
    v = cg.random_state(M, 16)
    if dtype == q.QSIM_C64:
        v = v.astype(np.float32).astype(np.float64)
    out = []
    for remap in (1, -1):
        with q.State(M, dtype, q.make_options(remap_qubits=remap, renorm_period=-1)) as s:
            s.set_amplitudes(v)
            s.profile(True)
            s.apply(gates)
            out.append(s.amplitudes())
            if remap == 1:
                assert s.stats()["remaps"] >= 1
    assert np.array_equal(out[0], out[1])
    assert np.array_equal(out[1], oracle.as_complex(oracle.run(v.copy(), M, gates)))


def test_m33_remap_agrees_with_plain_layout():
    """The large-register configuration (M = 33 complex64, half of the
    targets on the top four qubits): the automatic remap runs, and the state
    equals the one computed in the plain layout to complex64 rounding."""
    M = 33
    gates = cg.random_circuit(M, 300, M, top_bias=0.5)
    with q.State(M, q.QSIM_C64, q.make_options(lazy_qubits=-1)) as a, \
            q.State(M, q.QSIM_C64, q.make_options(lazy_qubits=-1, remap_qubits=-1)) as b:
        for s in (a, b):
            s.inject_errors(1e-3, 0.0, 0.0, seed=1033, trial=0)
            s.profile(True)
            s.apply(gates)
        assert a.stats()["remaps"] >= 1 and b.stats()["remaps"] == 0
        ab, aa, bb = a.overlap(b)
        assert 1.0 - abs(ab) ** 2 / (aa * bb) < 1e-10
