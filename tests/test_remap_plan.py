"""Qubit remap on the host (CPU only, through qsim_plan): when a call's
operations use top qubits far more than low ones, the call exchanges them
(three exact CNOT swaps per pair) at its start and back at its end; every
pass passes the library's own argument check."""
import numpy as np
import pytest

import circuitgen as cg
import paper_quant_ph_9804039_amd as q


@pytest.fixture(scope="module", autouse=True)
def _lib():
    try:
        q.lib()
    except ImportError as e:
        pytest.skip(str(e))


def _nops(M, gates, **kw):
    _, n = q.qsim_plan(M, q.QSIM_C64, gates, q.make_options(lazy_qubits=-1, **kw))
    return n


def test_large_register_with_top_heavy_targets_is_remapped():
    M = 33
    gates = cg.random_circuit(M, 500, M, top_bias=0.5)
    base = _nops(M, gates, remap_qubits=-1)
    auto = _nops(M, gates)
    assert base == len(gates)
    pairs = (auto - base) // 12  # three swaps per pair, at the start and at the end
    assert auto - base == 12 * pairs and 1 <= pairs <= 4


def test_complex128_remaps_only_when_asked():
    M = 32
    gates = cg.random_circuit(M, 500, M, top_bias=0.5)
    opt = q.make_options(lazy_qubits=-1)
    _, auto = q.qsim_plan(M, q.QSIM_C128, gates, opt)
    _, forced = q.qsim_plan(M, q.QSIM_C128, gates, q.make_options(lazy_qubits=-1, remap_qubits=1))
    assert auto == len(gates) and forced > len(gates)


def test_no_remap_below_the_size_or_without_top_heavy_use():
    gates = cg.random_circuit(30, 500, 30, top_bias=0.5)
    assert _nops(30, gates) == len(gates)
    uniform = cg.random_circuit(33, 500, 33)
    assert _nops(33, uniform) == len(uniform)


@pytest.mark.parametrize("M,mode,lazy", [(18, 0, -1), (18, 2, 1), (24, 0, 1), (34, 0, -1)])
def test_eager_remap_plans_are_consistent(M, mode, lazy):
    gates = cg.random_circuit(M, 300, M + 7, top_bias=0.6,
                              kinds=(cg.H, cg.RZ, cg.CNOT, cg.TOFFOLI, cg.CPHASE))
    for dtype in (q.QSIM_C64, q.QSIM_C128):
        opt = q.make_options(exec_mode=mode, lazy_qubits=lazy, remap_qubits=1)
        passes, nops = q.qsim_plan(M, dtype, gates, opt, sigma=0.01, p_bitflip=1e-3,
                                   p_phaseflip=1e-3, seed=3, trial=2)
        assert passes
    with pytest.raises(q.QsimError):
        q.qsim_plan(M, q.QSIM_C64, gates, q.make_options(remap_qubits=2))
