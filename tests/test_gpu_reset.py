"""A reset is written by the first fused pass of the next apply call (the
pass builds the basis state instead of loading the register), or before
anything else reads the register.  These tests go through every way a
pending reset can be consumed and compare with the FP64 oracle started from
the same basis state (Sec. 1.2, Fig. 1(a)).
"""
import numpy as np
import pytest

import circuitgen as cg
import oracle
import paper_quant_ph_9804039_amd as q

pytestmark = pytest.mark.gpu

TOL = {q.QSIM_C128: 1e-12, q.QSIM_C64: 2e-5}


def basis(M, k):
    v = np.zeros(1 << M, dtype=np.complex128)
    v[k] = 1.0
    return v


def scrambled(M, dtype, **kw):
    """A state whose memory holds something other than a basis state."""
    s = q.State(M, dtype, q.make_options(**kw) if kw else None)
    s.apply(cg.random_circuit(M, 60, 900 + M))
    return s


@pytest.mark.parametrize("dtype", [q.QSIM_C64, q.QSIM_C128])
@pytest.mark.parametrize("mode,lazy", [(0, -1), (2, -1), (1, -1), (0, 0)])
def test_reset_then_apply_matches_the_oracle(dtype, mode, lazy):
    # fused passes over the whole register build the basis state in their
    # first pass; per-gate passes and lazy passes write it first
    M, k = 16, 0b1011001110001101
    print(f"reset+apply M={M} dtype={dtype} mode={mode} lazy={lazy}", flush=True)
    g = cg.random_circuit(M, 150, 77)
    em = oracle.Errors(sigma=0.02, p_bitflip=0.01, p_phaseflip=0.01, seed=3, trial=4)
    ref = oracle.as_complex(oracle.simulate(M, g, em, k=k))
    with scrambled(M, dtype, exec_mode=mode, lazy_qubits=lazy) as s:
        s.reset(k)
        s.inject_errors(em.sigma, em.p_bitflip, em.p_phaseflip, em.seed, em.trial)
        s.apply(g[:70])
        s.apply(g[70:])
        got = s.amplitudes()
    assert np.max(np.abs(got - ref)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [q.QSIM_C64, q.QSIM_C128])
def test_pending_reset_is_written_before_every_readout(dtype):
    M, k = 14, 9001
    print(f"pending reset readouts M={M} dtype={dtype}", flush=True)
    want = basis(M, k)
    with scrambled(M, dtype) as s, scrambled(M, dtype) as t:
        s.reset(k)
        assert np.array_equal(s.amplitudes(), want)
        s.reset(k)
        p = s.probs()
        assert p[k] == 1.0 and np.count_nonzero(p) == 1
        s.reset(k)
        assert s.norm() == 1.0
        # fidelity against a state that is not reset: |<t|k>|^2
        s.reset(k)
        tv = t.amplitudes()
        F = s.fidelity(t)
        assert abs(F - abs(tv[k]) ** 2 / np.vdot(tv, tv).real) <= TOL[dtype]
        # both pending at once
        s.reset(k)
        t.reset(k)
        assert abs(s.fidelity(t) - 1.0) <= 1e-15
        # a partial write lands on the basis state, not on the old contents
        s.reset(k)
        s.set_amplitudes(np.full(4, 0.5, dtype=np.complex128), offset=8)
        got = s.amplitudes()
        exp = want.copy()
        exp[8:12] = 0.5
        assert np.array_equal(got, exp)
        # an empty call, and the device pointer
        s.reset(k)
        s.apply(cg.random_circuit(M, 0, 1))
        assert np.array_equal(s.amplitudes(), want)
        s.reset(k)
        assert s.info()["device_ptr"] != 0
        s.synchronize()
        assert np.array_equal(s.amplitudes(), want)


@pytest.mark.parametrize("dtype", [q.QSIM_C64, q.QSIM_C128])
def test_reset_twice_keeps_the_last_index(dtype):
    M = 15
    g = cg.random_circuit(M, 40, 12)
    ref = oracle.as_complex(oracle.simulate(M, g, None, k=77))
    with scrambled(M, dtype) as s:
        s.reset(5)
        s.reset(77)
        s.apply(g)
        assert np.max(np.abs(s.amplitudes() - ref)) <= TOL[dtype]


def test_direct_readers_see_the_reset_state_after_synchronize():
    # a reader of the device memory (here the allocation-free overlap, which
    # takes raw pointers) calls synchronize first, which writes a pending
    # reset and waits for it
    M, k = 12, 1234
    with scrambled(M, q.QSIM_C64) as a, scrambled(M, q.QSIM_C64) as b:
        a.reset(k)
        a.synchronize()
        b.synchronize()
        ia, ib = a.info(), b.info()
        ov, na, _ = q.qsim_overlap_noalloc(ia["device_ptr"], ia["dtype"], ib["device_ptr"],
                                           ib["dtype"], M)
        bv = b.amplitudes()
        assert na == 1.0
        assert abs(ov - bv[k]) <= 1e-7
