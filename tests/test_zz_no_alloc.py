"""qsim_overlap_noalloc (static device scratch, no allocation) against
qsim_overlap on the same registers, through the C-ABI.

Two calls in a row, the second on a smaller register, so the shared scratch
array keeps the first call's partials when the second starts; the results
must still equal the allocating entry point's bit for bit (same kernels, same
fixed reduction order), and the fidelity the oracle's within tolerance.
"""
import numpy as np
import pytest

import circuitgen as cg
import oracle
import paper_quant_ph_9804039_amd as q

pytestmark = pytest.mark.gpu


def _pair(M, dtype_a, dtype_b, seed):
    gates = cg.random_circuit(M, 120, seed)
    a = q.State(M, dtype_a)
    b = q.State(M, dtype_b)
    a.apply(gates)
    b.inject_errors(0.02, 1e-3, 1e-3, seed=seed + 1, trial=3)
    b.apply(gates)
    a.synchronize()
    b.synchronize()
    return gates, a, b


def _noalloc(a, b, M):
    ia, ib = a.info(), b.info()
    return q.qsim_overlap_noalloc(ia["device_ptr"], ia["dtype"], ib["device_ptr"], ib["dtype"], M)


@pytest.mark.parametrize("dtypes", [(q.QSIM_C64, q.QSIM_C64), (q.QSIM_C128, q.QSIM_C128),
                                    (q.QSIM_C64, q.QSIM_C128), (q.QSIM_C128, q.QSIM_C64)])
def test_noalloc_overlap_equals_overlap_two_calls_shrinking(dtypes):
    for M, seed in ((20, 71), (11, 72)):   # second call: smaller input
        gates, a, b = _pair(M, dtypes[0], dtypes[1], seed)
        with a, b:
            ref_ab, ref_aa, ref_bb = a.overlap(b)
            ab, aa, bb = _noalloc(a, b, M)
            assert (ab, aa, bb) == (ref_ab, ref_aa, ref_bb), M
            F = abs(ab) ** 2 / (aa * bb)
            if dtypes == (q.QSIM_C128, q.QSIM_C128) and M <= 11:
                em = oracle.Errors(sigma=0.02, p_bitflip=1e-3, p_phaseflip=1e-3, seed=seed + 1,
                                   trial=3)
                F_ref = oracle.fidelity(oracle.simulate(M, gates), oracle.simulate(M, gates, em), M)
                assert abs(F - F_ref) <= 1e-12


def test_noalloc_overlap_rejects_bad_arguments():
    M = 20
    with q.State(M, q.QSIM_C64) as a, q.State(M, q.QSIM_C64) as b:
        pa, pb = a.info()["device_ptr"], b.info()["device_ptr"]
        host = np.zeros(2 << M, dtype=np.float32)
        cases = [
            (pa, q.QSIM_C64, pb, q.QSIM_C64, 0),                    # M below range
            (pa, q.QSIM_C64, pb, q.QSIM_C64, q.QSIM_MAX_QUBITS + 1),  # M above range
            (pa, 7, pb, q.QSIM_C64, M),                              # bad dtype
            (None, q.QSIM_C64, pb, q.QSIM_C64, M),                   # NULL
            (pa + 8, q.QSIM_C64, pb, q.QSIM_C64, M),                 # misaligned
            (host.ctypes.data, q.QSIM_C64, pb, q.QSIM_C64, M),       # host memory
            (pa, q.QSIM_C64, pb, q.QSIM_C64, M + 2),                 # allocation too small
            (pa, q.QSIM_C128, pb, q.QSIM_C64, M),                    # too small as complex128
        ]
        for args in cases:
            with pytest.raises(q.QsimError) as ei:
                q.qsim_overlap_noalloc(*args)
            assert ei.value.code == q.QSIM_EINVAL, args
        with pytest.raises(q.QsimError) as ei:
            q.qsim_overlap_noalloc(pa, q.QSIM_C64, pb, q.QSIM_C64, M, device=99)
        assert ei.value.code == q.QSIM_EINVAL
        assert q.lib().qsim_overlap_noalloc(pa, 0, pb, 0, M, 0, None, None) == q.QSIM_EINVAL
        # the entry point still works after the rejected calls
        assert q.qsim_overlap_noalloc(pa, q.QSIM_C64, pb, q.QSIM_C64, M) == a.overlap(b)
