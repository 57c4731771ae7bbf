"""Host side of lazy qubits (CPU only, through qsim_plan): passes over a
register whose qubits come into play late span only the touched subspace,
every pass's kernel arguments pass the library's own consistency check, and
the stream rewrite decides controls on untouched qubits."""
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


def test_structured_circuit_on_top_qubits_spans_one_tile():
    M = 30
    qm = list(range(M - 9, M))
    gates = np.concatenate([cg.modexp15_circuit(5, qubit_map=qm), cg.qft_circuit(qm[:5])])
    passes, _ = q.qsim_plan(M, q.QSIM_C64, gates)
    assert passes and all(p["fused"] for p in passes)
    assert all(p["span_qubits"] == 13 and p["tiles"] == 1 for p in passes)
    full, _ = q.qsim_plan(M, q.QSIM_C64, gates, q.make_options(lazy_qubits=-1))
    assert all(p["span_qubits"] == M and p["tiles"] == 1 << (M - 13) for p in full)


def test_span_grows_with_the_touched_qubits():
    M = 30
    gates = cg.random_circuit(M, 1000, 30)
    passes, _ = q.qsim_plan(M, q.QSIM_C64, gates)
    spans = [p["span_qubits"] for p in passes]
    assert spans[0] == 13
    assert all(a <= b for a, b in zip(spans, spans[1:]))
    assert spans[-1] == M
    # algorithmic flops follow the span
    full, _ = q.qsim_plan(M, q.QSIM_C64, gates, q.make_options(lazy_qubits=-1))
    assert sum(p["flops"] for p in passes) < sum(p["flops"] for p in full)


def test_controls_on_untouched_qubits_are_decided():
    M = 16
    # qubit 9 holds 0: the CNOT and Toffoli it controls are dropped; after an
    # X on it (a value flip, no data moved) the CNOT runs uncontrolled
    gates = cg.gates_from_list([(cg.H, 0), (cg.CNOT, 1, 9), (cg.TOFFOLI, 2, 0, 9), (cg.X, 9),
                                (cg.CNOT, 3, 9), (cg.RZ, 12, -1, -1, 0.3), (cg.Z, 9)])
    passes, nops, order = q.qsim_plan(M, q.QSIM_C128, gates, return_order=True)
    # kept: H(0); CNOT(3) loses its decided control and, its target being
    # untouched too, only flips qubit 3's value; at the end two swaps move
    # qubits 3 and 9 to their new values and one scalar operation applies the
    # phase gathered from Rz(12) and Z(9)
    assert nops == 4
    full, nops_full = q.qsim_plan(M, q.QSIM_C128, gates, q.make_options(lazy_qubits=-1))
    assert nops_full == len(gates)


@pytest.mark.parametrize("M,seed,p", [(20, 1, 0.0), (24, 2, 0.01), (30, 3, 0.002), (34, 4, 0.001)])
def test_consistency_of_lazy_plans_with_flips(M, seed, p):
    rng = np.random.default_rng(seed)
    order = rng.permutation(M)
    items = []
    for g in range(400):
        m = min(M, 3 + g * M // 300)
        qs = [int(x) for x in rng.choice(order[:m], 3, replace=False)]
        kind = [cg.H, cg.RZ, cg.CNOT, cg.TOFFOLI, cg.CPHASE, cg.X][g % 6]
        ar = cg.ARITY[kind]
        c = qs[1:ar] + [-1] * (3 - ar)
        items.append((kind, qs[0], c[0], c[1], 0.7 if kind in cg.ANGLED else 0.0))
    gates = cg.gates_from_list(items)
    for mode in (0, 2):
        for dtype in (q.QSIM_C64, q.QSIM_C128):
            passes, _ = q.qsim_plan(M, dtype, gates, q.make_options(exec_mode=mode), sigma=0.01,
                                    p_bitflip=p, p_phaseflip=p, seed=seed, trial=1)
            spans = [x["span_qubits"] for x in passes if x["fused"]]
            assert spans and all(a <= b for a, b in zip(spans, spans[1:]))


def test_lazy_option_validated():
    with pytest.raises(q.QsimError):
        q.qsim_plan(12, q.QSIM_C64, cg.random_circuit(12, 5, 1), q.make_options(lazy_qubits=2))
    # the per-operation path never skips
    passes, _ = q.qsim_plan(12, q.QSIM_C64, cg.random_circuit(12, 5, 1),
                            q.make_options(exec_mode=1, lazy_qubits=1))
    assert all(p["span_qubits"] == 12 for p in passes)
