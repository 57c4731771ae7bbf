"""The execution order chosen by the pass scheduler (CPU only, through
qsim_plan): a permutation of the operation stream that keeps the relative
order of every two operations that do not commute, never moves an operation
across a renormalisation boundary, and keeps every fused pass's targets in its
tile.  The stream and the commutation rule are modelled here from the gates
and the oracle's flip draws, independently of the library."""
import numpy as np
import pytest

import circuitgen as cg
import oracle
import paper_quant_ph_9804039_amd as q


@pytest.fixture(scope="module", autouse=True)
def _lib():
    try:
        q.lib()
    except ImportError as e:
        pytest.skip(str(e))


def _stream(gates, M, em):
    """Per operation [x_qubits, z_qubits, target or None, step, step_end]:
    x = target of a non-diagonal transform, z = controls and diagonal
    targets; the target is kept when the operation needs it in the tile
    (everything but an uncontrolled diagonal)."""
    ops = []
    for s, g in enumerate(gates):
        kind, t = int(g["kind"]), int(g["target"])
        ctrls = {int(c) for c in (g["ctrl0"], g["ctrl1"]) if c >= 0}
        diag = kind in (cg.RZ, cg.Z, cg.CPHASE)
        ops.append([set() if diag else {t}, ctrls | ({t} if diag else set()),
                    t if (not diag or ctrls) else None, s, True])
        for qb in range(M):
            ev = oracle.flip_events(em, s, qb)
            if ev:
                ops[-1][4] = False
            if ev & 1:
                ops.append([{qb}, set(), qb, s, True])
            if ev & 2:
                if ev & 1:
                    ops[-1][4] = False
                ops.append([set(), {qb}, None, s, True])
    return ops


def _commute(a, b):
    return not (a[0] & (b[0] | b[1])) and not (b[0] & (a[0] | a[1]))


def _check(M, gates, em, opt, period=0):
    passes, nops, order = q.qsim_plan(M, q.QSIM_C64, gates, opt, sigma=em.sigma,
                                      p_bitflip=em.p_bitflip, p_phaseflip=em.p_phaseflip,
                                      seed=em.seed, trial=em.trial, return_order=True)
    ops = _stream(gates, M, em)
    assert nops == len(ops)
    assert sorted(order.tolist()) == list(range(nops))
    pos = np.empty(nops, dtype=np.int64)
    pos[order] = np.arange(nops)
    for i in range(nops):
        for j in range(i + 1, nops):
            if not _commute(ops[i], ops[j]):
                assert pos[i] < pos[j], (i, j)
    # renormalisation: the norm follows the first pass by which every
    # operation up to a boundary (the end of every period-th step) has run
    if period > 0:
        want = set()
        for i, op in enumerate(ops):
            if op[4] and (op[3] + 1) % period == 0:
                done_at = pos[: i + 1].max()
                want.add(next(n for n, p in enumerate(passes)
                              if p["first_op"] <= done_at < p["first_op"] + p["n_ops"]))
        assert {n for n, p in enumerate(passes) if p["norm_after"]} == want
    nxt = 0
    for p in passes:
        assert p["first_op"] == nxt
        nxt += p["n_ops"]
        if p["fused"]:
            for i in order[p["first_op"]: p["first_op"] + p["n_ops"]]:
                if ops[i][2] is not None:
                    assert (p["tile_mask"] >> ops[i][2]) & 1, (p, i)
    assert nxt == nops
    return passes, order, ops


@pytest.mark.parametrize("M,seed", [(12, 1), (16, 2), (20, 3), (30, 4)])
def test_order_keeps_every_non_commuting_pair(M, seed):
    gates = cg.random_circuit(M, 200, seed, kinds=(cg.H, cg.RZ, cg.X, cg.Z, cg.CNOT, cg.TOFFOLI,
                                                     cg.CPHASE))
    em = oracle.Errors(sigma=0.01, p_bitflip=0.01, p_phaseflip=0.01, seed=seed, trial=5)
    _check(M, gates, em, q.make_options(lazy_qubits=-1))


def test_tiles_hold_the_targets_at_full_tile_size():
    M = 24
    gates = cg.random_circuit(M, 300, 8)
    em = oracle.Errors(sigma=1e-3, p_bitflip=1e-3, p_phaseflip=1e-3, seed=8, trial=0)
    passes, _, _ = _check(M, gates, em, q.make_options(lazy_qubits=-1))
    assert all(p["fused"] and bin(p["tile_mask"]).count("1") == 13 for p in passes)


@pytest.mark.parametrize("mode", [0, 2])
def test_norm_follows_the_pass_that_completes_each_boundary(mode):
    M = 16
    gates = cg.random_circuit(M, 256, 11)
    em = oracle.Errors(sigma=0.0, p_bitflip=0.005, p_phaseflip=0.005, seed=11, trial=2)
    passes, _, _ = _check(M, gates, em, q.make_options(lazy_qubits=-1, renorm_period=16, exec_mode=mode),
                          period=16)
    assert 1 <= sum(p["norm_after"] for p in passes) <= 256 // 16


def test_in_order_mode_runs_the_stream_as_is():
    M = 20
    gates = cg.random_circuit(M, 300, 12)
    passes, nops, order = q.qsim_plan(M, q.QSIM_C64, gates, q.make_options(lazy_qubits=-1, exec_mode=2),
                                      return_order=True)
    assert np.array_equal(order, np.arange(nops))
    plain, _, order1 = q.qsim_plan(M, q.QSIM_C64, gates, q.make_options(lazy_qubits=-1, exec_mode=1),
                                   return_order=True)
    assert np.array_equal(order1, np.arange(nops)) and len(plain) == nops


def test_reordering_cuts_the_passes_of_a_uniform_random_circuit():
    # targets uniform over 30 qubits: commuting gates from further down the
    # stream fill each tile, so a third fewer passes than runs of the stream
    gates = cg.random_circuit(30, 1000, 30)
    reord, _ = q.qsim_plan(30, q.QSIM_C64, gates, q.make_options(lazy_qubits=-1))
    inorder, _ = q.qsim_plan(30, q.QSIM_C64, gates, q.make_options(lazy_qubits=-1, exec_mode=2))
    assert all(p["fused"] for p in reord + inorder)
    assert len(reord) * 1.3 < len(inorder)
    assert 1000 / len(reord) > 20
    # inside a pass, commuting operations are clustered by target, so fewer
    # register groups (LDS re-partitions) per operation
    per_op = lambda ps: sum(p["n_groups"] for p in ps) / sum(p["n_ops"] for p in ps)
    assert per_op(reord) < 0.8 * per_op(inorder)


@pytest.mark.parametrize("seed,most", [(30, 30), (31, 32), (32, 33)])
def test_lookahead_tile_sets_carry_more_operations(seed, most):
    # Growing each tile set by the qubits of the first operations met (first
    # come, first served) needs 36-39 passes for these circuits; picking the
    # qubits that let the pass take the most of the next operations needs
    # about a sixth fewer.  Every pass still holds the targets of its
    # operations and keeps every non-commuting pair in order.
    M = 30
    gates = cg.random_circuit(M, 1000, seed)
    em = oracle.Errors(sigma=1e-3, p_bitflip=1e-4, p_phaseflip=1e-4, seed=1030, trial=1)
    passes, _, _ = _check(M, gates, em, q.make_options(lazy_qubits=-1, renorm_period=64), period=64)
    assert len(passes) <= most
    assert all(p["n_ops"] >= 1 for p in passes)


@pytest.mark.parametrize("seed", [30, 31, 32])
def test_register_groups_close_to_the_target_bound(seed):
    # A pass needs at least ceil(distinct targets / G) register groups (G = 4).
    # Choosing each group's target bits by lookahead over the pass's
    # operations stays within a fifth of that bound (filling the bits first
    # come, first served was a quarter above it).
    M = 30
    gates = cg.random_circuit(M, 1000, seed)
    em = oracle.Errors(sigma=1e-3, p_bitflip=1e-4, p_phaseflip=1e-4, seed=1030, trial=1)
    passes, order, ops = _check(M, gates, em, q.make_options(lazy_qubits=-1, renorm_period=64),
                                period=64)
    bound = 0
    for p in passes:
        targets = {ops[i][2] for i in order[p["first_op"]: p["first_op"] + p["n_ops"]]
                   if ops[i][2] is not None}
        bound += -(-len(targets) // 4)
    groups = sum(p["n_groups"] for p in passes)
    assert bound <= groups <= 1.2 * bound
