"""The three-state (detailed Cirac-Zoller) model on the GPU against the FP64
three-state oracle, through the C-ABI: raw amplitudes within 1e-12
(complex128) / 2e-5 (complex64), exact CNOT truth table, marginals and
fidelity, and agreement with the two-state model when nothing goes wrong."""
import numpy as np
import pytest

import circuitgen as cg
import oracle
import paper_quant_ph_9804039_amd as q

pytestmark = pytest.mark.gpu

KINDS = (cg.H, cg.RZ, cg.X, cg.Z, cg.CNOT, cg.TOFFOLI, cg.CPHASE)
TOL = {q.QSIM_C128: 1e-12, q.QSIM_C64: 2e-5}


def binary_indices(M):
    return np.array([sum(((i >> b) & 1) * 3 ** b for b in range(M)) for i in range(1 << M)])


@pytest.mark.parametrize("dtype", [q.QSIM_C128, q.QSIM_C64])
def test_cnot_truth_table_in_the_detailed_model(dtype):
    M = 4
    with q.State3(M, dtype) as s:
        for c, t in [(1, 0), (0, 3), (3, 2)]:
            for bc in (0, 1):
                for bt in (0, 1):
                    k = bc * 3 ** c + bt * 3 ** t
                    s.reset(k)
                    s.apply(cg.gates_from_list([(cg.CNOT, t, c)]))
                    a = s.amplitudes()
                    want = bc * 3 ** c + (bt ^ bc) * 3 ** t
                    assert abs(a[want] - 1.0) < (1e-15 if dtype == q.QSIM_C128 else 1e-6)
                    assert np.max(np.abs(np.delete(a, want))) < (1e-15 if dtype == q.QSIM_C128
                                                                 else 1e-6)


@pytest.mark.parametrize("dtype", [q.QSIM_C128, q.QSIM_C64])
@pytest.mark.parametrize("M,seed", [(5, 1), (8, 2)])
def test_circuits_with_errors_and_flips_vs_oracle(dtype, M, seed):
    print(f"three-state M={M} seed={seed} dtype={dtype}", flush=True)
    g = cg.random_circuit(M, 60, 300 + seed, kinds=KINDS)
    em = oracle.Errors(sigma=0.02, p_bitflip=0.01, p_phaseflip=0.01, seed=seed, trial=3)
    ref = oracle.as_complex(oracle.simulate3(M, g, em))
    with q.State3(M, dtype) as s:
        s.inject_errors(em.sigma, em.p_bitflip, em.p_phaseflip, em.seed, em.trial)
        for part in np.array_split(g, 2):  # split calls draw the same errors
            s.apply(part)
        a = s.amplitudes()
        assert s.info()["step"] == len(g)
        assert s.info()["transformations"] == len(q.qsim3_lower(g, M))
    assert np.all(np.isfinite(a)) and np.max(np.abs(a - ref)) <= TOL[dtype]


def test_conditional_transformations_vs_oracle():
    M = 5
    rng = np.random.default_rng(55)
    pulses = []
    for _ in range(40):
        a, b = sorted(rng.choice(3, 2, replace=False).tolist())
        ion = int(rng.integers(M))
        p = {"kind": int(rng.integers(2)), "ion": ion, "a": a, "b": b, "cond_ion": -1,
             "cond_level": 0, "theta": float(rng.uniform(0, 7)), "phi": float(rng.uniform(-3, 3))}
        if rng.random() < 0.6:
            p["cond_ion"] = int(rng.choice([x for x in range(M) if x != ion]))
            p["cond_level"] = int(rng.integers(3))
        pulses.append(p)
    psi = oracle.init3(M, 7)
    for p in pulses:
        oracle.apply_pulse3(psi, M, p)
    with q.State3(M, q.QSIM_C128) as s:
        s.reset(7)
        s.apply_pulses(pulses)
        assert np.max(np.abs(s.amplitudes() - oracle.as_complex(psi))) < 1e-13


@pytest.mark.parametrize("dtype", [q.QSIM_C128, q.QSIM_C64])
def test_marginals_fidelity_and_two_state_agreement(dtype):
    M = 7
    g = cg.random_circuit(M, 80, 777, kinds=KINDS)
    em = oracle.Errors(sigma=0.05, seed=7, trial=1)
    ideal_ref = oracle.simulate3(M, g)
    noisy_ref = oracle.simulate3(M, g, em)
    with q.State3(M, dtype) as a, q.State3(M, dtype) as b, q.State(M, dtype) as two:
        a.apply(g)
        b.inject_errors(em.sigma, seed=em.seed, trial=em.trial)
        b.apply(g)
        two.apply(g)
        for mask in (0b1, 0b1011, 0b111111):
            pr = b.probs(mask)
            assert np.max(np.abs(pr - oracle.probs3(noisy_ref, M, mask))) < 10 * TOL[dtype]
        r1, r2 = oracle.as_complex(ideal_ref), oracle.as_complex(noisy_ref)
        F_ref = abs(np.vdot(r1, r2)) ** 2 / (np.vdot(r1, r1).real * np.vdot(r2, r2).real)
        assert abs(a.fidelity(b) - F_ref) < (1e-12 if dtype == q.QSIM_C128 else 1e-6)
        # error-free: the two-state register up to a global phase, nothing in level 2
        a3 = a.amplitudes()[binary_indices(M)]
        a2 = two.amplitudes()
        assert 1.0 - abs(np.vdot(a2, a3)) ** 2 < (1e-12 if dtype == q.QSIM_C128 else 1e-5)
        assert abs(1.0 - np.sum(np.abs(a3) ** 2)) < (1e-12 if dtype == q.QSIM_C128 else 1e-5)


def test_bad_arguments_rejected():
    with pytest.raises(q.QsimError):
        q.State3(21, q.QSIM_C64)
    with q.State3(4, q.QSIM_C64) as s:
        with pytest.raises(q.QsimError):
            s.apply(cg.gates_from_list([(cg.CNOT, 1, 1)]))
        with pytest.raises(q.QsimError):
            s.apply_pulses([{"kind": 0, "ion": 0, "a": 2, "b": 1}])
        with pytest.raises(q.QsimError):
            s.apply_pulses([{"kind": 0, "ion": 1, "a": 0, "b": 1, "cond_ion": 1}])
        with pytest.raises(q.QsimError):
            s.reset(81)
        with pytest.raises(q.QsimError):
            s.probs(0b1111111)
        assert s.info()["transformations"] == 0


def test_bench_size_register_matches_the_two_state_oracle_on_sampled_blocks():
    """19 ions (3^19 = 1.16e9 amplitudes), the bench's gate kinds, no errors:
    the amplitudes whose ions are all in levels 0/1 equal the two-state
    oracle's (up to one global phase), everything with a level-2 ion is zero.
    Checked on two contiguous blocks of 3^9 indices (ions 9..18 fixed to the
    high bits of two of the largest two-state amplitudes)."""
    M = 19
    print("three-state M=19 sampled blocks", flush=True)
    g = cg.random_circuit(M, 60, 319, kinds=(cg.H, cg.RZ, cg.X, cg.Z, cg.CNOT))
    ref = oracle.as_complex(oracle.simulate(M, g))
    order = np.argsort(-np.abs(ref))
    digits = (np.arange(3 ** 9)[:, None] // 3 ** np.arange(9)) % 3
    binary = np.all(digits < 2, axis=1)
    low = (digits[binary] * (1 << np.arange(9))).sum(axis=1)
    with q.State3(M, q.QSIM_C64) as s:
        s.apply(g)
        phase = None
        for top in (int(order[0]), int(order[len(order) // 8])):
            hi = [(top >> (9 + i)) & 1 for i in range(M - 9)]
            off = int(sum(b * 3 ** (9 + i) for i, b in enumerate(hi)))
            blk = s.amplitudes(off, 3 ** 9)
            want = ref[low + (top >> 9 << 9)]
            got = blk[binary]
            if phase is None:
                k = int(np.argmax(np.abs(want)))
                assert abs(want[k]) > 1e-3
                phase = got[k] / want[k]
            assert abs(abs(phase) - 1.0) < 1e-5
            assert np.max(np.abs(got - phase * want)) < 2e-5
            assert np.max(np.abs(blk[~binary])) < 2e-6
        assert abs(float(np.sum(s.probs(1))) - 1.0) < 1e-5


def test_largest_register_cnot_and_x_on_basis_states():
    """20 ions (3^20 = 3.5e9 amplitudes, 28 GB complex64), the largest the
    library takes: X and CNOT on basis states give basis states (to the
    rounding of the pulses' cos and sin: cos(pi/2) is 6e-17 in FP64)."""
    M = 20
    print("three-state M=20 basis states", flush=True)
    with q.State3(M, q.QSIM_C64) as s:
        s.apply(cg.gates_from_list([(cg.X, 19), (cg.CNOT, 0, 19), (cg.CNOT, 10, 0),
                                    (cg.X, 10)]))
        want = 3 ** 19 + 3 ** 0  # ions 19, 0 in level 1; ion 10 flipped twice
        a = s.amplitudes(want - 2, 5)
        # each X is a pi pulse, -i X: the two of ion 10 leave a global phase
        assert abs(abs(a[2]) - 1.0) < 1e-6 and np.max(np.abs(np.delete(a, 2))) < 1e-15
        assert abs(float(np.sum(s.probs(1 << 19))) - 1.0) < 1e-6


@pytest.mark.parametrize("dtype", [q.QSIM_C128, q.QSIM_C64])
@pytest.mark.parametrize("M,seed", [(9, 31), (12, 32)])
def test_fused_passes_vs_oracle_and_per_transformation_path(dtype, M, seed):
    """Registers larger than one tile (3^8 complex64 / 3^7 complex128
    amplitudes) run fused passes: against the oracle with errors and flips,
    against one launch per transformation (exec_mode 1), which does the same
    operations on each pair (the compiler may contract them into FMAs
    differently, so the two agree to rounding, not bit for bit), and against
    fused passes over runs of the stream in order (exec_mode 2): the default
    passes take commuting transformations from further down the stream."""
    print(f"three-state fused M={M} dtype={dtype}", flush=True)
    g = cg.random_circuit(M, 90, 500 + seed, kinds=KINDS)
    em = oracle.Errors(sigma=0.03, p_bitflip=0.01, p_phaseflip=0.01, seed=seed, trial=2)
    ref = oracle.as_complex(oracle.simulate3(M, g, em))
    out, launches = [], []
    npulses = len(q.qsim3_lower(g, M))
    for mode in (0, 1, 2):
        with q.State3(M, dtype, q.make_options(exec_mode=mode)) as s:
            s.inject_errors(em.sigma, em.p_bitflip, em.p_phaseflip, em.seed, em.trial)
            s.apply(g[:40])
            s.apply(g[40:])
            out.append(s.amplitudes())
            info = s.info()
            assert info["transformations"] == npulses
            launches.append(info["launches"])
            # fused: a few passes; per transformation: one launch each (flips too)
            assert (info["launches"] >= npulses) if mode == 1 else (info["launches"] < npulses // 3)
    assert launches[0] <= launches[2]
    for o in out:
        assert np.max(np.abs(o - ref)) <= TOL[dtype]
    assert np.max(np.abs(out[0] - out[1])) <= TOL[dtype]
    assert np.max(np.abs(out[2] - out[1])) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [q.QSIM_C128, q.QSIM_C64])
def test_fused_conditional_transformations_inside_and_outside_the_tile(dtype):
    """Conditions on ions inside and outside a pass's tile (M = 11: a tile
    holds 7 (complex128) or 8 (complex64) of the 11 ions), on the other ion
    of a register group, on a tile ion outside the group, and on an ion
    outside the tile."""
    M = 11
    rng = np.random.default_rng(77)
    pulses = []
    for _ in range(120):
        a, b = sorted(rng.choice(3, 2, replace=False).tolist())
        ion = int(rng.integers(M))
        p = {"kind": int(rng.integers(2)), "ion": ion, "a": a, "b": b, "cond_ion": -1,
             "cond_level": 0, "theta": float(rng.uniform(0, 7)), "phi": float(rng.uniform(-3, 3))}
        if rng.random() < 0.7:
            p["cond_ion"] = int(rng.choice([x for x in range(M) if x != ion]))
            p["cond_level"] = int(rng.integers(3))
        pulses.append(p)
    psi = oracle.init3(M, 5)
    # start from a spread state: every ion through a rotation first
    spread = [{"kind": 0, "ion": q_, "a": 0, "b": 1, "cond_ion": -1, "cond_level": 0,
               "theta": 1.1 + 0.1 * q_, "phi": 0.3} for q_ in range(M)]
    spread += [{"kind": 0, "ion": q_, "a": 1, "b": 2, "cond_ion": -1, "cond_level": 0,
                "theta": 0.7, "phi": -0.2 * q_} for q_ in range(M)]
    for p in spread + pulses:
        oracle.apply_pulse3(psi, M, p)
    tol = 1e-12 if dtype == q.QSIM_C128 else 2e-5
    for mode in (0, 2):
        with q.State3(M, dtype, q.make_options(exec_mode=mode)) as s:
            s.reset(5)
            s.apply_pulses(spread + pulses)
            assert np.max(np.abs(s.amplitudes() - oracle.as_complex(psi))) < tol
