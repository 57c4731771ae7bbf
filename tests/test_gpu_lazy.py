"""Lazy qubits (the flat form of Sec. 3.2's dynamically allocated state
vector) against the FP64 oracle, through the C-ABI.

Circuits here bring qubits into play one by one, decide controls on qubits
still holding one value, put diagonals and exact X on such qubits, and inject
flips everywhere, so every rule of the rewrite runs: decided controls, scalar
diagonals, virtual bit flips, the realigning swap before a qubit spreads and
the moving swap at the end of a call.  The bar is the parity bar: complex128
within 1e-12 of the oracle, complex64 within 2e-5, raw amplitudes.
"""
import numpy as np
import pytest

import circuitgen as cg
import oracle
import paper_quant_ph_9804039_amd as q

pytestmark = pytest.mark.gpu

TOL = {q.QSIM_C128: 1e-12, q.QSIM_C64: 2e-5}


def late_touch_circuit(M, G, seed, m0=2):
    """Gate g draws its qubits from the first m(g) qubits of a random order,
    m growing from m0 to M over the circuit; a control, a diagonal target or
    an X target is drawn from all M qubits with probability 0.3 (often an
    untouched one)."""
    rng = np.random.default_rng(seed)
    order = [int(x) for x in rng.permutation(M)]
    kinds = [cg.H, cg.RZ, cg.CNOT, cg.TOFFOLI, cg.CPHASE, cg.X, cg.Z]
    items = []
    for g in range(G):
        m = min(M, m0 + (M - m0) * g // max(1, G - G // 5))
        kind = kinds[int(rng.integers(len(kinds)))]
        pool = order[:m]
        wide = rng.random() < 0.3
        if kind in (cg.H,):
            items.append((kind, pool[int(rng.integers(m))]))
        elif kind in (cg.RZ, cg.Z, cg.X):
            src = order if wide else pool
            t = src[int(rng.integers(len(src)))]
            items.append((kind, t, -1, -1, float(rng.uniform(0, 2 * np.pi)) if kind == cg.RZ else 0.0))
        else:
            ar = cg.ARITY[kind]
            if m < ar:
                items.append((cg.H, pool[0]))
                continue
            t = pool[int(rng.integers(m))]
            src = [x for x in (order if wide else pool) if x != t]
            if len(src) < ar - 1:
                items.append((cg.H, t))
                continue
            cs = [int(c) for c in rng.choice(src, ar - 1, replace=False)]
            theta = float(rng.uniform(0, 2 * np.pi)) if kind == cg.CPHASE else 0.0
            items.append((kind, t, cs[0], cs[1] if ar > 2 else -1, theta))
    return cg.gates_from_list(items)


def lazy_state(M, dtype, mode=0, **kw):
    return q.State(M, dtype, q.make_options(exec_mode=mode, lazy_qubits=1, **kw))


def check(M, dtype, gates, em=None, k=0, mode=0, chunks=1):
    ref = oracle.simulate(M, gates, em, k=k)
    with lazy_state(M, dtype, mode) as s:
        s.reset(k)
        assert s.touched_qubits() == 0
        if em:
            s.inject_errors(em.sigma, em.p_bitflip, em.p_phaseflip, em.seed, em.trial)
        for part in np.array_split(np.arange(len(gates)), chunks):
            s.apply(gates[part])
        a = s.amplitudes()
        r = oracle.as_complex(ref)
        assert np.all(np.isfinite(a))
        err = float(np.max(np.abs(a - r)))
        assert err <= TOL[dtype], err
        touched = s.touched_qubits()
    return touched


@pytest.mark.parametrize("mode", [0, 2])
@pytest.mark.parametrize("dtype", [q.QSIM_C128, q.QSIM_C64])
@pytest.mark.parametrize("M,seed", [(14, 1), (17, 2)])
def test_late_touch_circuits_with_flips(mode, dtype, M, seed):
    print(f"lazy late-touch M={M} seed={seed} mode={mode} dtype={dtype}", flush=True)
    gates = late_touch_circuit(M, 240, seed)
    em = oracle.Errors(sigma=0.01, p_bitflip=0.01, p_phaseflip=0.01, seed=700 + seed, trial=3)
    check(M, dtype, gates, em, mode=mode)
    check(M, dtype, gates, None, mode=mode)


@pytest.mark.parametrize("dtype", [q.QSIM_C128, q.QSIM_C64])
def test_split_calls_basis_start_and_echo(dtype):
    """A circuit split over several calls (flipped untouched qubits are moved
    at every call's end), from a basis state with bits set, then undone by
    the inverse."""
    M = 16
    gates = late_touch_circuit(M, 300, 9, m0=3)
    em = oracle.Errors(sigma=0.02, p_bitflip=0.02, p_phaseflip=0.02, seed=909, trial=1)
    k = 0b1010_0110_0001_1101
    check(M, dtype, gates, em, k=k, chunks=5)
    with lazy_state(M, dtype) as s:
        s.reset(k)
        s.apply(gates)
        s.apply_inverse(gates)
        a = s.amplitudes()
        want = np.zeros(1 << M, complex)
        want[k] = 1.0
        assert np.max(np.abs(a - want)) <= 10 * TOL[dtype]


def test_untouched_qubits_cost_nothing_and_stay_exact():
    """The 7^A mod 15 circuit on the top 9 qubits of M = 30: every qubit below
    stays untouched, the passes span one tile, and the distribution is the
    exact one (permutation gates are exact swaps)."""
    M, a = 30, 5
    qm = list(range(M - 9, M))
    gates = np.concatenate([cg.modexp15_circuit(a, qubit_map=qm),
                            cg.qft_circuit(qm[:a])])
    with lazy_state(M, q.QSIM_C64) as s:
        s.profile(True)
        s.apply(gates)
        st = s.stats()
        touched = s.touched_qubits()
        assert touched & ((1 << (M - 9)) - 1) == 0
        pA = s.probs(sum(1 << qb for qb in qm[:a]))
        want = np.zeros(1 << a)
        want[::8] = 0.25
        assert np.max(np.abs(pA - want)) < 1e-6
        # bytes of the fused passes: one 2^13-amplitude tile each
        assert st["fused_bytes"] == st["fused_passes"] * 2 * 8 * (1 << 13)


@pytest.mark.parametrize("dtype", [q.QSIM_C128, q.QSIM_C64])
def test_lazy_equals_full_register_on_uniform_circuits(dtype):
    """Uniform random circuits touch every qubit within a few passes; the lazy
    register must agree with the oracle and with a register that streams
    every amplitude in every pass."""
    M = 18
    gates = cg.random_circuit(M, 400, 1818, kinds=(cg.H, cg.RZ, cg.CNOT, cg.TOFFOLI, cg.CPHASE))
    em = oracle.Errors(sigma=1e-3, p_bitflip=1e-3, p_phaseflip=1e-3, seed=1819, trial=0)
    touched = check(M, dtype, gates, em)
    assert touched == (1 << M) - 1
    with q.State(M, dtype, q.make_options(lazy_qubits=-1)) as f:
        assert f.touched_qubits() == (1 << M) - 1
        f.inject_errors(em.sigma, em.p_bitflip, em.p_phaseflip, em.seed, em.trial)
        f.apply(gates)
        r = oracle.as_complex(oracle.simulate(M, gates, em))
        assert np.max(np.abs(f.amplitudes() - r)) <= TOL[dtype]


def test_set_amplitudes_touches_everything_and_m34_register():
    M = 12
    with lazy_state(M, q.QSIM_C128) as s:
        v = cg.random_state(M, 4)
        v /= np.linalg.norm(v)
        s.set_amplitudes(v)
        assert s.touched_qubits() == (1 << M) - 1
        g = cg.random_circuit(M, 80, 4)
        s.apply(g)
        r = oracle.as_complex(oracle.run(v.copy(), M, g))
        assert np.max(np.abs(s.amplitudes() - r)) <= 1e-12
    # the largest register: a few gates on its low qubits cost one tile each
    M = 34
    gates = cg.gates_from_list([(cg.H, 0), (cg.CNOT, 1, 0), (cg.RZ, 33, -1, -1, 0.25),
                                (cg.X, 20), (cg.CNOT, 2, 20), (cg.CPHASE, 1, 2, -1, 0.5)])
    with lazy_state(M, q.QSIM_C64) as s:
        s.apply(gates)
        assert s.touched_qubits() == 0b11
        amp = s.amplitudes(0, 8)
        a20 = s.amplitudes(1 << 20, 8)
        h = float(np.float32(float.fromhex("0x1.6a09e667f3bcdp-1")))
        ph = np.exp(-0.125j)  # Rz(0.25) on |0> of qubit 33
        assert np.max(np.abs(amp)) == 0.0
        # X(20) and then CNOT(20 -> 2) flip untouched qubits 20 and 2 without
        # touching them; CPHASE(2 -> 1) then acts on qubit 1 alone
        assert abs(a20[4] - h * ph) < 1e-6 and abs(a20[7] - h * ph * np.exp(0.5j)) < 1e-6
        assert np.count_nonzero(a20) == 2
