/*
 * qsim oracle -- plain, slow, FP64 CPU reference of the error-injecting
 * state-vector simulator described by Obenland & Despain, "A Parallel Quantum
 * Computer Simulator" (arXiv quant-ph/9804039).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the CPU-baseline leg of the benchmark may load this library.  The GPU
 * library never calls it, and the two share no code, header or table: the
 * only common ground is the 24-byte gate record and the error-model fields,
 * which both sides define for themselves.
 *
 * Arithmetic is complex double written out as real operations, one gate at a
 * time, over the whole vector, in index order.  Build with -ffp-contract=off
 * so that every product and every sum is rounded on its own.  The pair loops
 * may run under OpenMP: every pair is independent, so the result does not
 * depend on the thread count.  Reductions (fidelity, probabilities) are
 * serial, in ascending index order.
 *
 * What it follows:
 *   state vector, index bits = qubit values ........ Sec. 1.2, Fig. 1
 *   a transformation = 2^M x 2^M matrix times vector  Sec. 1.3
 *   2x2 transform = V/2 independent pair transforms   Sec. 2.1, Fig. 3
 *   CNOT = swap of the amplitudes with control set    Sec. 1.3, Table 1, Fig. 2
 *   gate set: 1-, 2-, 3-bit controlled-NOT, rotations Sec. 2.0
 *   operational error = deviation of rotation angle   Sec. 1.4, Sec. 2.0
 *   decoherence = two extra transforms after each op  Sec. 3.4, EQ 8
 *   probability of a state = |amplitude|^2           Sec. 1.2
 *
 * Readings where the paper is silent (the same list is kept with the design
 * notes):
 *   - qubit q is index bit 2^q; with CNOT(control 1, target 0) on 2 qubits the
 *     amplitudes a2 and a3 swap, as in Fig. 2;
 *   - the superposition gate is the Hadamard, H = sqrt(1/2) [[1,1],[1,-1]];
 *   - Rz(theta) = diag(e^{-i theta/2}, e^{+i theta/2});
 *   - the controlled phase CPHASE(theta) multiplies the amplitudes whose
 *     control and target bits are both 1 by e^{i theta}: diag(1, e^{i theta})
 *     on the target where the control is set;
 *   - one angle error eps = sigma * z per gate (z standard normal); H, X,
 *     CNOT, Toffoli and Z are then i * R_n(pi + eps), with n the gate's own
 *     rotation axis, and Rz(theta) and CPHASE(theta) take theta + eps; with eps == 0
 *     every gate is its textbook form and X/CNOT/Toffoli/Z are exact swaps
 *     and sign flips;
 *   - decoherence after every gate: for each qubit q = 0..M-1 in turn, a
 *     bit flip X_q with probability p_bit, then a phase flip Z_q with
 *     probability p_phase, both exact;
 *   - random draws: Philox4x64-10 (Salmon et al., SC'11) with key
 *     (seed, trial) and counter (step, qubit, stream, 0); the angle draw uses
 *     counter (step, 0, 1, 0) and Box-Muller on the high 32 bits of output
 *     words 0 and 1; the flips of qubit q use counter (step, q, 2, 0): word 0
 *     decides the bit flip, word 1 the phase flip, firing when its high 32
 *     bits are below floor(p * 2^32);
 *   - fidelity F(a, b) = |<a|b>|^2 / (<a|a> <b|b>).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OQ_H = 0, OQ_RZ = 1, OQ_X = 2, OQ_CNOT = 3, OQ_TOFFOLI = 4, OQ_Z = 5, OQ_CPHASE = 6 };

typedef struct {
    uint32_t kind;
    int32_t target;
    int32_t ctrl0;
    int32_t ctrl1;
    double theta;
} oq_gate;

typedef struct {
    double sigma;        /* standard deviation of the per-gate angle error, radians */
    double p_bitflip;    /* per qubit per step */
    double p_phaseflip;  /* per qubit per step */
    uint64_t seed;
    uint64_t trial;
} oq_errors;

/* ------------------------------------------------------------------ draws */

/* Philox4x64-10, from the published description: ten rounds; each round
 * multiplies counter words 0 and 2 by the two round constants, and the new
 * counter is (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0));
 * the key is bumped by the two Weyl constants before every round but the
 * first. */
void oq_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw_block(const oq_errors *em, uint64_t step, uint64_t qubit, uint64_t stream,
                       uint64_t out[4])
{
    uint64_t key[2] = {em->seed, em->trial};
    uint64_t ctr[4] = {step, qubit, stream, 0};
    oq_philox4x64_10(ctr, key, out);
}

/* Standard normal deviate of a step: Box-Muller (1958) on two uniforms in
 * (0, 1) made from the high halves of words 0 and 1. */
double oq_gauss(const oq_errors *em, uint64_t step)
{
    uint64_t w[4];
    draw_block(em, step, 0, 1, w);
    double u1 = ((double)(w[0] >> 32) + 0.5) * 0x1p-32;
    double u2 = ((double)(w[1] >> 32) + 0.5) * 0x1p-32;
    const double two_pi = 6.283185307179586476925286766559;
    return sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
}

double oq_angle_error(const oq_errors *em, uint64_t step)
{
    if (em == NULL || em->sigma == 0.0)
        return 0.0;
    return em->sigma * oq_gauss(em, step);
}

static uint64_t flip_threshold(double p)
{
    return (uint64_t)floor(p * 4294967296.0);
}

/* Bit 0 of the result: bit flip fires; bit 1: phase flip fires. */
int oq_flip_events(const oq_errors *em, uint64_t step, int qubit)
{
    if (em == NULL || (em->p_bitflip == 0.0 && em->p_phaseflip == 0.0))
        return 0;
    uint64_t w[4];
    draw_block(em, step, (uint64_t)qubit, 2, w);
    int ev = 0;
    if ((w[0] >> 32) < flip_threshold(em->p_bitflip))
        ev |= 1;
    if ((w[1] >> 32) < flip_threshold(em->p_phaseflip))
        ev |= 2;
    return ev;
}

/* ------------------------------------------------------------ gate matrix */

/* The 2x2 that a gate applies to its target, as re/im pairs in the order
 * u00, u01, u10, u11.  Returns 0 for a general matrix, 1 when the gate is an
 * exact swap (X, CNOT, Toffoli with eps == 0) and 2 when it is an exact sign
 * flip of the |1> component (Z with eps == 0); u is filled in every case. */
int oq_gate_matrix(uint32_t kind, double theta, double eps, double u[8])
{
    const double h = 0x1.6a09e667f3bcdp-1; /* sqrt(1/2), correctly rounded */
    double c = cos(0.5 * eps), s = sin(0.5 * eps);
    memset(u, 0, 8 * sizeof(double));
    switch (kind) {
    case OQ_H:
        if (eps == 0.0) {
            u[0] = h; u[2] = h; u[4] = h; u[6] = -h;
        } else { /* -i s I + c H */
            u[0] = c * h; u[1] = -s;
            u[2] = c * h;
            u[4] = c * h;
            u[6] = -(c * h); u[7] = -s;
        }
        return 0;
    case OQ_RZ: {
        double phi = theta + eps;
        double cp = cos(0.5 * phi), sp = sin(0.5 * phi);
        u[0] = cp; u[1] = -sp;
        u[6] = cp; u[7] = sp;
        return 0;
    }
    case OQ_X:
    case OQ_CNOT:
    case OQ_TOFFOLI:
        if (eps == 0.0) {
            u[2] = 1.0; u[4] = 1.0;
            return 1;
        }
        /* -i s I + c X */
        u[1] = -s;
        u[2] = c;
        u[4] = c;
        u[7] = -s;
        return 0;
    case OQ_CPHASE: { /* diag(1, e^{i phi}); the control is applied by the caller */
        double phi = theta + eps;
        u[0] = 1.0;
        u[6] = cos(phi); u[7] = sin(phi);
        return 0;
    }
    case OQ_Z:
        if (eps == 0.0) {
            u[0] = 1.0; u[6] = -1.0;
            return 2;
        }
        /* -i s I + c Z */
        u[0] = c; u[1] = -s;
        u[6] = -c; u[7] = -s;
        return 0;
    default:
        return -1;
    }
}

/* ------------------------------------------------------------ transforms */

/* Sec. 2.1: for every index i with bit t clear and all control bits set,
 * (psi_i, psi_j) <- U (psi_i, psi_j) with j = i | 2^t. */
void oq_apply_matrix(double *psi, int M, int t, uint64_t cmask, const double u[8])
{
    const int64_t n = (int64_t)1 << M;
    const uint64_t tb = (uint64_t)1 << t;
#pragma omp parallel for schedule(static)
    for (int64_t ii = 0; ii < n; ++ii) {
        uint64_t i = (uint64_t)ii;
        if ((i & tb) != 0 || (i & cmask) != cmask)
            continue;
        uint64_t j = i | tb;
        double ar = psi[2 * i], ai = psi[2 * i + 1];
        double br = psi[2 * j], bi = psi[2 * j + 1];
        double xr = (u[0] * ar - u[1] * ai) + (u[2] * br - u[3] * bi);
        double xi = (u[0] * ai + u[1] * ar) + (u[2] * bi + u[3] * br);
        double yr = (u[4] * ar - u[5] * ai) + (u[6] * br - u[7] * bi);
        double yi = (u[4] * ai + u[5] * ar) + (u[6] * bi + u[7] * br);
        psi[2 * i] = xr; psi[2 * i + 1] = xi;
        psi[2 * j] = yr; psi[2 * j + 1] = yi;
    }
}

/* Table 1 / Fig. 2: a controlled NOT exchanges the two amplitudes. */
void oq_apply_swap(double *psi, int M, int t, uint64_t cmask)
{
    const int64_t n = (int64_t)1 << M;
    const uint64_t tb = (uint64_t)1 << t;
#pragma omp parallel for schedule(static)
    for (int64_t ii = 0; ii < n; ++ii) {
        uint64_t i = (uint64_t)ii;
        if ((i & tb) != 0 || (i & cmask) != cmask)
            continue;
        uint64_t j = i | tb;
        double r = psi[2 * i], im = psi[2 * i + 1];
        psi[2 * i] = psi[2 * j]; psi[2 * i + 1] = psi[2 * j + 1];
        psi[2 * j] = r; psi[2 * j + 1] = im;
    }
}

/* Z on qubit t: the amplitudes with bit t set change sign. */
void oq_apply_negate(double *psi, int M, int t, uint64_t cmask)
{
    const int64_t n = (int64_t)1 << M;
    const uint64_t tb = (uint64_t)1 << t;
#pragma omp parallel for schedule(static)
    for (int64_t ii = 0; ii < n; ++ii) {
        uint64_t i = (uint64_t)ii;
        if ((i & tb) == 0 || (i & cmask) != cmask)
            continue;
        psi[2 * i] = -psi[2 * i];
        psi[2 * i + 1] = -psi[2 * i + 1];
    }
}

/* Fig. 1(a): the basis state |k>. */
void oq_init(double *psi, int M, uint64_t k)
{
    const uint64_t n = (uint64_t)1 << M;
    memset(psi, 0, 2 * n * sizeof(double));
    psi[2 * k] = 1.0;
}

static int gate_valid(const oq_gate *g, int M)
{
    int need = (g->kind == OQ_CNOT || g->kind == OQ_CPHASE) ? 1 : (g->kind == OQ_TOFFOLI) ? 2 : 0;
    if (g->kind > OQ_CPHASE)
        return 0;
    if (g->target < 0 || g->target >= M)
        return 0;
    int have = (g->ctrl0 >= 0) + (g->ctrl1 >= 0);
    if (have != need || (need == 1 && g->ctrl0 < 0))
        return 0;
    if (g->ctrl0 >= M || g->ctrl1 >= M)
        return 0;
    if (g->ctrl0 >= 0 && g->ctrl0 == g->target)
        return 0;
    if (g->ctrl1 >= 0 && (g->ctrl1 == g->target || g->ctrl1 == g->ctrl0))
        return 0;
    if (!isfinite(g->theta))
        return 0;
    return 1;
}

/* Apply one gate of the circuit at global step `step`, then the decoherence
 * flips of that step (Sec. 3.4: two extra transformations after every
 * operation, read as a bit flip and a phase flip per qubit). */
static void apply_step(double *psi, int M, const oq_gate *g, const oq_errors *em, uint64_t step)
{
    double eps = oq_angle_error(em, step);
    uint64_t cmask = 0;
    if (g->ctrl0 >= 0)
        cmask |= (uint64_t)1 << g->ctrl0;
    if (g->ctrl1 >= 0)
        cmask |= (uint64_t)1 << g->ctrl1;
    double u[8];
    int form = oq_gate_matrix(g->kind, g->theta, eps, u);
    if (form == 1)
        oq_apply_swap(psi, M, g->target, cmask);
    else if (form == 2)
        oq_apply_negate(psi, M, g->target, cmask);
    else
        oq_apply_matrix(psi, M, g->target, cmask, u);
    if (em == NULL || (em->p_bitflip == 0.0 && em->p_phaseflip == 0.0))
        return;
    for (int q = 0; q < M; ++q) {
        int ev = oq_flip_events(em, step, q);
        if (ev & 1)
            oq_apply_swap(psi, M, q, 0);
        if (ev & 2)
            oq_apply_negate(psi, M, q, 0);
    }
}

/* Run gates g[0..n) on psi; gate k is step step0 + k.  em == NULL runs the
 * error-free circuit.  Returns 0, or -1 for an invalid gate or model (psi is
 * then untouched). */
int oq_run(double *psi, int M, const oq_gate *g, size_t n, const oq_errors *em, uint64_t step0)
{
    if (M < 1 || M > 34)
        return -1;
    for (size_t k = 0; k < n; ++k)
        if (!gate_valid(&g[k], M))
            return -1;
    if (em != NULL) {
        if (!(em->sigma >= 0.0) || !isfinite(em->sigma))
            return -1;
        if (!(em->p_bitflip >= 0.0 && em->p_bitflip <= 1.0))
            return -1;
        if (!(em->p_phaseflip >= 0.0 && em->p_phaseflip <= 1.0))
            return -1;
    }
    for (size_t k = 0; k < n; ++k)
        apply_step(psi, M, &g[k], em, step0 + k);
    return 0;
}

/* ------------------------------------------------------------ reductions */

typedef struct {
    double sum, comp;
} neumaier;

static void nm_add(neumaier *a, double x)
{
    double t = a->sum + x;
    if (fabs(a->sum) >= fabs(x))
        a->comp += (a->sum - t) + x;
    else
        a->comp += (x - t) + a->sum;
    a->sum = t;
}

static double nm_value(const neumaier *a) { return a->sum + a->comp; }

/* <a|b> = sum conj(a_i) b_i, <a|a> and <b|b>, each with compensated sums in
 * ascending index order.  out = {re <a|b>, im <a|b>, <a|a>, <b|b>}. */
void oq_overlap(const double *a, const double *b, int M, double out[4])
{
    const uint64_t n = (uint64_t)1 << M;
    neumaier re = {0, 0}, im = {0, 0}, na = {0, 0}, nb = {0, 0};
    for (uint64_t i = 0; i < n; ++i) {
        double ar = a[2 * i], ai = a[2 * i + 1], br = b[2 * i], bi = b[2 * i + 1];
        nm_add(&re, ar * br + ai * bi);
        nm_add(&im, ar * bi - ai * br);
        nm_add(&na, ar * ar + ai * ai);
        nm_add(&nb, br * br + bi * bi);
    }
    out[0] = nm_value(&re);
    out[1] = nm_value(&im);
    out[2] = nm_value(&na);
    out[3] = nm_value(&nb);
}

double oq_fidelity(const double *a, const double *b, int M)
{
    double o[4];
    oq_overlap(a, b, M, o);
    return (o[0] * o[0] + o[1] * o[1]) / (o[2] * o[3]);
}

/* Sec. 1.2: probability of index i is |psi_i|^2.  With a qubit mask of m
 * bits, out has 2^m entries; entry k sums the probabilities of every index
 * whose masked bits, read in ascending qubit order, spell k. */
void oq_probs(const double *psi, int M, uint64_t mask, double *out)
{
    const uint64_t n = (uint64_t)1 << M;
    int m = 0;
    for (int q = 0; q < M; ++q)
        m += (int)((mask >> q) & 1);
    memset(out, 0, ((size_t)1 << m) * sizeof(double));
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t k = 0;
        int pos = 0;
        for (int q = 0; q < M; ++q) {
            if ((mask >> q) & 1) {
                k |= ((i >> q) & 1) << pos;
                ++pos;
            }
        }
        out[k] += psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
    }
}

/* Monte Carlo trials: the error-free run from |0...0> is the reference; trial
 * t runs the same circuit from |0...0> with the error model keyed by
 * base->trial + t and scores F against the reference.  Returns 0 or -1. */
int oq_run_trials(const oq_gate *g, size_t n, int M, const oq_errors *base,
                  uint64_t n_trials, double *out_F)
{
    const size_t len = 2 * ((size_t)1 << M);
    double *ideal = (double *)malloc(len * sizeof(double));
    double *psi = (double *)malloc(len * sizeof(double));
    if (ideal == NULL || psi == NULL) {
        free(ideal);
        free(psi);
        return -1;
    }
    oq_init(ideal, M, 0);
    int rc = oq_run(ideal, M, g, n, NULL, 0);
    for (uint64_t t = 0; rc == 0 && t < n_trials; ++t) {
        oq_errors em = *base;
        em.trial = base->trial + t;
        oq_init(psi, M, 0);
        rc = oq_run(psi, M, g, n, &em, 0);
        if (rc == 0)
            out_F[t] = oq_fidelity(ideal, psi, M);
    }
    free(ideal);
    free(psi);
    return rc;
}

int oq_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the OpenMP pair loops from now on (n >= 1); used to time the
 * oracle on one core beside all of them.  The results do not depend on it. */
void oq_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
