/*
 * Three-state oracle -- plain FP64 CPU reference of the detailed model of
 * Obenland & Despain (arXiv quant-ph/9804039): each ion of the Cirac-Zoller
 * trap has the two levels of its QU-bit plus a third, temporary level used
 * inside controlled-not gates (Sec. 2.0), so M ions take 3^M states (Sec. 3.0,
 * 3.1) and one transformation is 3^(M-1) independent small operations, one
 * per group of states that differ only in the transformed ion.
 *
 * TEST INFRASTRUCTURE ONLY (see qsim_oracle.c): shares nothing with the GPU
 * library; only the gate record and the error-model fields are common ground.
 *
 * State index i = sum_q d_q 3^q with d_q in {0, 1, 2} the level of ion q.
 *
 * Readings (the paper names the scheme but not its pulses):
 *   - a laser transformation on ion q between levels a < b by angle theta
 *     with phase phi is exp(-i theta/2 (e^{i phi}|a><b| + e^{-i phi}|b><a|)),
 *     the third level untouched; a phase transformation multiplies levels
 *     a, b by e^{-i theta/2}, e^{+i theta/2} (on levels 0, 1: the Rz of the
 *     two-state model);
 *   - a transformation may be conditional on another ion being in a given
 *     level (the step that in the trap goes through the shared motional
 *     mode; here the control ion's temporary level carries it);
 *   - gates become transformations as follows (five for a CNOT, Sec. 2.0):
 *       X      = rot(01, pi, 0)
 *       H      = rot(01, pi/2, -pi/2) then rot(01, pi, 0)   (= -i H on 0, 1)
 *       Rz(t)  = phase(t)
 *       Z      = phase(pi)                                   (= -i Z on 0, 1)
 *       CNOT   = rot_t(01, pi/2, pi/2); rot_c(12, pi, 0);
 *                [c in 2] rot_t(12, 2 pi, 0); rot_c(12, pi, pi);
 *                rot_t(01, pi/2, -pi/2)                      (exactly CNOT)
 *       CPHASE(t) on (c, x) = phase_c(t/2); phase_x(t/2); CNOT(c, x);
 *                phase_x(-t/2); CNOT(c, x)                   (up to a global phase)
 *       Toffoli(c0, c1, x) = the textbook six-CNOT circuit with H on x and
 *                phases of +-pi/4                            (up to a global phase)
 *   - operational error: every transformation's angle deviates by
 *     eps = sigma z (Sec. 1.4, 2.0), z from Philox4x64-10 keyed by (seed,
 *     trial) at counter (step, k, 3, 0) for the k-th transformation of the
 *     gate at `step`, Box-Muller on the high halves of words 0 and 1;
 *   - decoherence after each gate (Sec. 3.4): per ion, a bit flip exchanges
 *     levels 0 and 1, a phase flip negates level 1, drawn as in the two-state
 *     model (counter (step, q, 2, 0)).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { Q3_H = 0, Q3_RZ = 1, Q3_X = 2, Q3_CNOT = 3, Q3_TOFFOLI = 4, Q3_Z = 5, Q3_CPHASE = 6 };
enum { P3_ROT = 0, P3_PHASE = 1 };

typedef struct {
    uint32_t kind;
    int32_t target, ctrl0, ctrl1;
    double theta;
} oq3_gate;

typedef struct {
    double sigma, p_bitflip, p_phaseflip;
    uint64_t seed, trial;
} oq3_errors;

/* One transformation of the detailed model. */
typedef struct {
    uint32_t kind;      /* P3_ROT or P3_PHASE */
    int32_t ion;        /* transformed ion */
    int32_t a, b;       /* levels of a rotation, a < b */
    int32_t cond_ion;   /* -1: unconditional */
    int32_t cond_level; /* level the condition ion must be in */
    double theta, phi;
} oq3_pulse;

void oq_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

static uint64_t pow3(int e)
{
    uint64_t p = 1;
    for (int i = 0; i < e; ++i)
        p *= 3;
    return p;
}

static int level_of(uint64_t i, uint64_t place) { return (int)((i / place) % 3); }

/* ---------------------------------------------------------------- lowering */

static size_t put(oq3_pulse *out, size_t cap, size_t n, uint32_t kind, int ion, int a, int b,
                  int ci, int cl, double theta, double phi)
{
    if (n < cap) {
        oq3_pulse p = {kind, ion, a, b, ci, cl, theta, phi};
        out[n] = p;
    }
    return n + 1;
}

static size_t lower_cnot(oq3_pulse *o, size_t cap, size_t n, int c, int x)
{
    const double pi = 3.14159265358979323846;
    n = put(o, cap, n, P3_ROT, x, 0, 1, -1, 0, pi / 2, pi / 2);
    n = put(o, cap, n, P3_ROT, c, 1, 2, -1, 0, pi, 0.0);
    n = put(o, cap, n, P3_ROT, x, 1, 2, c, 2, 2 * pi, 0.0);
    n = put(o, cap, n, P3_ROT, c, 1, 2, -1, 0, pi, pi);
    n = put(o, cap, n, P3_ROT, x, 0, 1, -1, 0, pi / 2, -pi / 2);
    return n;
}

static size_t lower_h(oq3_pulse *o, size_t cap, size_t n, int x)
{
    const double pi = 3.14159265358979323846;
    n = put(o, cap, n, P3_ROT, x, 0, 1, -1, 0, pi / 2, -pi / 2);
    n = put(o, cap, n, P3_ROT, x, 0, 1, -1, 0, pi, 0.0);
    return n;
}

static size_t phase(oq3_pulse *o, size_t cap, size_t n, int x, double t)
{
    return put(o, cap, n, P3_PHASE, x, 0, 1, -1, 0, t, 0.0);
}

/* Transformations of one gate into out[0 .. cap); returns how many the gate
 * takes (which may exceed cap). */
size_t oq3_lower_gate(const oq3_gate *g, oq3_pulse *out, size_t cap)
{
    const double pi = 3.14159265358979323846;
    size_t n = 0;
    const int x = g->target, c0 = g->ctrl0, c1 = g->ctrl1;
    switch (g->kind) {
    case Q3_X:
        n = put(out, cap, n, P3_ROT, x, 0, 1, -1, 0, pi, 0.0);
        break;
    case Q3_H:
        n = lower_h(out, cap, n, x);
        break;
    case Q3_RZ:
        n = phase(out, cap, n, x, g->theta);
        break;
    case Q3_Z:
        n = phase(out, cap, n, x, pi);
        break;
    case Q3_CNOT:
        n = lower_cnot(out, cap, n, c0, x);
        break;
    case Q3_CPHASE:
        n = phase(out, cap, n, c0, 0.5 * g->theta);
        n = phase(out, cap, n, x, 0.5 * g->theta);
        n = lower_cnot(out, cap, n, c0, x);
        n = phase(out, cap, n, x, -0.5 * g->theta);
        n = lower_cnot(out, cap, n, c0, x);
        break;
    default: /* Toffoli: controls c0, c1, target x */
        n = lower_h(out, cap, n, x);
        n = lower_cnot(out, cap, n, c1, x);
        n = phase(out, cap, n, x, -pi / 4);
        n = lower_cnot(out, cap, n, c0, x);
        n = phase(out, cap, n, x, pi / 4);
        n = lower_cnot(out, cap, n, c1, x);
        n = phase(out, cap, n, x, -pi / 4);
        n = lower_cnot(out, cap, n, c0, x);
        n = phase(out, cap, n, c1, pi / 4);
        n = phase(out, cap, n, x, pi / 4);
        n = lower_h(out, cap, n, x);
        n = lower_cnot(out, cap, n, c0, c1);
        n = phase(out, cap, n, c0, pi / 4);
        n = phase(out, cap, n, c1, -pi / 4);
        n = lower_cnot(out, cap, n, c0, c1);
        break;
    }
    return n;
}

/* ------------------------------------------------------------- transforms */

/* The 2x2 that a transformation applies to levels (a, b) of its ion, as
 * re/im pairs u00 u01 u10 u11 (a phase transformation is diagonal). */
void oq3_pulse_matrix(const oq3_pulse *p, double eps, double u[8])
{
    const double th = p->theta + eps;
    memset(u, 0, 8 * sizeof(double));
    if (p->kind == P3_PHASE) {
        u[0] = cos(0.5 * th); u[1] = -sin(0.5 * th);
        u[6] = cos(0.5 * th); u[7] = sin(0.5 * th);
        return;
    }
    const double c = cos(0.5 * th), s = sin(0.5 * th);
    /* -i s e^{i phi} = s sin(phi) - i s cos(phi) */
    u[0] = c;
    u[2] = s * sin(p->phi); u[3] = -s * cos(p->phi);
    u[4] = -s * sin(p->phi); u[5] = -s * cos(p->phi);
    u[6] = c;
}

/* One transformation over the whole 3^M vector: for every index i whose
 * transformed ion is in level a (and whose condition ion, if any, is in its
 * level), (psi_i, psi_j) <- U (psi_i, psi_j) with j the same index with the
 * ion in level b. */
void oq3_apply_pulse(double *psi, int M, const oq3_pulse *p, double eps)
{
    double u[8];
    oq3_pulse_matrix(p, eps, u);
    const uint64_t n = pow3(M), place = pow3(p->ion);
    const uint64_t cplace = p->cond_ion >= 0 ? pow3(p->cond_ion) : 1;
    const uint64_t step = (uint64_t)(p->b - p->a) * place;
#pragma omp parallel for schedule(static)
    for (int64_t ii = 0; ii < (int64_t)n; ++ii) {
        const uint64_t i = (uint64_t)ii;
        if (level_of(i, place) != p->a)
            continue;
        if (p->cond_ion >= 0 && level_of(i, cplace) != p->cond_level)
            continue;
        const uint64_t j = i + step;
        const double ar = psi[2 * i], ai = psi[2 * i + 1];
        const double br = psi[2 * j], bi = psi[2 * j + 1];
        psi[2 * i] = (u[0] * ar - u[1] * ai) + (u[2] * br - u[3] * bi);
        psi[2 * i + 1] = (u[0] * ai + u[1] * ar) + (u[2] * bi + u[3] * br);
        psi[2 * j] = (u[4] * ar - u[5] * ai) + (u[6] * br - u[7] * bi);
        psi[2 * j + 1] = (u[4] * ai + u[5] * ar) + (u[6] * bi + u[7] * br);
    }
}

/* Exact flips of ion q: exchange of levels 0 and 1, or sign of level 1. */
static void flip(double *psi, int M, int q, int phase_flip)
{
    const uint64_t n = pow3(M), place = pow3(q);
#pragma omp parallel for schedule(static)
    for (int64_t ii = 0; ii < (int64_t)n; ++ii) {
        const uint64_t i = (uint64_t)ii;
        const int d = level_of(i, place);
        if (phase_flip) {
            if (d == 1) {
                psi[2 * i] = -psi[2 * i];
                psi[2 * i + 1] = -psi[2 * i + 1];
            }
        } else if (d == 0) {
            const uint64_t j = i + place;
            const double r = psi[2 * i], im = psi[2 * i + 1];
            psi[2 * i] = psi[2 * j]; psi[2 * i + 1] = psi[2 * j + 1];
            psi[2 * j] = r; psi[2 * j + 1] = im;
        }
    }
}

void oq3_init(double *psi, int M, uint64_t k)
{
    memset(psi, 0, 2 * pow3(M) * sizeof(double));
    psi[2 * k] = 1.0;
}

static double pulse_eps(const oq3_errors *em, uint64_t step, uint64_t k)
{
    if (em == NULL || em->sigma == 0.0)
        return 0.0;
    uint64_t ctr[4] = {step, k, 3, 0}, key[2] = {em->seed, em->trial}, w[4];
    oq_philox4x64_10(ctr, key, w);
    const double u1 = ((double)(w[0] >> 32) + 0.5) * 0x1p-32;
    const double u2 = ((double)(w[1] >> 32) + 0.5) * 0x1p-32;
    return em->sigma * sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
}

static int gate_ok(const oq3_gate *g, int M)
{
    const int need = (g->kind == Q3_CNOT || g->kind == Q3_CPHASE) ? 1 : g->kind == Q3_TOFFOLI ? 2 : 0;
    if (g->kind > Q3_CPHASE || g->target < 0 || g->target >= M || !isfinite(g->theta))
        return 0;
    const int c[2] = {g->ctrl0, g->ctrl1};
    for (int i = 0; i < 2; ++i) {
        if (i >= need && c[i] != -1)
            return 0;
        if (i < need && (c[i] < 0 || c[i] >= M || c[i] == g->target))
            return 0;
    }
    return need < 2 || g->ctrl0 != g->ctrl1;
}

/* Run gates g[0..n): gate k is step step0 + k, lowered to transformations
 * each with its own angle error, then the step's flips.  0, or -1 for a bad
 * gate, model or size (psi untouched). */
int oq3_run(double *psi, int M, const oq3_gate *g, size_t n, const oq3_errors *em, uint64_t step0)
{
    if (M < 1 || M > 16)
        return -1;
    for (size_t k = 0; k < n; ++k)
        if (!gate_ok(&g[k], M))
            return -1;
    if (em != NULL && (!(em->sigma >= 0.0) || !isfinite(em->sigma) || !(em->p_bitflip >= 0.0) ||
                       em->p_bitflip > 1.0 || !(em->p_phaseflip >= 0.0) || em->p_phaseflip > 1.0))
        return -1;
    oq3_pulse pulses[64];
    for (size_t k = 0; k < n; ++k) {
        const uint64_t step = step0 + k;
        const size_t np = oq3_lower_gate(&g[k], pulses, 64);
        for (size_t j = 0; j < np; ++j)
            oq3_apply_pulse(psi, M, &pulses[j], pulse_eps(em, step, j));
        if (em == NULL || (em->p_bitflip == 0.0 && em->p_phaseflip == 0.0))
            continue;
        const uint64_t tb = (uint64_t)floor(em->p_bitflip * 4294967296.0);
        const uint64_t tp = (uint64_t)floor(em->p_phaseflip * 4294967296.0);
        for (int q = 0; q < M; ++q) {
            uint64_t ctr[4] = {step, (uint64_t)q, 2, 0}, key[2] = {em->seed, em->trial}, w[4];
            oq_philox4x64_10(ctr, key, w);
            if ((w[0] >> 32) < tb)
                flip(psi, M, q, 0);
            if ((w[1] >> 32) < tp)
                flip(psi, M, q, 1);
        }
    }
    return 0;
}

/* Probabilities |a_i|^2 summed over the ions outside `mask`; out has
 * 3^popcount(mask) entries, entry k spelling the masked ions' levels in
 * ascending ion order as base-3 digits. */
void oq3_probs(const double *psi, int M, uint64_t mask, double *out)
{
    int m = 0;
    for (int q = 0; q < M; ++q)
        m += (int)((mask >> q) & 1);
    memset(out, 0, pow3(m) * sizeof(double));
    const uint64_t n = pow3(M);
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t k = 0, kp = 1, rest = i;
        for (int q = 0; q < M; ++q) {
            const uint64_t d = rest % 3;
            rest /= 3;
            if ((mask >> q) & 1) {
                k += d * kp;
                kp *= 3;
            }
        }
        out[k] += psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
    }
}
