/* The FP64 oracle under AddressSanitizer / UBSan: seeded circuits with
 * errors on small registers, every readout, the Monte Carlo loop and the
 * rejection paths.  Exit status 0 when the results are sane (norm 1 within
 * 1e-12, fidelity in [0, 1]); the sanitizers abort on a memory or
 * undefined-behaviour error. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    uint32_t kind;
    int32_t target, ctrl0, ctrl1;
    double theta;
} gate;
typedef struct {
    double sigma, p_bitflip, p_phaseflip;
    uint64_t seed, trial;
} errors;

void oq_init(double *psi, int M, uint64_t k);
int oq_run(double *psi, int M, const gate *g, size_t n, const errors *em, uint64_t step0);
double oq_fidelity(const double *a, const double *b, int M);
void oq_probs(const double *psi, int M, uint64_t mask, double *out);
int oq_run_trials(const gate *g, size_t n, int M, const errors *base, uint64_t n_trials,
                  double *out_F);

static uint64_t rng = 12345;
static uint32_t next_u32(void)
{
    rng = rng * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(rng >> 33);
}

int main(void)
{
    int bad = 0;
    for (int M = 1; M <= 11; ++M) {
        size_t n = 150;
        gate *g = malloc(n * sizeof(gate));
        for (size_t i = 0; i < n; ++i) {
            uint32_t kind = next_u32() % 7;
            int need = (kind == 3 || kind == 6) ? 1 : kind == 4 ? 2 : 0;
            if (M < need + 1) {
                kind = 0;
                need = 0;
            }
            int q[3];
            for (int j = 0; j <= need; ++j) {
                int again;
                do {
                    q[j] = (int)(next_u32() % (uint32_t)M);
                    again = 0;
                    for (int k = 0; k < j; ++k)
                        again |= q[k] == q[j];
                } while (again);
            }
            g[i].kind = kind;
            g[i].target = q[0];
            g[i].ctrl0 = need >= 1 ? q[1] : -1;
            g[i].ctrl1 = need >= 2 ? q[2] : -1;
            g[i].theta = (double)(next_u32() % 6283) * 1e-3;
        }
        size_t len = 2 * ((size_t)1 << M);
        double *a = malloc(len * sizeof(double)), *b = malloc(len * sizeof(double));
        errors em = {0.05, 0.02, 0.02, 99, (uint64_t)M};
        oq_init(a, M, 0);
        oq_init(b, M, (uint64_t)1 << (M - 1));
        bad |= oq_run(a, M, g, n, NULL, 0) != 0;
        bad |= oq_run(b, M, g, n, &em, 5) != 0;
        double norm = 0.0;
        for (size_t i = 0; i < len; ++i)
            norm += b[i] * b[i];
        bad |= fabs(norm - 1.0) > 1e-12;
        double F = oq_fidelity(a, b, M);
        bad |= !(F >= 0.0 && F <= 1.0 + 1e-12);
        double *p = malloc(((size_t)1 << M) * sizeof(double));
        oq_probs(b, M, ((uint64_t)1 << M) - 1, p);
        oq_probs(b, M, 1, p);
        double Ft[3];
        bad |= oq_run_trials(g, n, M, &em, 3, Ft) != 0;
        gate wrong = {3, 0, 0, -1, 0.0};
        bad |= oq_run(a, M, &wrong, 1, NULL, 0) != -1;
        free(p);
        free(a);
        free(b);
        free(g);
    }
    printf("oracle driver: %s\n", bad ? "FAILED" : "ok");
    return bad;
}
