// Host-side code of the library under AddressSanitizer / UBSan, no GPU:
// the lowering, the lazy-qubit rewrite, the pass scheduler and the kernel
// argument checks (qsim_plan), the Monte Carlo group schedule
// (qsim_trial_plan) and the argument checks of the other entry points, on
// seeded random circuits with errors.  Exit status 0 when every call returns
// the expected status; the sanitizers abort on the first memory or
// undefined-behaviour error.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "qsim.h"

namespace {

uint64_t g_rng = 0x9E3779B97F4A7C15ull;
uint32_t next_u32()
{
    g_rng = g_rng * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(g_rng >> 33);
}

std::vector<qsim_gate> random_circuit(int M, int G, bool cphase)
{
    std::vector<qsim_gate> out;
    const int kinds = cphase ? 7 : 6;
    for (int g = 0; g < G; ++g) {
        qsim_gate x{};
        x.kind = next_u32() % kinds;
        int need = (x.kind == QSIM_CNOT || x.kind == QSIM_CPHASE) ? 1 : x.kind == QSIM_TOFFOLI ? 2 : 0;
        if (M < need + 1)
            x.kind = QSIM_H, need = 0;
        int q[3];
        for (int i = 0; i <= need; ++i) {
            bool again;
            do {
                q[i] = (int)(next_u32() % (uint32_t)M);
                again = false;
                for (int j = 0; j < i; ++j)
                    again = again || q[j] == q[i];
            } while (again);
        }
        x.target = q[0];
        x.ctrl0 = need >= 1 ? q[1] : -1;
        x.ctrl1 = need >= 2 ? q[2] : -1;
        x.theta = (double)(next_u32() % 6283) * 1e-3;
        out.push_back(x);
    }
    return out;
}

int failures = 0;
void expect(int got, int want, const char *what)
{
    if (got != want) {
        std::printf("FAIL %s: status %d, expected %d (%s)\n", what, got, want, qsim_last_error());
        ++failures;
    }
}

}  // namespace

int main()
{
    const int sizes[] = {1, 2, 5, 9, 10, 13, 17, 24, 30, 34};
    for (int M : sizes) {
        for (int mode = 0; mode <= 2; ++mode) {
            for (int lazy = -1; lazy <= 1; lazy += 2) {
                for (int dtype = 0; dtype <= 1; ++dtype) {
                    std::vector<qsim_gate> g = random_circuit(M, 300, true);
                    qsim_options o{};
                    o.exec_mode = mode;
                    o.lazy_qubits = lazy;
                    o.renorm_period = 16;
                    qsim_error_model em{0.01, 0.01, 0.02, 7, (uint64_t)M};
                    size_t np = 0, nops = 0;
                    expect(qsim_plan(M, dtype, &o, g.data(), g.size(), &em, 3, nullptr, 0, &np,
                                     &nops, nullptr, 0), QSIM_OK, "plan sizes");
                    std::vector<qsim_pass_info> passes(np + 1);
                    std::vector<uint32_t> order(nops + 1);
                    expect(qsim_plan(M, dtype, &o, g.data(), g.size(), &em, 3, passes.data(), np, &np,
                                     &nops, order.data(), nops), QSIM_OK, "plan");
                }
            }
        }
    }
    // every tile shape the options allow
    for (int k = 9; k <= 14; ++k)
        for (int low = 1; low < k; low += 3)
            for (int G = 3; G <= 5; ++G) {
                qsim_options o{};
                o.tile_bits = k;
                o.low_bits = low;
                o.group_bits = G;
                std::vector<qsim_gate> g = random_circuit(20, 200, false);
                const int ok = (k - G >= 6 && k - G <= 9) ? QSIM_OK : QSIM_EINVAL;
                for (int dtype = 0; dtype <= 1; ++dtype) {
                    const int want = (dtype == 1 && k == 14) ? QSIM_EINVAL : ok;
                    expect(qsim_plan(20, dtype, &o, g.data(), g.size(), nullptr, 0, nullptr, 0,
                                     nullptr, nullptr, nullptr, 0), want, "tile shape");
                }
            }
    // Monte Carlo register-group schedule
    for (int M = 10; M <= 14; ++M)
        for (int G = 4; G <= 5; ++G) {
            if (M - G < 6)
                continue;
            std::vector<qsim_gate> g = random_circuit(M, 2000, false);
            size_t ng = 0;
            expect(qsim_trial_plan(g.data(), g.size(), M, G, nullptr, 0, &ng), QSIM_OK, "trial plan");
            std::vector<uint32_t> rec(4 * (ng + 1));
            expect(qsim_trial_plan(g.data(), g.size(), M, G, rec.data(), ng, &ng), QSIM_OK,
                   "trial plan records");
        }
    // argument checks that return before any device call
    qsim_state *s = nullptr;
    expect(qsim_create(0, QSIM_C64, nullptr, &s), QSIM_EINVAL, "create M=0");
    expect(qsim_create(35, QSIM_C64, nullptr, &s), QSIM_EINVAL, "create M=35");
    expect(qsim_create(10, 5, nullptr, &s), QSIM_EINVAL, "create dtype");
    expect(qsim_create(10, QSIM_C64, nullptr, nullptr), QSIM_EINVAL, "create out NULL");
    expect(qsim_apply_circuit(nullptr, nullptr, 0), QSIM_EINVAL, "apply NULL");
    qsim_gate bad{QSIM_CNOT, 1, 1, -1, 0.0};
    expect(qsim_plan(4, QSIM_C64, nullptr, &bad, 1, nullptr, 0, nullptr, 0, nullptr, nullptr,
                     nullptr, 0), QSIM_EINVAL, "plan bad gate");
    qsim_error_model nan_em{-1.0, 0.0, 0.0, 0, 0};
    std::vector<qsim_gate> g = random_circuit(12, 10, false);
    double F[4];
    expect(qsim_run_trials(g.data(), g.size(), 15, QSIM_C64, &nan_em, 4, F), QSIM_EINVAL,
           "trials M");
    expect(qsim_run_trials(g.data(), g.size(), 12, QSIM_C64, &nan_em, 4, F), QSIM_EINVAL,
           "trials model");
    qsim_request r{};
    r.num_qubits = 40;
    qsim_result res{};
    expect(qsim_serve(&r, 1, nullptr, &res), QSIM_EINVAL, "serve M");
    expect(qsim_overlap_noalloc(nullptr, 0, nullptr, 0, 0, 0, nullptr, F), QSIM_EINVAL,
           "noalloc M");
    std::printf("host driver: %d failure(s)\n", failures);
    return failures == 0 ? 0 : 1;
}
