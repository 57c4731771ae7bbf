// Batched Monte Carlo trials entry point.
#include "qsim.h"

extern "C" int qsim_run_trials(const qsim_gate *, size_t, int, int, const qsim_error_model *,
                               uint64_t, double *)
{
    return QSIM_EINVAL;
}
