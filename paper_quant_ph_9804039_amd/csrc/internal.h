// Helpers the C-ABI entry points share across source files.
#pragma once

#include <cstddef>

#include "qsim.h"

namespace qsim {

// Record a message for qsim_last_error (per thread) and return `code`.
int set_error(int code, const char *fmt, ...);

// Kind, arity and qubit checks of one gate on an M-qubit register; `why`
// receives the reason when the gate is rejected.
bool gate_valid(const qsim_gate &g, int M, char *why, size_t n);

// sigma finite and >= 0, both p in [0, 1].
bool error_model_valid(const qsim_error_model &em);

}  // namespace qsim
