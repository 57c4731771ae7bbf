// Helpers the C-ABI entry points share across source files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <exception>
#include <new>

#include "qsim.h"

namespace qsim {

// Record a message for qsim_last_error (per thread) and return `code`.
// Allocates nothing.
int set_error(int code, const char *fmt, ...);

// Run the body of an exported function so that no C++ exception crosses the
// C-ABI: host memory exhaustion becomes QSIM_ENOMEM, any other exception
// QSIM_EDEVICE, each with a message naming the function.
template <typename F>
int guarded(const char *fn, F &&body) noexcept
{
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return set_error(QSIM_ENOMEM, "%s: host memory exhausted", fn);
    } catch (const std::exception &e) {
        return set_error(QSIM_EDEVICE, "%s: internal error: %s", fn, e.what());
    } catch (...) {
        return set_error(QSIM_EDEVICE, "%s: internal error", fn);
    }
}

// Kind, arity and qubit checks of one gate on an M-qubit register; `why`
// receives the reason when the gate is rejected.
bool gate_valid(const qsim_gate &g, int M, char *why, size_t n);

// sigma finite and >= 0, both p in [0, 1].
bool error_model_valid(const qsim_error_model &em);

// Serving slots: a state whose scratch buffers fit registers of up to
// max_qubits, on a borrowed stream, rebound to borrowed memory per request
// (so the serving loop never allocates or frees on its hot path).
int slot_state_create(int device, hipStream_t st, int max_qubits, qsim_state **out);
int slot_state_bind(qsim_state *s, int num_qubits, int dtype, void *psi);
void slot_state_destroy(qsim_state *s);
// Enqueue <a|b>, <a|a>, <b|b> on a's stream and an async copy of the four
// doubles to pinned host memory (no synchronisation).
int overlap_enqueue(const qsim_state *a, const qsim_state *b, double *host_out4);

}  // namespace qsim
