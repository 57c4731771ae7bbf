// Device-side entry points of the library replaced by stubs for the host-only
// sanitizer build: the host driver never launches a kernel (it has no GPU),
// so every launcher reports hipErrorInvalidValue.  tile_lds_bytes is a size
// the option checks use, so it keeps its value (one element per tile
// amplitude).
#include "launch.h"
#include "qsim.h"

namespace qsim {

size_t tile_lds_bytes(int k, int elem_bytes) { return ((size_t)1 << k) * (size_t)elem_bytes; }

template <typename R>
hipError_t launch_init_basis(cplx<R> *, int, uint64_t, hipStream_t) { return hipErrorInvalidValue; }
template <typename R>
hipError_t launch_plain(const Op &, cplx<R> *, int, hipStream_t) { return hipErrorInvalidValue; }
template <typename R>
hipError_t launch_scale(cplx<R> *, int, const double *, hipStream_t) { return hipErrorInvalidValue; }
template <typename R>
hipError_t launch_tile(const TileArgs<R> &, int, hipStream_t) { return hipErrorInvalidValue; }
template <typename Ra, typename Rb>
hipError_t launch_overlap(const cplx<Ra> *, const cplx<Rb> *, int, double *, double *, hipStream_t)
{
    return hipErrorInvalidValue;
}
template <typename R>
hipError_t launch_norm(const cplx<R> *, int, double *, double *, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_finish_norm(const double *, uint64_t, double *, double *, hipStream_t)
{
    return hipErrorInvalidValue;
}
template <typename R>
hipError_t launch_probs_full(const cplx<R> *, int, double *, hipStream_t) { return hipErrorInvalidValue; }
template <typename R>
hipError_t launch_probs_marginal(const cplx<R> *, int, uint64_t, double *, uint64_t, double *, hipStream_t)
{
    return hipErrorInvalidValue;
}
uint64_t probs_marginal_partial_len(int, uint64_t) { return 1; }
template <typename R>
hipError_t launch_to_f64(const cplx<R> *, uint64_t, double *, hipStream_t) { return hipErrorInvalidValue; }
template <typename R>
hipError_t launch_from_f64(const double *, uint64_t, cplx<R> *, hipStream_t) { return hipErrorInvalidValue; }
size_t trial_gate_op_bytes(int elem_bytes) { return elem_bytes == 8 ? 64 : 96; }
size_t trial_lds_bytes(int, int) { return 0; }
int trial_group_bits(int variant) { return variant == 2 ? 4 : variant == 3 ? 5 : 0; }
template <typename R>
hipError_t launch_trials(const TrialLaunch &, hipStream_t) { return hipErrorInvalidValue; }
int trial_variants() { return 4; }
const char *trial_variant_name(int) { return "stub"; }
int trial_grid(int, int, int) { return 0; }

#define QSIM_STUBS(R)                                                                          \
    template hipError_t launch_init_basis<R>(cplx<R> *, int, uint64_t, hipStream_t);           \
    template hipError_t launch_plain<R>(const Op &, cplx<R> *, int, hipStream_t);              \
    template hipError_t launch_scale<R>(cplx<R> *, int, const double *, hipStream_t);          \
    template hipError_t launch_tile<R>(const TileArgs<R> &, int, hipStream_t);                 \
    template hipError_t launch_norm<R>(const cplx<R> *, int, double *, double *, hipStream_t); \
    template hipError_t launch_probs_full<R>(const cplx<R> *, int, double *, hipStream_t);     \
    template hipError_t launch_probs_marginal<R>(const cplx<R> *, int, uint64_t, double *,     \
                                                 uint64_t, double *, hipStream_t);             \
    template hipError_t launch_to_f64<R>(const cplx<R> *, uint64_t, double *, hipStream_t);    \
    template hipError_t launch_from_f64<R>(const double *, uint64_t, cplx<R> *, hipStream_t);  \
    template hipError_t launch_trials<R>(const TrialLaunch &, hipStream_t);
QSIM_STUBS(float)
QSIM_STUBS(double)
template hipError_t launch_overlap<float, float>(const cplx<float> *, const cplx<float> *, int,
                                                 double *, double *, hipStream_t);
template hipError_t launch_overlap<float, double>(const cplx<float> *, const cplx<double> *, int,
                                                  double *, double *, hipStream_t);
template hipError_t launch_overlap<double, float>(const cplx<double> *, const cplx<float> *, int,
                                                  double *, double *, hipStream_t);
template hipError_t launch_overlap<double, double>(const cplx<double> *, const cplx<double> *,
                                                   int, double *, double *, hipStream_t);

}  // namespace qsim

// the no-allocation readout lives with its device array in a HIP source
extern "C" int qsim_overlap_noalloc(const void *, int, const void *, int, int, int, void *, double *)
{
    return QSIM_EINVAL;
}
