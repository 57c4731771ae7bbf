// Fused tile pass, complex128 instantiation.
#include "tile_kernel.h"

namespace qsim {

template hipError_t launch_tile<double>(const TileArgs<double> &, int, hipStream_t);

}  // namespace qsim
