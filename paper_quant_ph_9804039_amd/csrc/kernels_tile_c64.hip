// Fused tile pass, complex64 instantiation.
#include "tile_kernel.h"

namespace qsim {

size_t tile_lds_bytes(int k, int elem_bytes)
{
    return ((size_t)1 << k) * (size_t)elem_bytes;
}

template hipError_t launch_tile<float>(const TileArgs<float> &, int, hipStream_t);

}  // namespace qsim
