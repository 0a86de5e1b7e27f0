// fused_c64h.hip -- Hermitian complex64 instantiations of the single-launch
// schedules (fused.hpp: decomposition and reconstruction), in a translation unit of their own so they compile
// in parallel with the others.
#include "fused.hpp"

namespace ptd {

hipError_t fused_launch_c64_herm(int n, const void* A, int64_t lda, void* out, void* ws, int la, int cfg, bool unscaled,
                           hipStream_t st)
{
    return fused::fused_dispatch<float, true>(n, A, lda, out, ws, la, cfg, unscaled, st);
}

hipError_t fused_rec_c64_herm(int n, const void* coeff, void* A, int64_t lda, void* ws, int la, bool adjoint, hipStream_t st)
{
    return fused::fused_rec_dispatch<float, true>(n, coeff, A, lda, ws, la, adjoint, st);
}

}  // namespace ptd
