// Instantiations of the streaming / time-blocked kernels for stencil radius M = 8.
#include "fd_stream.h"
#include "fd_stream_configs.h"

namespace fdw {

template <int M, int T, int PY, int NW, int MODE>
static void launch_one(const SweepArgs &a, hipStream_t s)
{
    const dim3 grid(a.ntz * a.nty * a.ntx), block(64 * NW);
    if (a.w.iso) hipLaunchKernelGGL((k_stream<M, T, PY, NW, MODE, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_stream<M, T, PY, NW, MODE, false>), grid, block, 0, s, a);
}

#define FDW_LAUNCH_CASE(M_, T_, PY_, NW_, MODE_)                                          \
    if (k.T == T_ && k.PY == PY_ && k.NW == NW_ && k.mode == MODE_) {                     \
        launch_one<M_, T_, PY_, NW_, MODE_>(a, s);                                       \
        return true;                                                                     \
    }
#define FDW_HAS_CASE(M_, T_, PY_, NW_, MODE_)                                             \
    if (k.T == T_ && k.PY == PY_ && k.NW == NW_ && k.mode == MODE_) return true;

bool launch_stream_m8(const KernelKey &k, const SweepArgs &a, hipStream_t s)
{
    FDW_CONFIGS_M8(FDW_LAUNCH_CASE)
    return false;
}

bool has_stream_m8(const KernelKey &k)
{
    FDW_CONFIGS_M8(FDW_HAS_CASE)
    return false;
}

}  // namespace fdw
