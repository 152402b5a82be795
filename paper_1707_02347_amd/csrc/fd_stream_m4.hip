// Instantiations of the streaming / time-blocked kernels for stencil radius M = 4.
#include "fd_stream.h"
#include "fd_stream_configs.h"

namespace fdw {

template <int M, int T, int PY, int NW, int MODE>
static void launch_one(const SweepArgs &a, hipStream_t s)
{
    const int total = a.ntz * a.nty * a.ntx;
    const dim3 grid(total), block(64 * NW);
    const GroupEntry *none = nullptr;
    if (a.w.iso)
        hipLaunchKernelGGL((k_stream<M, T, PY, NW, MODE, true>), grid, block, 0, s, a, none, 0, total);
    else
        hipLaunchKernelGGL((k_stream<M, T, PY, NW, MODE, false>), grid, block, 0, s, a, none, 0, total);
}

template <int M, int T, int PY, int NW, int MODE>
static void launch_group(bool iso, const GroupEntry *list, int nlist, int total, int grid,
                         hipStream_t s)
{
    SweepArgs unused{};
    const dim3 g(grid), block(64 * NW);
    if (iso)
        hipLaunchKernelGGL((k_stream<M, T, PY, NW, MODE, true>), g, block, 0, s, unused, list, nlist,
                           total);
    else
        hipLaunchKernelGGL((k_stream<M, T, PY, NW, MODE, false>), g, block, 0, s, unused, list, nlist,
                           total);
}

template <int M, int T, int PY, int NW, int MODE>
static int occupancy(bool iso)
{
    int n = 0;
    hipError_t e;
    if (iso)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, reinterpret_cast<const void *>(&k_stream<M, T, PY, NW, MODE, true>), 64 * NW, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, reinterpret_cast<const void *>(&k_stream<M, T, PY, NW, MODE, false>), 64 * NW, 0);
    return e == hipSuccess ? n : 0;
}

#define FDW_MATCH(T_, PY_, NW_, MODE_) (k.T == T_ && k.PY == PY_ && k.NW == NW_ && k.mode == MODE_)
#define FDW_LAUNCH_CASE(M_, T_, PY_, NW_, MODE_)                                          \
    if (FDW_MATCH(T_, PY_, NW_, MODE_)) {                                                 \
        launch_one<M_, T_, PY_, NW_, MODE_>(a, s);                                       \
        return true;                                                                     \
    }
#define FDW_GROUP_CASE(M_, T_, PY_, NW_, MODE_)                                           \
    if (FDW_MATCH(T_, PY_, NW_, MODE_)) {                                                 \
        launch_group<M_, T_, PY_, NW_, MODE_>(iso, list, nlist, total, grid, s);         \
        return true;                                                                     \
    }
#define FDW_OCC_CASE(M_, T_, PY_, NW_, MODE_)                                             \
    if (FDW_MATCH(T_, PY_, NW_, MODE_)) return occupancy<M_, T_, PY_, NW_, MODE_>(iso);
#define FDW_HAS_CASE(M_, T_, PY_, NW_, MODE_)                                             \
    if (FDW_MATCH(T_, PY_, NW_, MODE_)) return true;

bool launch_stream_m4(const KernelKey &k, const SweepArgs &a, hipStream_t s)
{
    FDW_CONFIGS_M4(FDW_LAUNCH_CASE)
    return false;
}

bool launch_group_m4(const KernelKey &k, bool iso, const GroupEntry *list, int nlist, int total,
                     int grid, hipStream_t s)
{
    FDW_CONFIGS_M4(FDW_GROUP_CASE)
    return false;
}

int occupancy_m4(const KernelKey &k, bool iso)
{
    FDW_CONFIGS_M4(FDW_OCC_CASE)
    return 0;
}

bool has_stream_m4(const KernelKey &k)
{
    FDW_CONFIGS_M4(FDW_HAS_CASE)
    return false;
}

}  // namespace fdw
