// fd_stream_entry.h -- registry of compiled streaming-kernel configurations.
// One entry per X(...) line of fd_stream_configs.h; the entries and the
// registry are generated at build time (build.py), one source file per entry.
#pragma once

#include "fd_internal.h"

namespace fdw {

struct StreamEntry {
    int M, T, PY, NW, mode, flags;  // flags: bit 0 anisotropic form, bit 1 grouped kernel
    bool (*launch)(const SweepArgs &a, hipStream_t s);
    bool (*launch_group)(bool iso, bool ntl, bool ps, const GroupEntry *list, int nlist, int total,
                         int grid, hipStream_t s);
    int (*occupancy)(bool iso, bool grouped);
};

// All compiled entries (generated).
const StreamEntry *const *stream_registry(int *count);

// Two-level passes without redundant halos: one entry per W(...) line of
// fd_stream_configs.h (both Laplacian forms).
struct WaveEntry {
    int M, PY, NW;
    bool (*launch)(const SweepArgs &a, hipStream_t s);
    int (*occupancy)(bool iso);
};
const WaveEntry *const *wave_registry(int *count);

}  // namespace fdw
