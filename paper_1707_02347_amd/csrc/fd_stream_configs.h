// fd_stream_configs.h -- compiled configurations per stencil radius M:
// X(M, T, PY, NW, MODE, F).  Owned region: 64 columns x NW*PY rows; output
// core: (64 - 2M(T-1)) columns x (NW*PY - 2M(T-1)) rows.  Every entry has an
// isotropic single-pass kernel; F adds the anisotropic form (bit 0) and the
// grouped batch kernel (bit 1) for the configurations the planner
// picks by default (other entries serve the tuner's search space).
#pragma once

#define FDW_A 1
#define FDW_G 2
#define FDW_AG 3

#define FDW_CONFIGS_M1(X)                                                                  \
    X(1, 1, 8, 4, 0, FDW_AG) X(1, 1, 4, 4, 0, FDW_AG) X(1, 1, 4, 8, 0, FDW_AG)             \
    X(1, 1, 16, 2, 0, 0) X(1, 1, 8, 4, 1, FDW_AG) X(1, 1, 8, 4, 2, FDW_AG)                 \
    X(1, 1, 4, 8, 1, FDW_AG) X(1, 1, 4, 8, 2, FDW_AG) X(1, 2, 4, 8, 0, FDW_AG)             \
    X(1, 2, 2, 16, 0, FDW_AG) X(1, 3, 4, 8, 0, FDW_G) X(1, 3, 2, 16, 0, FDW_G)              \
    X(1, 4, 4, 8, 0, 0) X(1, 4, 2, 16, 0, 0) X(1, 2, 4, 8, 1, FDW_G) X(1, 2, 4, 8, 2, FDW_G)             \
    X(1, 1, 4, 8, 3, FDW_A) X(1, 1, 4, 8, 4, FDW_A)

#define FDW_CONFIGS_M2(X)                                                                  \
    X(2, 1, 8, 4, 0, FDW_AG) X(2, 1, 4, 4, 0, FDW_AG) X(2, 1, 4, 8, 0, FDW_AG)             \
    X(2, 1, 16, 2, 0, 0) X(2, 1, 8, 4, 1, FDW_AG) X(2, 1, 8, 4, 2, FDW_AG)                 \
    X(2, 1, 4, 8, 1, FDW_AG) X(2, 1, 4, 8, 2, FDW_AG) X(2, 2, 4, 8, 0, FDW_AG)             \
    X(2, 2, 2, 16, 0, FDW_AG) X(2, 3, 4, 8, 0, FDW_G) X(2, 3, 2, 16, 0, FDW_G)              \
    X(2, 4, 2, 16, 0, 0) X(2, 2, 4, 8, 1, FDW_G) X(2, 2, 4, 8, 2, FDW_G) X(2, 1, 4, 8, 3, FDW_A)    \
    X(2, 1, 4, 8, 4, FDW_A)

#define FDW_CONFIGS_M3(X)                                                                  \
    X(3, 1, 8, 4, 0, FDW_AG) X(3, 1, 8, 4, 1, FDW_AG) X(3, 1, 8, 4, 2, FDW_AG)             \
    X(3, 1, 4, 8, 0, FDW_AG) X(3, 1, 4, 8, 1, FDW_AG) X(3, 1, 4, 8, 2, FDW_AG) X(3, 1, 4, 8, 3, FDW_A)  \
    X(3, 1, 4, 8, 4, FDW_A)
#define FDW_CONFIGS_M5(X)                                                                  \
    X(5, 1, 8, 4, 0, FDW_AG) X(5, 1, 8, 4, 1, FDW_AG) X(5, 1, 8, 4, 2, FDW_AG)             \
    X(5, 1, 4, 4, 0, FDW_AG) X(5, 1, 4, 4, 1, FDW_AG) X(5, 1, 4, 4, 2, FDW_AG) X(5, 1, 4, 4, 3, FDW_A)
#define FDW_CONFIGS_M6(X)                                                                  \
    X(6, 1, 8, 4, 0, FDW_AG) X(6, 1, 8, 4, 1, FDW_AG) X(6, 1, 8, 4, 2, FDW_AG)             \
    X(6, 1, 4, 4, 0, FDW_AG) X(6, 1, 4, 4, 1, FDW_AG) X(6, 1, 4, 4, 2, FDW_AG) X(6, 1, 4, 4, 3, FDW_A)
#define FDW_CONFIGS_M7(X)                                                                  \
    X(7, 1, 8, 4, 0, FDW_AG) X(7, 1, 8, 4, 1, FDW_AG) X(7, 1, 8, 4, 2, FDW_AG)             \
    X(7, 1, 4, 4, 0, FDW_AG) X(7, 1, 4, 4, 1, FDW_AG) X(7, 1, 4, 4, 2, FDW_AG) X(7, 1, 4, 4, 3, FDW_A)

#define FDW_CONFIGS_M4(X)                                                                  \
    X(4, 1, 8, 4, 0, FDW_AG) X(4, 1, 4, 4, 0, FDW_AG) X(4, 1, 16, 2, 0, 0)                 \
    X(4, 1, 8, 2, 0, 0) X(4, 1, 4, 8, 0, FDW_AG) X(4, 1, 2, 16, 0, 0) X(4, 1, 2, 8, 0, 0)  \
    X(4, 1, 8, 4, 1, FDW_G) X(4, 1, 8, 4, 2, FDW_A) X(4, 1, 4, 8, 1, FDW_AG)             \
    X(4, 1, 4, 8, 2, FDW_AG) X(4, 2, 4, 8, 0, FDW_A) X(4, 2, 2, 16, 0, FDW_AG)            \
    X(4, 3, 4, 8, 0, 0) X(4, 3, 2, 16, 0, 0)                      \
    X(4, 2, 4, 8, 1, FDW_G) X(4, 2, 4, 8, 2, FDW_G) X(4, 2, 2, 16, 1, FDW_G)              \
    X(4, 2, 2, 16, 2, 0) X(4, 1, 4, 8, 3, FDW_A) X(4, 1, 4, 8, 4, FDW_A) X(4, 1, 2, 8, 4, FDW_A)

#define FDW_CONFIGS_M8(X)                                                                  \
    X(8, 1, 8, 4, 0, FDW_AG) X(8, 1, 4, 4, 0, FDW_AG) X(8, 1, 8, 2, 0, 0)                  \
    X(8, 1, 4, 8, 0, FDW_AG) X(8, 1, 2, 16, 0, 0) X(8, 1, 8, 4, 1, FDW_AG)                 \
    X(8, 1, 8, 4, 2, FDW_AG) X(8, 1, 4, 4, 1, FDW_AG) X(8, 1, 4, 4, 2, FDW_AG)             \
    X(8, 2, 4, 8, 0, FDW_AG) X(8, 2, 4, 8, 1, FDW_G) X(8, 1, 4, 4, 3, FDW_A)

// Two-level passes without redundant halos (fd_wave.h): W(M, PY, NW), tiles of
// 64 columns x NW*PY rows; both Laplacian forms.
#define FDW_WAVE_CONFIGS(W)                                                                \
    W(1, 4, 4) W(1, 2, 8) W(2, 4, 4) W(2, 2, 8) W(3, 4, 4) W(3, 2, 8) W(4, 4, 4) W(4, 2, 8) \
    W(4, 2, 4) W(5, 2, 8) W(6, 2, 8) W(7, 2, 8) \
    W(8, 2, 8) W(8, 2, 4)
