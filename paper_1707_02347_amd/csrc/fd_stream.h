// fd_stream.h -- streaming (space-tiled, T = 1) and time-blocked (T >= 2)
// stencil kernels for gfx950.
//
// Each workgroup owns a (y, z) tile and streams the x axis (the slowest axis)
// over a chunk of planes.  Lanes of a wave64 map to consecutive z (the
// contiguous axis, so every plane row is one coalesced 256-byte access); each
// thread holds PY consecutive rows in y.  Along x every thread keeps, per time
// level, a register queue of the 2M+1 planes its stencil needs; y and z
// neighbours come from an LDS copy of the current plane.
//
// Time blocking (paper Secs. 5.2-5.4): the update at level t needs level t-1
// within distance M in x, y and z, so level t is evaluated M planes behind
// level t-1 (the skew by the stencil radius that makes the dependence vectors
// non-negative, Sec. 5.2), and on a (y, z) region that shrinks by M per level
// (overlapped tiles).  One pass therefore reads u^n, u^{n-1} and q once and
// writes u^{n+T}, u^{n+T-1}: 20 bytes per point per T steps instead of 16 per
// step.  The paper's CPU code skews x and y and tiles (x, y, t) with a time tile
// bounded by the modulo buffer (Sec. 6.3.2); on the GPU the time tile lives in
// registers and LDS instead of a modulo-indexed array.
//
// The per-point FP32 operation order is the one fixed by the untiled kernel
// (fd_naive.hip), so every configuration returns bit-identical results.
#pragma once

#include "fd_internal.h"

namespace fdw {

template <int M_, int T_, int PY_, int NW_>
struct Geo {
    static constexpr int M = M_, T = T_, PY = PY_, NW = NW_;
    static constexpr int NT = 64 * NW;           // threads per workgroup
    static constexpr int RY = NW * PY;           // rows of the owned region (level 1)
    static constexpr int RZ = 64;                // columns of the owned region
    static constexpr int H1 = M * (T - 1);       // owned-region margin around the core
    static constexpr int TY = RY - 2 * H1;       // core (output) rows
    static constexpr int TZ = RZ - 2 * H1;       // core (output) columns
    static constexpr int L0H = RY + 2 * M;       // level-0 LDS plane (owned region + halo M)
    static constexpr int L0W = RZ + 2 * M;
    static constexpr int Q = 2 * M + 1;          // register queue length along x
    static constexpr int NHALO = 2 * M * L0W + RY * 2 * M;
    static constexpr int HS = (NHALO + NT - 1) / NT;
    static constexpr int AQ = (T - 1) * M + 1;   // imaging accumulator queue length
    static_assert(TY >= 1 && TZ >= 1, "core tile must be non-empty");
};

template <int M, int T, int PY, int NW, int MODE>
struct StreamKernel {
    using G = Geo<M, T, PY, NW>;

    // Level-0 plane with its M-wide halo ring; planes of levels 1..T-1 over the
    // owned region, padded by M rows above and below so that the rows a thread
    // reads next to its own (used only where they lie inside the level's
    // region) always stay inside the buffer.
    struct Smem {
        float s0[2][G::L0H * G::L0W];
        float s1[(T > 1) ? (T - 1) : 1][2][(T > 1) ? (G::RY + 2 * M) * G::RZ : 1];
    };

    __device__ static void run(const SweepArgs &a, Smem &sm)
    {
        // -------- tile decode (optionally XCD-aware: consecutive tiles on one XCD)
        int bid = blockIdx.x;
        const int ntiles = gridDim.x;
        if (a.remap && (ntiles & 7) == 0) {
            const int per = ntiles >> 3;
            bid = (bid & 7) * per + (bid >> 3);
        }
        const int bz = bid % a.ntz;
        const int rest = bid / a.ntz;
        const int by = rest % a.nty;
        const int bx = rest / a.nty;
        const int z1 = bz * G::TZ - G::H1;
        const int y1 = by * G::TY - G::H1;
        const int x0 = bx * a.lx;
        const int xend = min(x0 + a.lx, a.nx);

        const int lane = threadIdx.x & 63;
        const int wv = threadIdx.x >> 6;
        const int z = z1 + lane;
        const bool zin = (unsigned)z < (unsigned)a.nz;
        const float pzv = zin ? a.pz[z] : 0.0f;

        int32_t yz[PY];
        bool din[PY];      // point inside the grid (y and z)
        float pyz[PY];     // py[y] + pz[z]
        bool core[PY];     // inside the output tile (and the grid)
#pragma unroll
        for (int r = 0; r < PY; ++r) {
            const int rr = wv * PY + r;
            const int y = y1 + rr;
            const bool yin = (unsigned)y < (unsigned)a.ny;
            din[r] = yin && zin;
            yz[r] = y * a.nz + z;
            pyz[r] = din[r] ? (a.py[y] + pzv) : 0.0f;
            core[r] = din[r] && rr >= G::H1 && rr < G::RY - G::H1 && lane >= G::H1 &&
                      lane < G::RZ - G::H1;
        }

        // -------- halo ring of the level-0 plane (positions fixed for the whole pass)
        int32_t hg[G::HS];  // in-plane global offset, -1 if outside the grid or unused
#pragma unroll
        for (int s = 0; s < G::HS; ++s) {
            const int h = threadIdx.x + s * G::NT;
            int row = 0, col = 0;
            bool used = h < G::NHALO;
            if (h < 2 * M * G::L0W) {
                const int band = h / G::L0W;
                col = h - band * G::L0W;
                row = band < M ? band : band + G::RY;
            } else {
                const int h2 = h - 2 * M * G::L0W;
                row = M + h2 / (2 * M);
                const int cj = h2 % (2 * M);
                col = cj < M ? cj : cj + G::RZ;
            }
            const int gy = y1 - M + row, gz = z1 - M + col;
            hg[s] = (used && (unsigned)gy < (unsigned)a.ny && (unsigned)gz < (unsigned)a.nz)
                        ? gy * a.nz + gz
                        : -1;
        }

        float qu[T][PY][G::Q];  // level t's queue of u^{t-1}: planes c_t - M .. c_t + M
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int r = 0; r < PY; ++r)
#pragma unroll
                for (int j = 0; j < G::Q; ++j) qu[t][r][j] = 0.0f;

        double acc[(MODE == kImaging) ? PY : 1][(MODE == kImaging) ? G::AQ : 1];
        if constexpr (MODE == kImaging) {
#pragma unroll
            for (int r = 0; r < PY; ++r)
#pragma unroll
                for (int j = 0; j < G::AQ; ++j) acc[r][j] = 0.0;
        }

        const int ibeg = x0 - T * M;
        const int iend = xend + T * M;
        const int64_t N = (int64_t)a.nx * a.sxy;

        // Every global load of an iteration is issued one iteration ahead: the
        // head plane i of u^n, the level-0 halo ring and u^{n-1} at plane i - M,
        // and q at each level's plane i - t M.  A load is skipped (value 0) when
        // its plane is outside the grid or outside the planes the level needs.
        Pre nx_;
        load(a, nx_, ibeg, x0, xend, yz, din, hg);
        for (int i = ibeg; i < iend; ++i) {
            const int par = i & 1;
            Pre cur = nx_;
            if (i + 1 < iend) load(a, nx_, i + 1, x0, xend, yz, din, hg);
            if constexpr (MODE == kImaging) {
#pragma unroll
                for (int r = 0; r < PY; ++r)
#pragma unroll
                    for (int j = 0; j + 1 < G::AQ; ++j) acc[r][j] = acc[r][j + 1];
            }
            float val[PY];  // value produced by the previous level in this iteration
#pragma unroll
            for (int r = 0; r < PY; ++r) val[r] = cur.head[r];
            level<1>(a, sm, qu, acc, val, cur, i, par, x0, xend, N, lane, wv, yz, din, pyz, core);
        }
    }

    struct Pre {
        float head[PY];
        float halo[G::HS];
        float up1[PY];
        float q[T][PY];
    };

    // Planes level t must produce: [x0 - (T - t) M, xend + (T - t) M) within the grid.
    __device__ static __forceinline__ bool needed(const SweepArgs &a, int t, int c, int x0, int xend)
    {
        return (unsigned)c < (unsigned)a.nx && c >= x0 - (T - t) * M && c < xend + (T - t) * M;
    }

    __device__ static __forceinline__ void load(const SweepArgs &a, Pre &P, int i, int x0, int xend,
                                                const int32_t (&yz)[PY], const bool (&din)[PY],
                                                const int32_t (&hg)[G::HS])
    {
        const bool hin = (unsigned)i < (unsigned)a.nx;
        const float *hp = a.u0 + (int64_t)(hin ? i : 0) * a.sxy;
#pragma unroll
        for (int r = 0; r < PY; ++r) P.head[r] = (hin && din[r]) ? hp[yz[r]] : 0.0f;
        const int c1 = i - M;
        const bool l1 = needed(a, 1, c1, x0, xend);
        const bool cin = (unsigned)c1 < (unsigned)a.nx;
        const float *cp = a.u0 + (int64_t)(cin ? c1 : 0) * a.sxy;
#pragma unroll
        for (int s = 0; s < G::HS; ++s) P.halo[s] = (l1 && hg[s] >= 0) ? cp[hg[s]] : 0.0f;
        const float *mp = a.um + (int64_t)(cin ? c1 : 0) * a.sxy;
#pragma unroll
        for (int r = 0; r < PY; ++r) P.up1[r] = (l1 && din[r]) ? mp[yz[r]] : 0.0f;
#pragma unroll
        for (int t = 1; t <= T; ++t) {
            const int ct = i - t * M;
            const bool lt = needed(a, t, ct, x0, xend);
            const float *qp = a.q + (int64_t)(lt ? ct : 0) * a.sxy;
#pragma unroll
            for (int r = 0; r < PY; ++r) P.q[t - 1][r] = (lt && din[r]) ? qp[yz[r]] : 0.0f;
        }
    }

    // Process level t (1..T) at plane c = i - t*M, then recurse to level t+1.
    template <int t, class QU, class ACC>
    __device__ static __forceinline__ void level(const SweepArgs &a, Smem &sm, QU &qu, ACC &acc,
                                                 float (&val)[PY], const Pre &P,
                                                 int i, int par, int x0, int xend, int64_t N,
                                                 int lane, int wv, const int32_t (&yz)[PY],
                                                 const bool (&din)[PY], const float (&pyz)[PY],
                                                 const bool (&core)[PY])
    {
        constexpr int Q = G::Q;
        const int c = i - t * M;
        // shift level t's queue and push the newest plane (c + M)
#pragma unroll
        for (int r = 0; r < PY; ++r) {
#pragma unroll
            for (int j = 0; j + 1 < Q; ++j) qu[t - 1][r][j] = qu[t - 1][r][j + 1];
            qu[t - 1][r][Q - 1] = val[r];
        }
        // publish the centre plane c of u^{t-1} for y/z neighbours
        float *S;
        constexpr int W = (t == 1) ? G::L0W : G::RZ;
        constexpr int OFF = M;          // row offset (and, for t == 1, column offset)
        constexpr int COFF = (t == 1) ? M : 0;
        if constexpr (t == 1) {
            S = sm.s0[par];
#pragma unroll
            for (int s = 0; s < G::HS; ++s)
                if (threadIdx.x + s * G::NT < G::NHALO) {
                    // slot positions are recomputed from the slot index (cheap, no registers)
                    const int h = threadIdx.x + s * G::NT;
                    int row, col;
                    if (h < 2 * M * G::L0W) {
                        const int band = h / G::L0W;
                        col = h - band * G::L0W;
                        row = band < M ? band : band + G::RY;
                    } else {
                        const int h2 = h - 2 * M * G::L0W;
                        row = M + h2 / (2 * M);
                        const int cj = h2 % (2 * M);
                        col = cj < M ? cj : cj + G::RZ;
                    }
                    S[row * G::L0W + col] = P.halo[s];
                }
        } else {
            S = sm.s1[t - 2][par];
        }
#pragma unroll
        for (int r = 0; r < PY; ++r) S[(wv * PY + r + OFF) * W + lane + COFF] = qu[t - 1][r][M];
        __syncthreads();

        // level t's region: owned region shrunk by M (t - 1)
        constexpr int lo = M * (t - 1);
        const bool xin = (unsigned)c < (unsigned)a.nx;
        const bool zreg = lane >= lo && lane < G::RZ - lo;
        float out[PY];
        if (needed(a, t, c, x0, xend)) {
            const float pxv = a.px[c];
            // y neighbours: rows above / below the thread's PY rows come from LDS
            float colv[PY + 2 * M];
#pragma unroll
            for (int j = 0; j < M; ++j) {
                colv[j] = S[(wv * PY - M + j + OFF) * W + lane + COFF];
                colv[M + PY + j] = S[(wv * PY + PY + j + OFF) * W + lane + COFF];
            }
#pragma unroll
            for (int r = 0; r < PY; ++r) colv[M + r] = qu[t - 1][r][M];
#pragma unroll
            for (int r = 0; r < PY; ++r) {
                const int rr = wv * PY + r;
                const bool active = din[r] && zreg && rr >= lo && rr < G::RY - lo;
                float o = 0.0f;
                if (active) {
                    const float uc = qu[t - 1][r][M];
                    const float *row = S + (rr + OFF) * W + lane + COFF;
                    float lap = 0.0f;
#pragma unroll
                    for (int k = 1; k <= M; ++k) {
                        const float xs = qu[t - 1][r][M - k] + qu[t - 1][r][M + k];
                        const float ys = colv[M + r - k] + colv[M + r + k];
                        const float zs = row[-k] + row[k];
                        lap = fmaf(a.w.wx[k - 1], fmaf(-2.0f, uc, xs), lap);
                        lap = fmaf(a.w.wy[k - 1], fmaf(-2.0f, uc, ys), lap);
                        lap = fmaf(a.w.wz[k - 1], fmaf(-2.0f, uc, zs), lap);
                    }
                    const float qv = P.q[t - 1][r];
                    float up;
                    if constexpr (t == 1) up = P.up1[r];
                    else up = qu[t - 2][r][0];
                    const float eta = qv * (pxv + pyz[r]);
                    const float num = fmaf(qv, lap, fmaf(eta - 1.0f, up, 2.0f * uc));
                    o = num;
                    if (eta != 0.0f) o = num / (1.0f + eta);
                }
                out[r] = o;
            }
            const int step = a.step0 + t - 1;
            if (a.inj.cnt > 0) {
                const int jb = a.inj.xptr[c], je = a.inj.xptr[c + 1];
                if (jb < je) {
                    const float *arow = a.amp + (a.abase + (int64_t)a.adir * step) * a.inj.stride;
                    for (int j = jb; j < je; ++j) {
                        const int32_t p = a.inj.yz[j];
                        const float sc = a.inj.scale[j];
                        const float w = arow[a.inj.id[j]];
#pragma unroll
                        for (int r = 0; r < PY; ++r) {
                            const int rr = wv * PY + r;
                            const bool active = din[r] && zreg && rr >= lo && rr < G::RY - lo;
                            if (active && yz[r] == p) out[r] = fmaf(sc, w, out[r]);
                        }
                    }
                }
            }
            const bool own = c >= x0 && c < xend;
            if (own && a.rec.cnt > 0) {
                const int jb = a.rec.xptr[c], je = a.rec.xptr[c + 1];
                if (jb < je) {
                    float *orow = a.rec_out + (a.rbase + (int64_t)a.rdir * step) * a.rec.stride;
                    for (int j = jb; j < je; ++j) {
                        const int32_t p = a.rec.yz[j];
#pragma unroll
                        for (int r = 0; r < PY; ++r)
                            if (core[r] && yz[r] == p) orow[a.rec.id[j]] = out[r] * a.rscale;
                    }
                }
            }
            if constexpr (MODE == kSaveD2) {
                if (own) {
                    float *dp = a.d2 + (a.dslot0 + (int64_t)a.ddir * (t - 1)) * N +
                                (int64_t)c * a.sxy;
#pragma unroll
                    for (int r = 0; r < PY; ++r) {
                        if (core[r]) {
                            float um;
                            if constexpr (t == 1) um = P.up1[r];
                            else um = qu[t - 2][r][0];
                            dp[yz[r]] = fmaf(-2.0f, qu[t - 1][r][M], out[r]) + um;
                        }
                    }
                }
            }
            if constexpr (MODE == kImaging) {
                if (own) {
                    const float *dp = a.d2 + (a.dslot0 + (int64_t)a.ddir * (t - 1)) * N +
                                      (int64_t)c * a.sxy;
                    double *gp = a.g + (int64_t)c * a.sxy;
                    constexpr int J = (T - t) * M;
#pragma unroll
                    for (int r = 0; r < PY; ++r) {
                        if (core[r]) {
                            double base;
                            if constexpr (t == 1) base = gp[yz[r]];
                            else base = acc[r][J];
                            const double nv = fma((double)out[r], (double)dp[yz[r]], base);
                            if constexpr (t == T) gp[yz[r]] = nv;
                            else acc[r][J] = nv;
                        }
                    }
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < PY; ++r) out[r] = 0.0f;
        }

        if constexpr (t == T) {
            // the pass's outputs at plane c: u^{n+T} and (T >= 2) u^{n+T-1}
            if (xin && c >= x0 && c < xend) {
                float *o1 = a.o1 + (int64_t)c * a.sxy;
#pragma unroll
                for (int r = 0; r < PY; ++r)
                    if (core[r]) o1[yz[r]] = out[r];
                if constexpr (T >= 2) {
                    float *o2 = a.o2 + (int64_t)c * a.sxy;
#pragma unroll
                    for (int r = 0; r < PY; ++r)
                        if (core[r]) o2[yz[r]] = qu[T - 1][r][M];
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < PY; ++r) val[r] = out[r];
            level<t + 1>(a, sm, qu, acc, val, P, i, par, x0, xend, N, lane, wv, yz, din, pyz, core);
        }
    }
};

template <int M, int T, int PY, int NW, int MODE>
__global__ __launch_bounds__(64 * NW) void k_stream(SweepArgs a)
{
    using K = StreamKernel<M, T, PY, NW, MODE>;
    __shared__ typename K::Smem sm;
    K::run(a, sm);
}

}  // namespace fdw
