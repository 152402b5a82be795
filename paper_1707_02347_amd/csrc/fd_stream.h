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
// Memory access: every global load of an iteration is issued one plane ahead
// as a raw buffer load: the buffer resource covers exactly one plane of one
// field (record count 0 for a plane outside the grid or not needed), and the
// per-lane byte offset of a point outside the grid is 0x80000000, beyond any
// plane.  Out-of-range buffer loads return 0 on CDNA, so the Dirichlet zeros
// come from the hardware range check: no load sits behind a branch or a
// select, and no wait on a late load drains the prefetch.  Per-plane scalars
// (sponge profile, point table ranges) are staged in LDS once per workgroup.
//
// The per-point FP32 operation order is the one fixed by the untiled kernel
// (fd_naive.hip), so every configuration returns bit-identical results.
#pragma once

#include "fd_internal.h"
#include "fd_stream_entry.h"

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
    static constexpr int SPAN = kMaxLx + 2 * (T - 1) * M + 2;  // per-plane table entries
    static_assert(TY >= 1 && TZ >= 1, "core tile must be non-empty");
};

__device__ __forceinline__ float ld(const float *base, uint32_t byte_off)
{
    return *(const float *)((const char *)base + byte_off);
}

constexpr uint32_t kOutside = 0x80000000u;  // byte offset of a point outside the grid

// Buffer resource over plane `plane` of a field (an empty range if !valid).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float *field, int plane,
                                                             int64_t sxy, bool valid)
{
    const float *base = field + (int64_t)(valid ? plane : 0) * sxy;
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0,
                                             valid ? (int)(uint32_t)(sxy * 4) : 0, 0x00020000);
}

__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t byte_off)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 0));
}

__device__ __forceinline__ float *at(float *base, uint32_t byte_off)
{
    return (float *)((char *)base + byte_off);
}

template <int M, int T, int PY, int NW, int MODE, bool ISO>
struct StreamKernel {
    using G = Geo<M, T, PY, NW>;
    // Register queues along x: for short queues the x loop is unrolled by the
    // queue length Q and the queues rotate by renaming (slot of logical entry j
    // at phase PH is (PH + 1 + j) mod Q); long queues (M > 4) shift instead, to
    // keep the loop body small enough for the instruction cache.
    static constexpr int Q = G::Q;
    static constexpr bool ROT = (Q <= 9);
    static constexpr int UNROLL = ROT ? Q : 1;
    // prefetch depth in planes: two for short stencils; one for M > 4, where the
    // extra registers would cost a wave per SIMD
    static constexpr int PD = (M <= 4) ? 2 : 1;
    // slot of logical queue entry j at phase PH, after / before this phase's push
    template <int PH>
    __device__ static constexpr int pj(int j)
    {
        return ROT ? (PH + 1 + j) % Q : j;
    }
    template <int PH>
    __device__ static constexpr int pjb(int j)
    {
        return ROT ? (PH + j) % Q : j;
    }

    // Level-0 plane with its M-wide halo ring; planes of levels 1..T-1 over the
    // owned region, padded by M rows above and below so that the rows a thread
    // reads next to its own (used only where they lie inside the level's
    // region) always stay inside the buffer; per-plane tables of the chunk.
    struct Smem {
        float s0[2][G::L0H * G::L0W];
        float s1[(T > 1) ? (T - 1) : 1][2][(T > 1) ? (G::RY + 2 * M) * G::RZ : 1];
        float px[G::SPAN];
        int ixp[G::SPAN];
        int rxp[G::SPAN];
    };

    struct Pre {
        float head[PY];
        float halo[G::HS];
        float up1[PY];
        float q[T][PY];
    };

    struct Thread {
        int lane, wv, x0, xend, cbase;
        uint32_t bo[PY];    // byte offset of each owned point in a plane (kOutside if outside)
        bool din[PY];       // owned point inside the grid
        bool core[PY];      // owned point inside the output tile
        float pyz[PY];      // py[y] + pz[z]
        uint32_t hb[G::HS]; // byte offsets of this thread's halo slots (kOutside if outside)
        bool hv[G::HS];     // halo slot inside the grid
    };

    // Run tile `bid` of the ntiles tiles of one shot's pass.
    __device__ static void run(const SweepArgs &a, Smem &sm, int bid, int ntiles)
    {
        // -------- tile decode (optionally XCD-aware: consecutive tiles on one XCD)
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

        Thread th;
        th.x0 = bx * a.lx;
        th.xend = min(th.x0 + a.lx, a.nx);
        th.cbase = th.x0 - (T - 1) * M;
        th.lane = threadIdx.x & 63;
        th.wv = threadIdx.x >> 6;
        const int z = z1 + th.lane;
        const bool zin = (unsigned)z < (unsigned)a.nz;
        const float pzv = zin ? a.pz[z] : 0.0f;
#pragma unroll
        for (int r = 0; r < PY; ++r) {
            const int rr = th.wv * PY + r;
            const int y = y1 + rr;
            const bool yin = (unsigned)y < (unsigned)a.ny;
            th.din[r] = yin && zin;
            th.bo[r] = th.din[r] ? (uint32_t)(y * a.nz + z) * 4u : kOutside;
            th.pyz[r] = th.din[r] ? (a.py[y] + pzv) : 0.0f;
            th.core[r] = th.din[r] && rr >= G::H1 && rr < G::RY - G::H1 && th.lane >= G::H1 &&
                         th.lane < G::RZ - G::H1;
        }
        // halo ring of the level-0 plane (positions fixed for the whole pass)
#pragma unroll
        for (int s = 0; s < G::HS; ++s) {
            int row, col;
            const bool used = halo_pos(threadIdx.x + s * G::NT, row, col);
            const int gy = y1 - M + row, gz = z1 - M + col;
            th.hv[s] = used && (unsigned)gy < (unsigned)a.ny && (unsigned)gz < (unsigned)a.nz;
            th.hb[s] = th.hv[s] ? (uint32_t)(gy * a.nz + gz) * 4u : kOutside;
        }
        // per-plane tables of the planes any level of this chunk computes
        const int span = th.xend - th.x0 + 2 * (T - 1) * M + 1;
        for (int j = threadIdx.x; j < span; j += G::NT) {
            const int c = th.cbase + j;
            const bool cin = (unsigned)c < (unsigned)a.nx;
            sm.px[j] = cin ? a.px[c] : 0.0f;
            sm.ixp[j] = (a.inj.cnt > 0 && c >= 0 && c <= a.nx) ? a.inj.xptr[c] : 0;
            sm.rxp[j] = (a.rec.cnt > 0 && c >= 0 && c <= a.nx) ? a.rec.xptr[c] : 0;
        }
        // (the first barrier of the loop orders these writes before any read)

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

        const int ibeg = th.x0 - T * M;
        const int iend = th.xend + T * M;
        const int64_t N = (int64_t)a.nx * a.sxy;

        Pre pf[PD];  // pf[d] holds the loads of iteration i + d
#pragma unroll
        for (int d = 0; d < PD; ++d) load(a, th, pf[d], ibeg + d);
        for (int i0 = ibeg; i0 < iend; i0 += UNROLL) block<0>(a, sm, th, qu, acc, pf, i0, iend, N);
    }

    // Iterations i0 + PH .. i0 + UNROLL - 1 of the x loop (one per phase).  Each
    // iteration publishes the y/z planes of all T levels first (level t needs
    // u^{t-1} at plane c_t, which entered its queue M iterations ago), so one
    // barrier per iteration serves every level.
    template <int PH, class QU, class ACC>
    __device__ static __forceinline__ void block(const SweepArgs &a, Smem &sm, const Thread &th,
                                                 QU &qu, ACC &acc, Pre (&pf)[PD], int i0, int iend,
                                                 int64_t N)
    {
        if constexpr (PH < UNROLL) {
            const int i = i0 + PH;
            if (i < iend) {
                const int par = i & 1;
                const Pre cur = pf[0];
#pragma unroll
                for (int d = 0; d + 1 < PD; ++d) pf[d] = pf[d + 1];
                if (i + PD < iend) load(a, th, pf[PD - 1], i + PD);
                if constexpr (MODE == kImaging) {
#pragma unroll
                    for (int r = 0; r < PY; ++r)
#pragma unroll
                        for (int j = 0; j + 1 < G::AQ; ++j) acc[r][j] = acc[r][j + 1];
                }
                publish<1, PH>(sm, th, qu, cur, par);
                __syncthreads();
                float val[PY];  // value produced by the previous level in this iteration
#pragma unroll
                for (int r = 0; r < PY; ++r) val[r] = cur.head[r];
                level<1, PH>(a, sm, th, qu, acc, val, cur, i, par, N);
                block<PH + 1>(a, sm, th, qu, acc, pf, i0, iend, N);
            }
        }
    }

    // Write the centre plane c_t of u^{t-1} (queue entry M after this phase's
    // push, M + 1 before it) into level t's LDS plane; level 1 adds the halo ring.
    template <int t, int PH, class QU>
    __device__ static __forceinline__ void publish(Smem &sm, const Thread &th, QU &qu, const Pre &P,
                                                   int par)
    {
        if constexpr (t <= T) {
            constexpr int W = (t == 1) ? G::L0W : G::RZ;
            constexpr int COFF = (t == 1) ? M : 0;
            float *S;
            if constexpr (t == 1) {
                S = sm.s0[par];
#pragma unroll
                for (int s = 0; s < G::HS; ++s) {
                    int row, col;
                    if (halo_pos(threadIdx.x + s * G::NT, row, col)) S[row * G::L0W + col] = P.halo[s];
                }
            } else {
                S = sm.s1[t - 2][par];
            }
#pragma unroll
            for (int r = 0; r < PY; ++r)
                S[(th.wv * PY + r + M) * W + th.lane + COFF] = qu[t - 1][r][pjb<PH>(M + 1)];
            publish<t + 1, PH>(sm, th, qu, P, par);
        }
    }

    // Position (row, col) in the level-0 LDS plane of halo slot h; false if unused.
    __device__ static __forceinline__ bool halo_pos(int h, int &row, int &col)
    {
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
        return h < G::NHALO;
    }

    // Planes level t must produce: [x0 - (T - t) M, xend + (T - t) M) within the grid.
    __device__ static __forceinline__ bool needed(const SweepArgs &a, const Thread &th, int t, int c)
    {
        return (unsigned)c < (unsigned)a.nx && c >= th.x0 - (T - t) * M &&
               c < th.xend + (T - t) * M;
    }

    // Issue the loads of iteration i: head plane i of u^n; level-0 halo ring and
    // u^{n-1} at plane i - M; q at every level's plane i - t M.
    __device__ static __forceinline__ void load(const SweepArgs &a, const Thread &th, Pre &P, int i)
    {
        const auto rh = plane_rsrc(a.u0, i, a.sxy, (unsigned)i < (unsigned)a.nx);
#pragma unroll
        for (int r = 0; r < PY; ++r) P.head[r] = bload(rh, th.bo[r]);
        const int c1 = i - M;
        const bool l1 = needed(a, th, 1, c1);
        const auto rc = plane_rsrc(a.u0, c1, a.sxy, l1);
#pragma unroll
        for (int s = 0; s < G::HS; ++s) P.halo[s] = bload(rc, th.hb[s]);
        const auto rm = plane_rsrc(a.um, c1, a.sxy, l1);
#pragma unroll
        for (int r = 0; r < PY; ++r) P.up1[r] = bload(rm, th.bo[r]);
#pragma unroll
        for (int t = 1; t <= T; ++t) {
            const int ct = i - t * M;
            const auto rq = plane_rsrc(a.q, ct, a.sxy, needed(a, th, t, ct));
#pragma unroll
            for (int r = 0; r < PY; ++r) P.q[t - 1][r] = bload(rq, th.bo[r]);
        }
    }

    // Process level t (1..T) at plane c = i - t*M, then recurse to level t+1.
    template <int t, int PH, class QU, class ACC>
    __device__ static __forceinline__ void level(const SweepArgs &a, Smem &sm, const Thread &th,
                                                 QU &qu, ACC &acc, float (&val)[PY], const Pre &P,
                                                 int i, int par, int64_t N)
    {
        const int c = i - t * M;
        const int lane = th.lane, wv = th.wv;
        // push the newest plane (c + M) into level t's queue
#pragma unroll
        for (int r = 0; r < PY; ++r) {
            if constexpr (ROT) {
                qu[t - 1][r][PH] = val[r];  // the slot of the oldest entry
            } else {
#pragma unroll
                for (int j = 0; j + 1 < Q; ++j) qu[t - 1][r][j] = qu[t - 1][r][j + 1];
                qu[t - 1][r][Q - 1] = val[r];
            }
        }
        // level t's y/z plane (published before this iteration's barrier)
        constexpr int W = (t == 1) ? G::L0W : G::RZ;
        constexpr int OFF = M;          // row offset (and, for t == 1, column offset)
        constexpr int COFF = (t == 1) ? M : 0;
        const float *S;
        if constexpr (t == 1) S = sm.s0[par];
        else S = sm.s1[t - 2][par];

        // level t's region: owned region shrunk by M (t - 1)
        constexpr int lo = M * (t - 1);
        const bool xin = (unsigned)c < (unsigned)a.nx;
        const bool zreg = lane >= lo && lane < G::RZ - lo;
        float out[PY];
        if (needed(a, th, t, c)) {
            const int tj = c - th.cbase;  // index into the per-plane tables
            const float pxv = sm.px[tj];
            // y neighbours: rows above / below the thread's PY rows come from LDS
            float colv[PY + 2 * M];
#pragma unroll
            for (int j = 0; j < M; ++j) {
                colv[j] = S[(wv * PY - M + j + OFF) * W + lane + COFF];
                colv[M + PY + j] = S[(wv * PY + PY + j + OFF) * W + lane + COFF];
            }
#pragma unroll
            for (int r = 0; r < PY; ++r) colv[M + r] = qu[t - 1][r][pj<PH>(M)];
#pragma unroll
            for (int r = 0; r < PY; ++r) {
                // computed for every owned point (all operands are finite: loads
                // outside the grid read as 0); points outside the grid or the
                // level's region are then set to 0
                const int rr = wv * PY + r;
                const bool active = th.din[r] && zreg && rr >= lo && rr < G::RY - lo;
                const float uc = qu[t - 1][r][pj<PH>(M)];
                const float *row = S + (rr + OFF) * W + lane + COFF;
                float lap = 0.0f;
#pragma unroll
                for (int k = 1; k <= M; ++k) {
                    const float xs = qu[t - 1][r][pj<PH>(M - k)] + qu[t - 1][r][pj<PH>(M + k)];
                    const float ys = colv[M + r - k] + colv[M + r + k];
                    const float zs = row[-k] + row[k];
                    if constexpr (ISO) {
                        lap = fmaf(a.w.wx[k - 1], fmaf(a.w.cc, uc, (xs + ys) + zs), lap);
                    } else {
                        lap = fmaf(a.w.wx[k - 1], fmaf(-2.0f, uc, xs), lap);
                        lap = fmaf(a.w.wy[k - 1], fmaf(-2.0f, uc, ys), lap);
                        lap = fmaf(a.w.wz[k - 1], fmaf(-2.0f, uc, zs), lap);
                    }
                }
                const float qv = P.q[t - 1][r];
                float up;
                if constexpr (t == 1) up = P.up1[r];
                else up = qu[t - 2][r][pj<PH>(0)];
                const float eta = qv * (pxv + th.pyz[r]);
                const float num = fmaf(qv, lap, fmaf(eta - 1.0f, up, 2.0f * uc));
                float o = num;
                if (eta != 0.0f) o = num / (1.0f + eta);
                out[r] = active ? o : 0.0f;
            }
            const int step = a.step0 + t - 1;
            {
                const int jb = __builtin_amdgcn_readfirstlane(sm.ixp[tj]);
                const int je = __builtin_amdgcn_readfirstlane(sm.ixp[tj + 1]);
                if (jb < je) {
                    const float *arow = a.amp + (a.abase + (int64_t)a.adir * step) * a.inj.stride;
                    for (int j = jb; j < je; ++j) {
                        const uint32_t p = (uint32_t)a.inj.yz[j] * 4u;
                        const float sc = a.inj.scale[j];
                        const float w = arow[a.inj.id[j]];
#pragma unroll
                        for (int r = 0; r < PY; ++r) {
                            const int rr = wv * PY + r;
                            const bool active = th.din[r] && zreg && rr >= lo && rr < G::RY - lo;
                            if (active && th.bo[r] == p) out[r] = fmaf(sc, w, out[r]);
                        }
                    }
                }
            }
            const bool own = c >= th.x0 && c < th.xend;
            if (own) {
                const int jb = __builtin_amdgcn_readfirstlane(sm.rxp[tj]);
                const int je = __builtin_amdgcn_readfirstlane(sm.rxp[tj + 1]);
                if (jb < je) {
                    float *orow = a.rec_out + (a.rbase + (int64_t)a.rdir * step) * a.rec.stride;
                    for (int j = jb; j < je; ++j) {
                        const uint32_t p = (uint32_t)a.rec.yz[j] * 4u;
#pragma unroll
                        for (int r = 0; r < PY; ++r)
                            if (th.core[r] && th.bo[r] == p) orow[a.rec.id[j]] = out[r] * a.rscale;
                    }
                }
            }
            if constexpr (MODE == kSaveD2) {
                if (own) {
                    float *dp = a.d2 + (a.dslot0 + (int64_t)a.ddir * (t - 1)) * N +
                                (int64_t)c * a.sxy;
#pragma unroll
                    for (int r = 0; r < PY; ++r) {
                        if (th.core[r]) {
                            float um;
                            if constexpr (t == 1) um = P.up1[r];
                            else um = qu[t - 2][r][pj<PH>(0)];
                            *at(dp, th.bo[r]) = fmaf(-2.0f, qu[t - 1][r][pj<PH>(M)], out[r]) + um;
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
                        if (th.core[r]) {
                            const uint32_t e = th.bo[r] >> 2;
                            double base;
                            if constexpr (t == 1) base = gp[e];
                            else base = acc[r][J];
                            const double nv = fma((double)out[r], (double)ld(dp, th.bo[r]), base);
                            if constexpr (t == T) gp[e] = nv;
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
            if (xin && c >= th.x0 && c < th.xend) {
                float *o1 = a.o1 + (int64_t)c * a.sxy;
#pragma unroll
                for (int r = 0; r < PY; ++r)
                    if (th.core[r]) *at(o1, th.bo[r]) = out[r];
                if constexpr (T >= 2) {
                    float *o2 = a.o2 + (int64_t)c * a.sxy;
#pragma unroll
                    for (int r = 0; r < PY; ++r)
                        if (th.core[r]) *at(o2, th.bo[r]) = qu[T - 1][r][pj<PH>(M)];
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < PY; ++r) val[r] = out[r];
            level<t + 1, PH>(a, sm, th, qu, acc, val, P, i, par, N);
        }
    }
};

// One pass of one shot: workgroup b runs tile b (arguments by value, so every
// field lives in scalar registers or the kernel-argument segment).
template <int M, int T, int PY, int NW, int MODE, bool ISO>
__global__ __launch_bounds__(64 * NW) void k_stream(SweepArgs a)
{
    using K = StreamKernel<M, T, PY, NW, MODE, ISO>;
    __shared__ typename K::Smem sm;
    K::run(a, sm, blockIdx.x, gridDim.x);
}

// Grouped persistent pass: the workgroups walk the flat tile range of all the
// entries (one per shot) of a batch.
template <int M, int T, int PY, int NW, int MODE, bool ISO>
__global__ __launch_bounds__(64 * NW) void k_stream_grouped(const GroupEntry *__restrict__ list,
                                                            int nlist, int total)
{
    using K = StreamKernel<M, T, PY, NW, MODE, ISO>;
    __shared__ typename K::Smem sm;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        int e = 0;
        while (e + 1 < nlist && list[e + 1].tile0 <= item) ++e;
        const SweepArgs &a = list[e].a;
        K::run(a, sm, item - list[e].tile0, a.ntz * a.nty * a.ntx);
        __syncthreads();  // the next tile rewrites the LDS tables and planes
    }
}

// Launch helpers shared by the generated entry files.
template <int M, int T, int PY, int NW, int MODE, int F>
bool entry_launch(const SweepArgs &a, hipStream_t s)
{
    const dim3 grid(a.ntz * a.nty * a.ntx), block(64 * NW);
    if (a.w.iso) {
        hipLaunchKernelGGL((k_stream<M, T, PY, NW, MODE, true>), grid, block, 0, s, a);
        return true;
    }
    if constexpr ((F & 1) != 0) {
        hipLaunchKernelGGL((k_stream<M, T, PY, NW, MODE, false>), grid, block, 0, s, a);
        return true;
    }
    return false;
}

template <int M, int T, int PY, int NW, int MODE, int F>
bool entry_launch_group(bool iso, const GroupEntry *list, int nlist, int total, int grid,
                        hipStream_t s)
{
    if constexpr ((F & 2) != 0) {
        const dim3 g(grid), block(64 * NW);
        if (iso) {
            hipLaunchKernelGGL((k_stream_grouped<M, T, PY, NW, MODE, true>), g, block, 0, s, list,
                               nlist, total);
            return true;
        }
        if constexpr ((F & 1) != 0) {
            hipLaunchKernelGGL((k_stream_grouped<M, T, PY, NW, MODE, false>), g, block, 0, s, list,
                               nlist, total);
            return true;
        }
    }
    return false;
}

template <int M, int T, int PY, int NW, int MODE, int F>
int entry_occupancy(bool iso)
{
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    if constexpr ((F & 2) != 0) {
        if (iso)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &n, reinterpret_cast<const void *>(&k_stream_grouped<M, T, PY, NW, MODE, true>),
                64 * NW, 0);
        else if constexpr ((F & 1) != 0)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &n, reinterpret_cast<const void *>(&k_stream_grouped<M, T, PY, NW, MODE, false>),
                64 * NW, 0);
    }
    return e == hipSuccess ? n : 0;
}

}  // namespace fdw
