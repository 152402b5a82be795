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
    // the M-wide ring of the level-0 plane without its corners (the star
    // stencil never reads them): M rows above and below the owned columns, M
    // columns left and right of the owned rows
    static constexpr int NHALO = 2 * M * RZ + RY * 2 * M;
    static constexpr int HS = (NHALO + NT - 1) / NT;
    static constexpr int AQ = (T - 1) * M + 1;   // imaging accumulator queue length
    static constexpr int SPAN = kMaxLx + 2 * (T - 1) * M + 2;  // per-plane table entries
    static_assert(TY >= 1 && TZ >= 1, "core tile must be non-empty");
};

constexpr uint32_t kOutside = 0x80000000u;  // byte offset of a point outside the grid

// Buffer resource over plane `plane` of a field (an empty range if !valid).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float *field, int plane,
                                                             int64_t sxy, bool valid)
{
    const float *base = field + (int64_t)(valid ? plane : 0) * sxy;
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0,
                                             valid ? (int)(uint32_t)(sxy * 4) : 0, 0x00020000);
}

// Cache policy of a buffer access (the instruction's cache-policy bits):
// kKeep for data that other workgroups or the next step read again soon,
// kStream (non-temporal) for data touched once per step.  Non-temporal stores
// of the new field are faster at every size measured; non-temporal loads of
// u^{n-1} and q only when the fields do not fit the Infinity Cache (they keep
// q from staying there for the next step).  The saved second differences are
// read exactly once and always load non-temporally (256^3 gradient: 4.29 ->
// 4.57 per second, the wavefields and the image stay in the cache).
constexpr int kKeep = 0;
constexpr int kStream = 2;

template <int CP = kKeep>
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t byte_off)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, CP));
}

// Buffer store: dropped by the hardware when byte_off is beyond the resource's
// range, so a store for a point outside the output needs no branch.
template <int CP = kKeep>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t byte_off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)byte_off, 0, CP);
}

// Resource over `nbytes` bytes at `base` (an empty range if !valid).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t span_rsrc(const void *base, int64_t nbytes,
                                                            bool valid)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0,
                                             valid ? (int)(uint32_t)nbytes : 0, 0x00020000);
}


template <int M, int T, int PY, int NW, int MODE, bool ISO, bool NTL, bool PS>
struct StreamKernel {
    using G = Geo<M, T, PY, NW>;
    // cache policy of the loads each point needs once per step (u^{n-1}, q,
    // and the gradient fields)
    static constexpr int LP = NTL ? kStream : kKeep;
    // kBornFused: background and perturbation in one pass (two fields, F = 2)
    static constexpr bool FUSED = (MODE == kBornFused);
    static_assert(!FUSED || T == 1, "fused Born passes are single-step");
    static constexpr int F = FUSED ? 2 : 1;
    // PS: the chunk's point entries are staged in LDS (the host launches this
    // form only when every chunk's entries fit); otherwise the per-plane walk
    // reads the tables in memory.  Each form holds one walk only: both in one
    // body cost the streaming loop 3.5 % (a larger unrolled body).
    static constexpr bool STAGE = PS;
    static constexpr int PC = PS ? kPtsCap / T : 1;
    // Register queues along x.  Short queues (M <= 4) rotate by renaming: the
    // x loop is unrolled by QS (the queue length 2M + 1 rounded up to a
    // multiple of NS below) and the slot of logical entry j (0 = oldest,
    // 2M = newest) at phase PH is (PH - 2M + j) mod QS.  Long queues (M > 4)
    // shift instead, to keep the loop body small enough for the instruction
    // cache; so do the time-blocked gradient modes, whose unrolled bodies
    // would not fit in the register file.
    static constexpr bool ROT = (M <= 4) && !(T >= 2 && MODE != kPlain);
    // Global loads are issued ahead through NS register slots: iteration i
    // consumes slot i mod NS and, at its start, refills slot (i + NS - 1) mod NS
    // (consumed in iteration i - 1) with the loads of iteration i + NS - 1.
    // Every load and store of the loop is issued unconditionally (a point or
    // plane outside the range gets an offset or resource that the hardware
    // range check discards), so the compiler can count outstanding memory
    // operations exactly and never drains the loads still in flight.
    // Shifting queues (T = 1) use two slots as well, with the loop unrolled by
    // two (512^3 so 16: 256 -> 287 GPts/s, although the extra registers halve
    // the occupancy); time-blocked kernels with shifting queues, short of
    // registers, copy a single slot each iteration.
    static constexpr int NS = (ROT || T == 1) ? 2 : 1;
    static constexpr int Q = G::Q;
    static constexpr int QS = ROT ? (Q + NS - 1) / NS * NS : Q;
    static constexpr int UNROLL = ROT ? QS : NS;
    static_assert(UNROLL % NS == 0, "prefetch slots must be compile-time constants");
    // slot of logical queue entry j at phase PH, after / before this phase's push
    template <int PH>
    __device__ static constexpr int pj(int j)
    {
        return ROT ? (PH - 2 * M + j + 2 * QS) % QS : j;
    }
    template <int PH>
    __device__ static constexpr int pjb(int j)
    {
        return ROT ? (PH - 1 - 2 * M + j + 2 * QS) % QS : j;
    }

    // Level-0 plane with its M-wide halo ring; planes of levels 1..T-1 over the
    // owned region, padded by M rows above and below so that the rows a thread
    // reads next to its own (used only where they lie inside the level's
    // region) always stay inside the buffer; per-plane tables of the chunk.
    struct Smem {
        float s0[F][2][G::L0H * G::L0W];  // field f's level-0 plane (two parities)
        float s1[(T > 1) ? (T - 1) : 1][2][(T > 1) ? (G::RY + 2 * M) * G::RZ : 1];
        float px[G::SPAN];
        int ixb[G::SPAN], ixe[G::SPAN];  // per plane: source entries this tile may hold
        int rxb[G::SPAN], rxe[G::SPAN];  // per plane: receiver entries its core may hold
        // The point entries of the chunk's planes, staged when they fit (i0,
        // r0: first staged table index, or -1: walk the table in memory).
        // Sources: node, owning wave (-1: outside the owned region), scale and
        // the amplitude of each of the pass's T steps.  Receivers: node, owning
        // wave (-1: outside the output core or the chunk's own planes), trace
        // column (or entry slot), and the T samples the pass records, written
        // out after the loop.
        // A node is coded (wave << 16) | (row in the wave << 8) | column.
        int i0, r0;
        int iyz[PC];
        float isc[PC], iamp[T][PC];
        int rcode[PC], rdst[PC];
        float rval[T][PC];
    };

    static constexpr bool IMG = (MODE == kImaging);
    static constexpr bool BORN = (MODE == kBorn);
    static_assert(!BORN || T == 1, "Born passes are single-step");

    struct Pre {
        float head[PY];
        float halo[G::HS];
        float up1[PY];
        float q[T][PY];
        // imaging: the image's partial sums at level 1's plane and the saved
        // second differences at every level's plane
        float g[IMG ? PY : 1];
        float d2[IMG ? T : 1][IMG ? PY : 1];
        // Born: the scattering coefficient and the background's second
        // difference at level 1's plane
        float bs[(BORN || FUSED) ? PY : 1], bd[BORN ? PY : 1];
        // fused Born: the perturbation field's head, halo and previous level
        float head2[FUSED ? PY : 1], halo2[FUSED ? G::HS : 1], up2[FUSED ? PY : 1];
    };

    struct Thread {
        int lane, wv, x0, xend, cbase, iend;
        int refl;           // -1: stream upward; else plane of position i is refl - i
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
        // -------- tile decode
        int bz, by, bx;
        if (a.remap) {
            // slot s of XCD k (workgroups are dealt to the 8 XCDs round-robin)
            // runs tile s of that XCD's super-tiles k, k + 8, ...; a super-tile
            // is all ntz z-tiles of gy consecutive y-tiles and gx x-chunks, z
            // fastest, so the tiles of one super-tile start together
            const int xcd = bid & 7, slot = bid >> 3;
            const int tps = a.ntz * a.gy * a.gx;
            const int sup = (slot / tps) * 8 + xcd;
            const int loc = slot % tps;
            const int nsy = a.nty / a.gy;
            bz = loc % a.ntz;
            by = (sup % nsy) * a.gy + (loc / a.ntz) % a.gy;
            bx = (sup / nsy) * a.gx + loc / (a.ntz * a.gy);
        } else {
            bz = bid % a.ntz;
            by = (bid / a.ntz) % a.nty;
            bx = bid / (a.ntz * a.nty);
        }
        const int z1 = bz * G::TZ - G::H1;
        const int y1 = by * G::TY - G::H1;

        Thread th;
        th.x0 = a.xoff + bx * (a.xstride > 0 ? a.xstride : a.lx);
        th.xend = min(th.x0 + a.lx, a.nx);
        if constexpr (T == 2 && MODE == kPlain) {
            // first phase of a split pass: the chunk's planes are its base (level
            // 1); level 2 leaves out M planes at each end another chunk shares
            if (a.split) {
                if (th.x0 > 0) th.x0 += M;
                if (th.xend < a.nx) th.xend -= M;
            }
        }
        // stream position i maps to plane i (upward) or x0 + xend - 1 - i
        // (downward); the set of planes a chunk touches is symmetric under
        // that reflection, so both directions visit the same planes, and the
        // x stencil is symmetric, so the results are the same bits
        th.refl = (a.alt && (bx & 1)) ? th.x0 + th.xend - 1 : -1;
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
            th.bo[r] = th.din[r] ? (uint32_t)(y * a.nzp + z) * 4u : kOutside;
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
            th.hb[s] = th.hv[s] ? (uint32_t)(gy * a.nzp + gz) * 4u : kOutside;
        }
        // per-plane tables of the planes any level of this chunk computes: the
        // sponge profile and each plane's range of point entries, emptied when
        // the bounding box of the plane's points misses this tile (its owned
        // region for sources, its output core for receivers)
        const int span = th.xend - th.x0 + 2 * (T - 1) * M;
        // the chunk's range of each point table (issued here, so that its
        // latency overlaps the per-plane loads below)
        const int cf = max(th.cbase, 0), cl = min(th.cbase + span, a.nx);
        const bool iwant = STAGE && a.inj.cnt > 0 && cf < cl;
        const bool rwant = STAGE && a.rec.cnt > 0 && cf < cl;
        const int ib = iwant ? a.inj.xptr[cf] : 0, ie = iwant ? a.inj.xptr[cl] : 0;
        const int rb = rwant ? a.rec.xptr[cf] : 0, re = rwant ? a.rec.xptr[cl] : 0;
        for (int j = threadIdx.x; j < span; j += G::NT) {
            const int c = th.cbase + j;
            const bool cin = (unsigned)c < (unsigned)a.nx;
            sm.px[j] = cin ? a.px[c] : 0.0f;
            sm.ixb[j] = sm.ixe[j] = 0;
            if (cin && a.inj.cnt > 0) {
                const int b = a.inj.xptr[c], e = a.inj.xptr[c + 1];
                const int32_t *bx = a.inj.box + 4 * c;
                if (b < e && bx[1] >= y1 && bx[0] < y1 + G::RY && bx[3] >= z1 && bx[2] < z1 + G::RZ) {
                    sm.ixb[j] = b;
                    sm.ixe[j] = e;
                }
            }
            sm.rxb[j] = sm.rxe[j] = 0;
            if (cin && a.rec.cnt > 0) {
                const int b = a.rec.xptr[c], e = a.rec.xptr[c + 1];
                const int32_t *bx = a.rec.box + 4 * c;
                if (b < e && bx[1] >= y1 + G::H1 && bx[0] < y1 + G::H1 + G::TY &&
                    bx[3] >= z1 + G::H1 && bx[2] < z1 + G::H1 + G::TZ) {
                    sm.rxb[j] = b;
                    sm.rxe[j] = e;
                }
            }
        }
        // Stage the chunk's point entries (all planes it computes; the table is
        // sorted by plane, so they are one contiguous range) in LDS.  The loop
        // then touches only LDS for points: a global load or store inside it
        // would make the next plane's wait also cover the prefetched loads (the
        // counter is in order), draining the pipeline on every plane that holds
        // points, and its per-entry work runs across lanes.
        if constexpr (STAGE) {
            const bool istg = iwant && ie - ib <= PC, rstg = rwant && re - rb <= PC;
            if (threadIdx.x == 0) {
                sm.i0 = istg ? ib : -1;
                sm.r0 = rstg ? rb : -1;
            }
            if (istg)
                for (int j = threadIdx.x; j < ie - ib; j += G::NT) {
                    sm.iyz[j] = a.inj.yz[ib + j];
                    sm.isc[j] = a.inj.scale[ib + j];
                    const int id = a.inj.id[ib + j];
#pragma unroll
                    for (int t = 0; t < T; ++t)
                        sm.iamp[t][j] = a.amp[(a.abase + (int64_t)a.adir * (a.step0 + t)) * a.inj.stride + id];
                }
            if (rstg) {
                const bool ent = a.rec.etr != nullptr;
                for (int j = threadIdx.x; j < re - rb; j += G::NT) {
                    const int yz = a.rec.yz[rb + j], x = a.rec.xe[rb + j];
                    const int y = yz / a.nzp, rr = y - y1, cz = yz - y * a.nzp - z1;
                    const bool core = rr >= G::H1 && rr < G::RY - G::H1 && cz >= G::H1 &&
                                      cz < G::RZ - G::H1 && x >= th.x0 && x < th.xend;
                    sm.rcode[j] = core ? ((rr / PY) << 16) | ((rr % PY) << 8) | cz : -1;
                    sm.rdst[j] = ent ? rb + j : a.rec.id[rb + j];
                }
            }
        }
        // (the first barrier of the loop orders these writes before any read)

        // level t's queue of u^{t-1}: planes c_t - M .. c_t + M (the fused Born
        // kernel keeps the perturbation's queue in entry T)
        float qu[T + F - 1][PY][QS];
#pragma unroll
        for (int t = 0; t < T + F - 1; ++t)
#pragma unroll
            for (int r = 0; r < PY; ++r)
#pragma unroll
                for (int j = 0; j < QS; ++j) qu[t][r][j] = 0.0f;

        float acc[(MODE == kImaging) ? PY : 1][(MODE == kImaging) ? G::AQ : 1];
        if constexpr (MODE == kImaging) {
#pragma unroll
            for (int r = 0; r < PY; ++r)
#pragma unroll
                for (int j = 0; j < G::AQ; ++j) acc[r][j] = 0.0f;
        }

        const int ibeg = th.x0 - T * M;
        th.iend = th.xend + T * M;
        const int64_t N = (int64_t)a.nx * a.sxy;

        // The first 2M iterations would only fill level 1's queue (no level
        // computes a plane it needs before then): load those 2M head planes at
        // once, all in flight together, and start the loop behind them.  The
        // queue then holds, before the first push, planes istart - 2M - 1 + j
        // in logical entries j = 1 .. 2M (entry 0 is never read).
        const int istart = ibeg + 2 * M;
#pragma unroll
        for (int j = 0; j < 2 * M; ++j) {
            const int ph = plane(th, ibeg + j);
            const auto rh = plane_rsrc(a.u0, ph, a.sxy, (unsigned)ph < (unsigned)a.nx);
#pragma unroll
            for (int r = 0; r < PY; ++r) qu[0][r][pjb<0>(j + 1)] = bload(rh, th.bo[r]);
            if constexpr (FUSED) {
                const auto rh2 = plane_rsrc(a.u0b, ph, a.sxy, (unsigned)ph < (unsigned)a.nx);
#pragma unroll
                for (int r = 0; r < PY; ++r) qu[T][r][pjb<0>(j + 1)] = bload(rh2, th.bo[r]);
            }
        }

        Pre pf[NS];  // slot (i - istart) mod NS holds the loads of iteration i
#pragma unroll
        for (int d = 0; d < ((NS > 1) ? NS - 1 : 1); ++d) load(a, th, pf[d], istart + d);
        for (int i0 = istart; i0 < th.iend; i0 += UNROLL) block<0>(a, sm, th, qu, acc, pf, i0, N);

        // the samples the staged receivers recorded, one trace row per level
        if (STAGE && re > rb && __builtin_amdgcn_readfirstlane(sm.r0) >= 0) {
            __syncthreads();
            const bool ent = a.rec.etr != nullptr;
            for (int j = threadIdx.x; j < re - rb; j += G::NT) {
                if (sm.rcode[j] < 0) continue;
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    const int64_t row = a.rbase + (int64_t)a.rdir * (a.step0 + t);
                    float *orow = ent ? a.rec.etr + row * a.rec.cnt : a.rec_out + row * a.rec.stride;
                    orow[sm.rdst[j]] = sm.rval[t][j];
                }
            }
        }
    }

    // Iterations i0 + PH .. i0 + UNROLL - 1 of the x loop (one per phase).  Each
    // iteration publishes the y/z planes of all T levels first (level t needs
    // u^{t-1} at plane c_t, which entered its queue M iterations ago), so one
    // barrier per iteration serves every level.
    template <int PH, class QU, class ACC>
    __device__ static __forceinline__ void block(const SweepArgs &a, Smem &sm, const Thread &th,
                                                 QU &qu, ACC &acc, Pre (&pf)[NS], int i0, int64_t N)
    {
        if constexpr (PH < UNROLL) {
            const int i = i0 + PH;
            if (i < th.iend) {
                if constexpr (NS == 1) {
                    const Pre cur = pf[0];
                    load(a, th, pf[0], i + 1);
                    step<PH>(a, sm, th, qu, acc, cur, i, N);
                } else {
                    load(a, th, pf[(PH + NS - 1) % NS], i + NS - 1);
                    step<PH>(a, sm, th, qu, acc, pf[PH % NS], i, N);
                }
                block<PH + 1>(a, sm, th, qu, acc, pf, i0, N);
            }
        }
    }

    // One iteration: publish, barrier, the T levels.
    template <int PH, class QU, class ACC>
    __device__ static __forceinline__ void step(const SweepArgs &a, Smem &sm, const Thread &th,
                                                QU &qu, ACC &acc, const Pre &cur, int i, int64_t N)
    {
        {
            {
                const int par = i & 1;
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
                S = sm.s0[0][par];
#pragma unroll
                for (int s = 0; s < G::HS; ++s) {
                    int row, col;
                    if (halo_pos(threadIdx.x + s * G::NT, row, col)) S[row * G::L0W + col] = P.halo[s];
                }
                if constexpr (FUSED) {
                    float *S2 = sm.s0[1][par];
#pragma unroll
                    for (int s = 0; s < G::HS; ++s) {
                        int row, col;
                        if (halo_pos(threadIdx.x + s * G::NT, row, col)) S2[row * G::L0W + col] = P.halo2[s];
                    }
#pragma unroll
                    for (int r = 0; r < PY; ++r)
                        S2[(th.wv * PY + r + M) * W + th.lane + COFF] = qu[T][r][pjb<PH>(M + 1)];
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
        if (h < 2 * M * G::RZ) {
            const int band = h / G::RZ;
            col = M + (h - band * G::RZ);
            row = band < M ? band : band + G::RY;
        } else {
            const int h2 = h - 2 * M * G::RZ;
            row = M + h2 / (2 * M);
            const int cj = h2 % (2 * M);
            col = cj < M ? cj : cj + G::RZ;
        }
        return h < G::NHALO;
    }

    // Offset of owned point r for output stores: beyond the plane unless the
    // point is inside the output tile (computed per use: a register per row
    // held for the whole pass costs occupancy at M = 8).
    __device__ static __forceinline__ uint32_t out_off(const Thread &th, int r)
    {
        return th.core[r] ? th.bo[r] : kOutside;
    }

    // Plane at stream position i.
    __device__ static __forceinline__ int plane(const Thread &th, int i)
    {
        return th.refl < 0 ? i : th.refl - i;
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
        const int ph = plane(th, i);
        const auto rh = plane_rsrc(a.u0, ph, a.sxy, (unsigned)ph < (unsigned)a.nx && i < th.iend);
#pragma unroll
        for (int r = 0; r < PY; ++r) P.head[r] = bload(rh, th.bo[r]);
        const int c1 = plane(th, i - M);
        const bool l1 = needed(a, th, 1, c1);
        const auto rc = plane_rsrc(a.u0, c1, a.sxy, l1);
#pragma unroll
        for (int s = 0; s < G::HS; ++s) P.halo[s] = bload(rc, th.hb[s]);
        const auto rm = plane_rsrc(a.um, c1, a.sxy, l1);
#pragma unroll
        for (int r = 0; r < PY; ++r) P.up1[r] = bload<LP>(rm, th.bo[r]);
        if constexpr (FUSED) {
            const auto rh2 = plane_rsrc(a.u0b, ph, a.sxy, (unsigned)ph < (unsigned)a.nx && i < th.iend);
#pragma unroll
            for (int r = 0; r < PY; ++r) P.head2[r] = bload(rh2, th.bo[r]);
            const auto rc2 = plane_rsrc(a.u0b, c1, a.sxy, l1);
#pragma unroll
            for (int s = 0; s < G::HS; ++s) P.halo2[s] = bload(rc2, th.hb[s]);
            const auto rm2 = plane_rsrc(a.umb, c1, a.sxy, l1);
            const auto rs = plane_rsrc(a.bs, c1, a.sxy, l1);
#pragma unroll
            for (int r = 0; r < PY; ++r) {
                P.up2[r] = bload<LP>(rm2, th.bo[r]);
                P.bs[r] = bload<LP>(rs, th.bo[r]);
            }
        }
#pragma unroll
        for (int t = 1; t <= T; ++t) {
            const int ct = plane(th, i - t * M);
            const auto rq = plane_rsrc(a.q, ct, a.sxy, needed(a, th, t, ct));
#pragma unroll
            for (int r = 0; r < PY; ++r) P.q[t - 1][r] = bload<LP>(rq, th.bo[r]);
        }
        if constexpr (BORN) {
            const auto rs = plane_rsrc(a.bs, c1, a.sxy, l1);
            const auto rd = plane_rsrc(a.d2 + a.dslot0 * (int64_t)a.nx * a.sxy, c1, a.sxy, l1);
#pragma unroll
            for (int r = 0; r < PY; ++r) {
                P.bs[r] = bload<LP>(rs, th.bo[r]);
                P.bd[r] = bload<kStream>(rd, th.bo[r]);
            }
        }
        if constexpr (IMG) {
            // only planes this chunk owns are read (and later written); offsets
            // of points outside the output tile are beyond the plane
            const bool o1 = c1 >= th.x0 && c1 < th.xend;
            const auto rg = span_rsrc(a.g + (int64_t)(o1 ? c1 : 0) * a.sxy, a.sxy * 4, o1);
#pragma unroll
            for (int r = 0; r < PY; ++r) P.g[r] = bload<LP>(rg, out_off(th, r));
            const int64_t N = (int64_t)a.nx * a.sxy;
#pragma unroll
            for (int t = 1; t <= T; ++t) {
                const int ct = plane(th, i - t * M);
                const bool ot = ct >= th.x0 && ct < th.xend;
                const float *dp = a.d2 + (a.dslot0 + (int64_t)a.ddir * (t - 1)) * N +
                                  (int64_t)(ot ? ct : 0) * a.sxy;
                const auto rd = span_rsrc(dp, a.sxy * 4, ot);
#pragma unroll
                for (int r = 0; r < PY; ++r) P.d2[t - 1][r] = bload<kStream>(rd, out_off(th, r));
            }
        }
    }

    // Process level t (1..T) at plane c = i - t*M, then recurse to level t+1.
    template <int t, int PH, class QU, class ACC>
    __device__ static __forceinline__ void level(const SweepArgs &a, Smem &sm, const Thread &th,
                                                 QU &qu, ACC &acc, float (&val)[PY], const Pre &P,
                                                 int i, int par, int64_t N)
    {
        const int c = plane(th, i - t * M);
        const int lane = th.lane, wv = th.wv;
        // push the newest plane (c + M) into level t's queue
#pragma unroll
        for (int r = 0; r < PY; ++r) {
            if constexpr (ROT) {
                qu[t - 1][r][PH] = val[r];  // newest entry; the slot held one no longer used
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
        if constexpr (FUSED) {
#pragma unroll
            for (int r = 0; r < PY; ++r) {
                if constexpr (ROT) {
                    qu[T][r][PH] = P.head2[r];
                } else {
#pragma unroll
                    for (int j = 0; j + 1 < Q; ++j) qu[T][r][j] = qu[T][r][j + 1];
                    qu[T][r][Q - 1] = P.head2[r];
                }
            }
        }
        const float *S;
        if constexpr (t == 1) S = sm.s0[0][par];
        else S = sm.s1[t - 2][par];

        // level t's region: owned region shrunk by M (t - 1)
        constexpr int lo = M * (t - 1);
        const bool xin = (unsigned)c < (unsigned)a.nx;
        const bool zreg = lane >= lo && lane < G::RZ - lo;
        float out[PY];
        float out2[FUSED ? PY : 1];  // fused Born: the perturbation's new level
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
                float num = fmaf(qv, lap, fmaf(eta - 1.0f, up, 2.0f * uc));
                if constexpr (BORN) num = fmaf(P.bs[r], P.bd[r], num);
                out[r] = active ? damped(num, eta) : 0.0f;
            }
            const int step = a.step0 + t - 1;
            // point entries of this plane (table order; entries at one node
            // are applied in that order), from LDS when the chunk's entries
            // were staged
            {
                const int jb = __builtin_amdgcn_readfirstlane(sm.ixb[tj]);
                const int je = __builtin_amdgcn_readfirstlane(sm.ixe[tj]);
                if (jb < je) {
                    const float *arow = a.amp + (a.abase + (int64_t)a.adir * step) * a.inj.stride;
                    if constexpr (STAGE) {
                        // staged: the plane's entries are sorted by (y, z), so
                        // each thread finds the run of entries at its own node
                        // by binary search and applies it in table order
                        const int s0 = __builtin_amdgcn_readfirstlane(sm.i0);
                        const int kb = jb - s0, ke = je - s0;
#pragma unroll
                        for (int r = 0; r < PY; ++r) {
                            const int rr = wv * PY + r;
                            const bool active = th.din[r] && zreg && rr >= lo && rr < G::RY - lo;
                            const int key = (int)(th.bo[r] >> 2);
                            int kl = kb, kh = ke;
                            while (kl < kh) {
                                const int km = (kl + kh) >> 1;
                                if (sm.iyz[km] < key) kl = km + 1;
                                else kh = km;
                            }
                            for (int k = kl; active && k < ke && sm.iyz[k] == key; ++k)
                                out[r] = fmaf(sm.isc[k], sm.iamp[t - 1][k], out[r]);
                        }
                    } else {
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
            }
            if constexpr (FUSED) {
                // the perturbation: the same update of its own field, plus the
                // Born source s d2 inside the division, d2 the background's
                // second difference at this point (after its injection)
                const float *S2 = sm.s0[1][par];
                float colv[PY + 2 * M];
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    colv[j] = S2[(wv * PY - M + j + OFF) * W + lane + COFF];
                    colv[M + PY + j] = S2[(wv * PY + PY + j + OFF) * W + lane + COFF];
                }
#pragma unroll
                for (int r = 0; r < PY; ++r) colv[M + r] = qu[T][r][pj<PH>(M)];
#pragma unroll
                for (int r = 0; r < PY; ++r) {
                    const int rr = wv * PY + r;
                    const bool active = th.din[r] && zreg && rr >= lo && rr < G::RY - lo;
                    const float d2 = fmaf(-2.0f, qu[0][r][pj<PH>(M)], out[r]) + P.up1[r];
                    const float uc = qu[T][r][pj<PH>(M)];
                    const float *row = S2 + (rr + OFF) * W + lane + COFF;
                    float lap = 0.0f;
#pragma unroll
                    for (int k = 1; k <= M; ++k) {
                        const float xs = qu[T][r][pj<PH>(M - k)] + qu[T][r][pj<PH>(M + k)];
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
                    const float qv = P.q[0][r];
                    const float eta = qv * (pxv + th.pyz[r]);
                    float num = fmaf(qv, lap, fmaf(eta - 1.0f, P.up2[r], 2.0f * uc));
                    num = fmaf(P.bs[r], d2, num);
                    out2[r] = active ? damped(num, eta) : 0.0f;
                }
            }
            // the field receivers sample: the perturbation in the fused Born pass
            float recv[PY];
#pragma unroll
            for (int r = 0; r < PY; ++r) {
                if constexpr (FUSED) recv[r] = out2[r];
                else recv[r] = out[r];
            }
            // receivers record the levels a workgroup owns: its chunk's planes,
            // and in the first phase of a split pass every plane level 1
            // computes (the walk in memory only: such passes do not stage)
            bool rown = c >= th.x0 && c < th.xend;
            if constexpr (T == 2 && t == 1 && MODE == kPlain) rown = rown || a.split != 0;
            if (rown) {
                const int jb = __builtin_amdgcn_readfirstlane(sm.rxb[tj]);
                const int je = __builtin_amdgcn_readfirstlane(sm.rxe[tj]);
                if (jb < je) {
                    // points between nodes record the value at every entry
                    // (summed per point after the sweep); points on nodes
                    // write their trace sample
                    const int64_t row = a.rbase + (int64_t)a.rdir * step;
                    const bool ent = a.rec.etr != nullptr;
                    float *orow = ent ? a.rec.etr + row * a.rec.cnt : a.rec_out + row * a.rec.stride;
                    const float rs = ent ? 1.0f : a.rscale;
                    if constexpr (STAGE) {
                        const int s0 = __builtin_amdgcn_readfirstlane(sm.r0);
                        const int sw = __builtin_amdgcn_readfirstlane(wv);
                        // staged: lane k takes entry j0 + k and fetches the sample
                        // from the lane that computed it (one permute per row);
                        // the samples stay in LDS until the end of the chunk
                        for (int j0 = jb; j0 < je; j0 += 64) {
                            const int k = j0 + lane - s0;
                            const int code = (lane < je - j0) ? sm.rcode[k] : -1;
                            const int rk = (code >> 8) & 0xff, lk = code & 0xff;
                            float v = 0.0f;
#pragma unroll
                            for (int r = 0; r < PY; ++r) {
                                const float o = __int_as_float(
                                    __builtin_amdgcn_ds_bpermute(lk << 2, __float_as_int(recv[r])));
                                if (r == rk) v = o;
                            }
                            if (code >= 0 && (code >> 16) == sw) sm.rval[t - 1][k] = v * rs;
                        }
                    } else {
                        for (int j = jb; j < je; ++j) {
                            const uint32_t p = (uint32_t)a.rec.yz[j] * 4u;
                            const int dst = ent ? j : a.rec.id[j];
#pragma unroll
                            for (int r = 0; r < PY; ++r)
                                if (th.core[r] && th.bo[r] == p) orow[dst] = recv[r] * rs;
                        }
                    }
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < PY; ++r) out[r] = 0.0f;
            if constexpr (FUSED) {
#pragma unroll
                for (int r = 0; r < PY; ++r) out2[r] = 0.0f;
            }
        }
        if constexpr (T == 2 && t == 1 && MODE == kPlain) {
            // first phase of a split pass: level 1 is stored on the chunk's
            // planes outside level 2's range too (the second phase reads it);
            // an empty resource otherwise, so the store is issued unconditionally
            const bool wing = a.split != 0 && xin && (c < th.x0 || c >= th.xend) && needed(a, th, 1, c);
            const auto rw = plane_rsrc(a.o2, c, a.sxy, wing);
#pragma unroll
            for (int r = 0; r < PY; ++r) bstore<kStream>(rw, out_off(th, r), out[r]);
        }
        // gradient support (outside the branch above, so that every memory
        // operation of the iteration is issued unconditionally; own planes are
        // always needed)
        const bool own = c >= th.x0 && c < th.xend;
        if constexpr (MODE == kSaveD2) {
            const float *dp = a.d2 + (a.dslot0 + (int64_t)a.ddir * (t - 1)) * N +
                              (int64_t)(own ? c : 0) * a.sxy;
            const auto rd = span_rsrc(dp, a.sxy * 4, own);
#pragma unroll
            for (int r = 0; r < PY; ++r) {
                float um;
                if constexpr (t == 1) um = P.up1[r];
                else um = qu[t - 2][r][pj<PH>(0)];
                bstore<kStream>(rd, out_off(th, r), fmaf(-2.0f, qu[t - 1][r][pj<PH>(M)], out[r]) + um);
            }
        }
        if constexpr (MODE == kImaging) {
            // g (level 1's plane) and d2 were loaded with this iteration's other
            // inputs; points outside the output tile read 0 and are not stored
            const auto rg = span_rsrc(a.g + (int64_t)(own ? c : 0) * a.sxy, a.sxy * 4, own);
            constexpr int J = (T - t) * M;
#pragma unroll
            for (int r = 0; r < PY; ++r) {
                float base;
                if constexpr (t == 1) base = P.g[r];
                else base = acc[r][J];
                const float nv = fmaf(out[r], P.d2[t - 1][r], base);
                if constexpr (t == T) bstore<LP>(rg, out_off(th, r), nv);
                else acc[r][J] = nv;
            }
        }

        if constexpr (t == T) {
            // the pass's outputs at plane c: u^{n+T} and (T >= 2) u^{n+T-1}
            const bool outp = xin && own;
            const auto r1 = plane_rsrc(a.o1, c, a.sxy, outp);
#pragma unroll
            for (int r = 0; r < PY; ++r) bstore<kStream>(r1, out_off(th, r), out[r]);
            if constexpr (FUSED) {
                const auto r2 = plane_rsrc(a.o2, c, a.sxy, outp);
#pragma unroll
                for (int r = 0; r < PY; ++r) bstore<kStream>(r2, out_off(th, r), out2[r]);
            }
            if constexpr (T >= 2) {
                const auto r2 = plane_rsrc(a.o2, c, a.sxy, outp);
#pragma unroll
                for (int r = 0; r < PY; ++r) bstore<kStream>(r2, out_off(th, r), qu[T - 1][r][pj<PH>(M)]);
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
template <int M, int T, int PY, int NW, int MODE, bool ISO, bool NTL, bool PS>
__global__ __launch_bounds__(64 * NW) void k_stream(SweepArgs a)
{
    using K = StreamKernel<M, T, PY, NW, MODE, ISO, NTL, PS>;
    __shared__ typename K::Smem sm;
    K::run(a, sm, blockIdx.x, gridDim.x);
}

// Grouped pass: the workgroups walk the flat tile range of all the entries (one
// per shot) of a batch, one tile each when the grid covers the range, else
// persistently.  Workgroup b runs on XCD b % 8; when the
// grid is a multiple of 8, the items of one round are dealt so that each XCD
// takes a contiguous block of them (neighbouring tiles of one shot share that
// XCD's L2).
template <int M, int T, int PY, int NW, int MODE, bool ISO, bool NTL, bool PS>
__global__ __launch_bounds__(64 * NW) void k_stream_grouped(const GroupEntry *__restrict__ list,
                                                            int nlist, int total)
{
    using K = StreamKernel<M, T, PY, NW, MODE, ISO, NTL, PS>;
    __shared__ typename K::Smem sm;
    const int b = blockIdx.x;
    const int first = ((gridDim.x & 7) == 0) ? (b & 7) * (gridDim.x >> 3) + (b >> 3) : b;
    // The table is read through the constant address space: it does not change
    // during the launch, so the compiler may keep the entry's fields in scalar
    // registers across the whole tile instead of reloading them after every
    // store of the streaming loop.
    // (The host pass only sees a stub of this body; it has no constant
    // address space, so it reads the table directly.)
#if defined(__HIP_DEVICE_COMPILE__)
    using CEntry = const __attribute__((address_space(4))) GroupEntry;
    CEntry *clist = (CEntry *)list;
#else
    const GroupEntry *clist = list;
#endif
    for (int item = first; item < total; item += gridDim.x) {
        int e = 0;
        while (e + 1 < nlist && clist[e + 1].tile0 <= item) ++e;
        const SweepArgs a = clist[e].a;
        K::run(a, sm, item - clist[e].tile0, a.ntz * a.nty * a.ntx);
        __syncthreads();  // the next tile rewrites the LDS tables and planes
    }
}

// Launch helpers shared by the generated entry files.  The forms differ in the
// cache policy of once-per-step loads (a.ntl, or ntl for a grouped launch) and
// in the point walk (a.ps / ps: staged, for configurations that can stage);
// all forms give identical results.
template <int M, int T, int PY, int NW, int MODE, bool ISO, bool NTL>
void issue_stream_p(const SweepArgs &a, dim3 grid, dim3 block, hipStream_t s)
{
    if constexpr (points_stageable(M, T, PY, NW)) {
        if (a.ps) {
            hipLaunchKernelGGL((k_stream<M, T, PY, NW, MODE, ISO, NTL, true>), grid, block, 0, s, a);
            return;
        }
    }
    hipLaunchKernelGGL((k_stream<M, T, PY, NW, MODE, ISO, NTL, false>), grid, block, 0, s, a);
}

template <int M, int T, int PY, int NW, int MODE, bool ISO>
void issue_stream(const SweepArgs &a, dim3 grid, dim3 block, hipStream_t s)
{
    if (a.ntl) issue_stream_p<M, T, PY, NW, MODE, ISO, true>(a, grid, block, s);
    else issue_stream_p<M, T, PY, NW, MODE, ISO, false>(a, grid, block, s);
}

template <int M, int T, int PY, int NW, int MODE, int F>
bool entry_launch(const SweepArgs &a, hipStream_t s)
{
    const dim3 grid(a.ntz * a.nty * a.ntx), block(64 * NW);
    if (a.w.iso) {
        issue_stream<M, T, PY, NW, MODE, true>(a, grid, block, s);
        return true;
    }
    if constexpr ((F & 1) != 0) {
        issue_stream<M, T, PY, NW, MODE, false>(a, grid, block, s);
        return true;
    }
    return false;
}

template <int M, int T, int PY, int NW, int MODE, bool ISO, bool NTL>
void issue_grouped_p(bool ps, const GroupEntry *list, int nlist, int total, dim3 grid, dim3 block,
                     hipStream_t s)
{
    if constexpr (points_stageable(M, T, PY, NW)) {
        if (ps) {
            hipLaunchKernelGGL((k_stream_grouped<M, T, PY, NW, MODE, ISO, NTL, true>), grid, block, 0,
                               s, list, nlist, total);
            return;
        }
    }
    hipLaunchKernelGGL((k_stream_grouped<M, T, PY, NW, MODE, ISO, NTL, false>), grid, block, 0, s,
                       list, nlist, total);
}

template <int M, int T, int PY, int NW, int MODE, bool ISO>
void issue_grouped(bool ntl, bool ps, const GroupEntry *list, int nlist, int total, dim3 grid,
                   dim3 block, hipStream_t s)
{
    if (ntl) issue_grouped_p<M, T, PY, NW, MODE, ISO, true>(ps, list, nlist, total, grid, block, s);
    else issue_grouped_p<M, T, PY, NW, MODE, ISO, false>(ps, list, nlist, total, grid, block, s);
}

template <int M, int T, int PY, int NW, int MODE, int F>
bool entry_launch_group(bool iso, bool ntl, bool ps, const GroupEntry *list, int nlist, int total,
                        int grid, hipStream_t s)
{
    if constexpr ((F & 2) != 0) {
        const dim3 g(grid), block(64 * NW);
        if (iso) {
            issue_grouped<M, T, PY, NW, MODE, true>(ntl, ps, list, nlist, total, g, block, s);
            return true;
        }
        if constexpr ((F & 1) != 0) {
            issue_grouped<M, T, PY, NW, MODE, false>(ntl, ps, list, nlist, total, g, block, s);
            return true;
        }
    }
    return false;
}

// Resident workgroups per CU of the single-pass or the grouped kernel (0 if the
// requested form is not compiled).  All cache-policy and point-walk forms use
// the same registers and LDS closely enough that the plain form stands for them.
template <int M, int T, int PY, int NW, int MODE, int F>
int entry_occupancy(bool iso, bool grouped)
{
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    const void *fn = nullptr;
    if (grouped) {
        if constexpr ((F & 2) != 0) {
            if (iso)
                fn = reinterpret_cast<const void *>(&k_stream_grouped<M, T, PY, NW, MODE, true, false, false>);
            else if constexpr ((F & 1) != 0)
                fn = reinterpret_cast<const void *>(&k_stream_grouped<M, T, PY, NW, MODE, false, false, false>);
        }
    } else {
        if (iso) fn = reinterpret_cast<const void *>(&k_stream<M, T, PY, NW, MODE, true, false, false>);
        else if constexpr ((F & 1) != 0)
            fn = reinterpret_cast<const void *>(&k_stream<M, T, PY, NW, MODE, false, false, false>);
    }
    if (fn) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, 64 * NW, 0);
    return e == hipSuccess ? n : 0;
}

}  // namespace fdw
