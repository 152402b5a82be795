// fd_wave.h -- two-level time blocks without redundant halos: neighbouring
// workgroups exchange the intermediate level through memory.
//
// As in the overlapped time blocks of fd_stream.h, level 2 of a pass is
// evaluated behind level 1 along x, skewed by the stencil radius so that every
// dependence points backwards in the stream (paper Secs. 5.2-5.4).  Here each
// workgroup computes both levels on its own (y, z) tile only, over the whole x
// axis, so no point is computed twice.  Level 2 at a tile's edge needs level 1
// on the M-wide ring around the tile, which the four neighbouring workgroups
// compute.  Level 1 is the pass's u^{n+1}, stored in full anyway: it is
// stored with device-coherent stores, and each workgroup publishes after
// every iteration a progress counter; a workgroup loads the ring of a level-1
// plane from memory, with device-coherent loads, once its neighbours'
// counters show that plane stored.  A pass thus moves u^n, u^{n-1} and q in,
// both output levels out, and the level-1 rings (served mostly by the
// Infinity Cache, where the neighbours' stores just went).  The paper's CPU
// code gets the same effect from the sequential order of its skewed tiles
// (Sec. 5.5); on the GPU the tiles run concurrently, so the order is enforced
// by the counters.
//
// Visibility.  The device-coherent form of a buffer access (the SC1
// cache-policy bit, the form the compiler gives device-scope atomics) writes
// through to, and reads from, the point of coherence of all XCDs; no
// cache-wide write-back or invalidation is needed.  Loads are issued D
// iterations ahead: iteration j + 1 issues the loads of iteration j + 1 + D
// after the stores of iteration j, and waits for them in iteration j + 1 + D;
// vector memory operations complete in issue order, so by the barrier of
// iteration k every store of iteration k - D - 1 and before has completed.
// Thread 0 then stores the counter k - D ("iterations below k - D complete"),
// also device-coherently, every P-th iteration; each counter has a 256-byte
// line of its own.  A reader polls its neighbours' counters before
// issuing the ring loads they gate, and only when the values it last saw would
// not admit them.
//
// Progress.  The host launches a pass only when all of its workgroups can be
// resident at once (occupancy x compute units).  A workgroup at iteration i
// waits only for neighbours to have reached iteration i + 2D + P - (M + E),
// below its own (M + E >= 2D + P + 1): the workgroup furthest behind never
// waits, so every wait ends.
// Each wait is still bounded (kWaveSpin polls); a wait that runs out sets the
// pass's error word, which every later wait checks, so a launch that somehow
// did not run all of its workgroups at once ends with an error instead of a
// hang.
//
// The per-point FP32 operation order is that of the untiled kernel
// (fd_naive.hip), so the results are bit-identical to every other variant.
#pragma once

#include "fd_stream.h"

namespace fdw {

// Cache policy of the exchanged level (device-coherent: SC1).
constexpr int kCoherent = 16;

// Prefetch distance: iteration i issues the loads of iteration i + kWaveAhead.
// Measured at 512^3 so 8 (2 x 8 tiles, GPts/s): distance 1 317, 2 327, 3 339,
// 4 329, 5 328, each with the shortest lag the counters allow (2D + 3); at
// so 4, distance 2 (lag 7) 310 against distance 3 (lag 11) 387.
constexpr int kWaveAhead = 3;

// Level 2 lags level 1 by M + E planes; the E extra planes are slack that lets
// a neighbour's counter run that many iterations late without a wait.  More
// slack costs registers (every queue holds 2M + 1 + E planes) and pays while
// they last.  Measured at 512^3 (2 x 8 tiles, GPts/s), counters every second
// iteration: so 4, lag 11 / 13 / 15 / 17 / 19: 389 / 399 / 411 / 425 / 425;
// so 8, lag 11 / 15 / 17 / 19: 350 / 363 / 363 / 364.  Every eighth
// iteration (below): so 4, lag 17 / 19: 428 / 441; so 8: 378 / 367.  Tiles of
// two rows per thread take the long lags up to M = 4; the other shapes keep
// the short one (their queues would not fit the registers).
constexpr int kWaveLagShort = 11;
constexpr int kWaveLagLong = 17;    // two-row tiles, M = 3, 4
constexpr int kWaveLagLonger = 19;  // two-row tiles, M <= 2
constexpr int wave_lag(int M, int PY)
{
    return PY > 2 || M > 4 ? kWaveLagShort : M > 2 ? kWaveLagLong : kWaveLagLonger;
}
constexpr int wave_extra(int M, int PY) { return M >= wave_lag(M, PY) ? 0 : wave_lag(M, PY) - M; }

// Counters are published every P-th iteration (a device-coherent store in the
// wave's in-order memory queue); the lag must cover the staler counts:
// M + E >= 2D + P + 1.  Measured at 512^3 with lag 17 (2 x 8 tiles, GPts/s):
// P = 2 / 4 / 8: so 8 364 / 368-372 / 379-381, so 4 420 / 426-430 / 428;
// P = 16 (lag 23 / 25, M = 2 only: M = 4 spills): so 4 414 / 427.  With the
// short lag P = 4 ran slower than P = 2 (so 4, 4 x 4 tiles: 306 against 320).
constexpr int kWavePubShort = 2;
constexpr int kWavePubLong = 8;  // with either long lag
static_assert(kWaveLagShort >= 2 * kWaveAhead + kWavePubShort + 1 &&
                  kWaveLagLong >= 2 * kWaveAhead + kWavePubLong + 1 &&
                  kWaveLagLonger >= 2 * kWaveAhead + kWavePubLong + 1,
              "level 2 must trail level 1 by more than the counters lag");
constexpr int wave_pub(int M, int PY) { return wave_lag(M, PY) > kWaveLagShort ? kWavePubLong : kWavePubShort; }

// Bound of one wait, in polls of the neighbours' counters (a poll is one
// device-coherent load round trip plus a short sleep).
constexpr int kWaveSpin = 1 << 18;

template <int M, int PY, int NW, bool ISO>
struct WaveKernel {
    static constexpr int NT = 64 * NW;       // threads per workgroup
    static constexpr int RY = NW * PY;       // tile rows (y)
    static constexpr int RZ = 64;            // tile columns (z)
    static constexpr int E = wave_extra(M, PY);
    static constexpr int PUB = wave_pub(M, PY);  // counter publication interval P
    static_assert((PUB & (PUB - 1)) == 0 && M + E >= 2 * kWaveAhead + PUB + 1, "lag too short for the interval");
    static constexpr int Q = 2 * M + 1 + E;  // queue length of u^n and of level 1 along x
    static constexpr int QQ = M + E + 1;     // queue of q: level 1's plane down to level 2's
    // The x loop is unrolled by U = D + 1 (D the prefetch distance), with U
    // prefetch slots: phase PH consumes slot PH and refills the slot the
    // previous phase consumed, so every slot index is a compile-time constant
    // and no loaded register is copied (a copy would wait for the loads in
    // flight).  Phase PH also pushes into slot (queue length) + PH of each
    // register queue, so a queue's window of planes sits at slots
    // [PH, PH + length) before that push and [PH + 1, PH + 1 + length) after
    // it; the slots move back by U once per body (one register move per slot
    // every U iterations instead of every iteration).
    static constexpr int D = kWaveAhead;
    static constexpr int U = D + 1;
    static constexpr int QX = Q + U, QQX = QQ + U;  // slots: the last push lands in Q + U - 1
    static constexpr int LW = RZ + 2 * M;    // LDS plane with its M-wide ring
    static constexpr int LH = RY + 2 * M;
    // the ring without its corners (the star stencil never reads them)
    static constexpr int NHALO = 2 * M * RZ + RY * 2 * M;
    static constexpr int HS = (NHALO + NT - 1) / NT;

    struct Smem {
        float s0[2][LH * LW];  // u^n at level 1's plane, with its ring (two parities)
        float s1[2][LH * LW];  // level 1 at level 2's plane, with its ring
    };

    // Loads of one iteration, issued D iterations ahead.  The per-plane
    // scalars of both levels (SweepArgs::ptab: sponge profile, point table
    // ranges, flags) are one vector load, lane k holding slot k of level 1's
    // plane and lane kTab + k that of level 2's (read back with readlane): a
    // scalar load would be waited for by the barrier's LDS wait (one counter
    // covers both), exposing its latency every iteration.
    struct Pre {
        float head[PY];       // u^n at the head plane i
        float h0[HS];         // u^n ring at level 1's plane
        float um[PY];         // u^{n-1} at level 1's plane
        float q1[PY];         // q at level 1's plane (level 2 takes it M + E iterations later)
        float h1[HS];         // level-1 ring at level 2's plane (the neighbours' values)
        int tab;              // lanes 0-7: level 1's plane, 8-15: level 2's (kPx .. kRd)
    };
    enum { kPx = 0, kIb = 1, kIe = 2, kRb = 3, kRe = 4, kFl = 5, kRy = 6, kRd = 7, kTab = 8 };
    static_assert(kTab <= kPlaneTab, "per-plane table slots");

    struct Thread {
        int lane, wv, tile, nbt;  // nbt: the neighbour tile lane 0..3 polls (-1: none)
        uint32_t bo[PY];          // byte offset of each owned point in a plane (kOutside if outside)
        bool din[PY];
        float pyz[PY];
        uint32_t hb[HS];          // byte offsets of this thread's ring slots
        bool gaveup;              // a wait of this wave ran out (the pass has failed)
    };

    // Position (row, col) in an LDS plane of ring slot h; false if unused.
    __device__ static __forceinline__ bool halo_pos(int h, int &row, int &col)
    {
        if (h < 2 * M * RZ) {
            const int band = h / RZ;
            col = M + (h - band * RZ);
            row = band < M ? band : band + RY;
        } else {
            const int h2 = h - 2 * M * RZ;
            row = M + h2 / (2 * M);
            const int cj = h2 % (2 * M);
            col = cj < M ? cj : cj + RZ;
        }
        return h < NHALO;
    }

    // Scalar k of the per-plane table of level t (1, 2) from the lanes of v.
    template <int t, int k>
    __device__ static __forceinline__ int tab(int v)
    {
        return __builtin_amdgcn_readlane(v, (t - 1) * kTab + k);
    }

    __device__ static void run(const SweepArgs &a, Smem &sm)
    {
        Thread th;
        const int ntiles = a.ntz * a.nty;
        const int b = blockIdx.x;
        // workgroup b runs on XCD b % 8: each XCD takes a contiguous block of
        // tiles (whole rows of z-tiles), so z neighbours share its L2
        th.tile = (a.remap && (ntiles & 7) == 0) ? (b & 7) * (ntiles >> 3) + (b >> 3) : b;
        const int bz = th.tile % a.ntz, by = th.tile / a.ntz;
        const int z0 = bz * RZ, y0 = by * RY;
        th.lane = threadIdx.x & 63;
        th.wv = threadIdx.x >> 6;
        th.gaveup = false;
        {
            const int l = th.lane;
            th.nbt = (l == 0 && bz > 0)             ? th.tile - 1
                     : (l == 1 && bz + 1 < a.ntz)   ? th.tile + 1
                     : (l == 2 && by > 0)           ? th.tile - a.ntz
                     : (l == 3 && by + 1 < a.nty)   ? th.tile + a.ntz
                                                    : -1;
        }
        const int z = z0 + th.lane;
        const bool zin = (unsigned)z < (unsigned)a.nz;
        const float pzv = zin ? a.pz[z] : 0.0f;
#pragma unroll
        for (int r = 0; r < PY; ++r) {
            const int y = y0 + th.wv * PY + r;
            th.din[r] = zin && (unsigned)y < (unsigned)a.ny;
            th.bo[r] = th.din[r] ? (uint32_t)(y * a.nzp + z) * 4u : kOutside;
            th.pyz[r] = th.din[r] ? (a.py[y] + pzv) : 0.0f;
        }
#pragma unroll
        for (int s = 0; s < HS; ++s) {
            int row, col;
            const bool used = halo_pos(threadIdx.x + s * NT, row, col);
            const int gy = y0 - M + row, gz = z0 - M + col;
            const bool in = used && (unsigned)gy < (unsigned)a.ny && (unsigned)gz < (unsigned)a.nz;
            th.hb[s] = in ? (uint32_t)(gy * a.nzp + gz) * 4u : kOutside;
        }
        // a pass that follows one whose wait ran out does not wait at all
        if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) th.gaveup = true;

        // queues along x, entry 0 the oldest: u^n (qa) and level 1 (qb)
        float qa[PY][QX], qb[PY][QX], qq[PY][QQX];
#pragma unroll
        for (int r = 0; r < PY; ++r) {
#pragma unroll
            for (int j = 0; j < QX; ++j) qa[r][j] = qb[r][j] = 0.0f;
#pragma unroll
            for (int j = 0; j < QQX; ++j) qq[r][j] = 0.0f;
        }
        // planes 0 .. M-1 of u^n enter before the first iteration (i = M, level
        // 1 at plane 0); the queue then holds planes M - Q + j in entries j
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const uint32_t sxy4 = (uint32_t)a.sxy * 4u;
            const auto rh = wplane(a.u0, (uint32_t)j * sxy4, j < a.nx, sxy4);
#pragma unroll
            for (int r = 0; r < PY; ++r) qa[r][Q - M + j] = bload(rh, th.bo[r]);
        }
        const int ibeg = M, iend = a.nx + 2 * M + E;  // level 2's last plane nx - 1 at iend - 1
        uint64_t flag = poll(a, th);
        Pre pf[U];
#pragma unroll
        for (int d = 0; d < D; ++d) load(a, th, pf[d], ibeg + d);
        for (int i = ibeg; i < iend; i += U) {
            if (!body<0>(a, sm, th, qa, qb, qq, flag, pf, i, iend)) break;
#pragma unroll
            for (int r = 0; r < PY; ++r) {
#pragma unroll
                for (int j = 0; j < Q; ++j) {
                    qa[r][j] = qa[r][j + U];
                    qb[r][j] = qb[r][j + U];
                }
#pragma unroll
                for (int j = 0; j < QQ; ++j) qq[r][j] = qq[r][j + U];
            }
        }
    }

    // Phases PH .. U - 1 of the unrolled body (iterations i0 + PH ...);
    // false once the stream has ended.
    template <int PH>
    __device__ static __forceinline__ bool body(const SweepArgs &a, Smem &sm, Thread &th,
                                                float (&qa)[PY][QX], float (&qb)[PY][QX], float (&qq)[PY][QQX],
                                                uint64_t &flag, Pre (&pf)[U], int i0, int iend)
    {
        if constexpr (PH < U) {
            if (i0 + PH >= iend) return false;
            iteration<PH>(a, sm, th, qa, qb, qq, flag, pf[(PH + D) % U], pf[PH], i0 + PH);
            return body<PH + 1>(a, sm, th, qa, qb, qq, flag, pf, i0, iend);
        }
        return true;
    }

    // Iteration i: the ring loads of iteration i + D read level 1 from the
    // neighbours, so first wait until they have stored it, poll again if
    // needed, issue iteration i + D's loads into `next` (the slot the
    // previous iteration consumed), then compute from `cur`.
    template <int PH>
    __device__ static __forceinline__ void iteration(const SweepArgs &a, Smem &sm, Thread &th,
                                                     float (&qa)[PY][QX], float (&qb)[PY][QX], float (&qq)[PY][QQX],
                                                     uint64_t &flag, Pre &next, const Pre &cur, int i)
    {
        wait_for(a, th, flag, i + D);
        // poll again only if the counters last seen would not admit the next
        // iteration's ring loads (in step with the neighbours, every few
        // iterations): a poll is a device-coherent round trip, and the
        // loads issued after it complete only after it
        if (!__all(flag >= want_of(a, i + D + 1))) flag = poll(a, th);
        load(a, th, next, i + D);
        step<PH>(a, sm, th, qa, qb, qq, cur, i);
        // keep this iteration's stores ahead of the next iteration's loads in
        // issue order (the counter protocol relies on it)
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }

    // Device-coherent load of the neighbour counter lane 0..3 watches.
    __device__ static __forceinline__ uint64_t poll(const SweepArgs &a, const Thread &th)
    {
        uint64_t f = ~(uint64_t)0;
        if (th.nbt >= 0) f = __hip_atomic_load(a.prog + (int64_t)kWaveProgStride * th.nbt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return f;
    }

    // Counter value every neighbour must show before the ring loads of
    // iteration i1: level 1 at level 2's plane c2 = i1 - 2M - E was computed
    // in iteration c2 + M, and the counter k means iterations below k are
    // complete (none needed outside the grid).
    __device__ static __forceinline__ uint64_t want_of(const SweepArgs &a, int i1)
    {
        const int c2 = i1 - 2 * M - E;
        if (c2 < 0 || c2 >= a.nx) return 0;
        return ((uint64_t)a.epoch << 32) | (uint32_t)(c2 + M + 1);
    }

    // Wait until every neighbour has completed the iteration that computed
    // level 1 at level 2's plane of iteration i1 (bounded; see the header);
    // `flag` keeps the counters last seen.
    __device__ static __forceinline__ void wait_for(const SweepArgs &a, Thread &th, uint64_t &flag, int i1)
    {
        const uint64_t want = want_of(a, i1);
        if (want == 0 || th.gaveup) return;
        if (__all(flag >= want)) {
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            return;
        }
        for (int n = 0; n < kWaveSpin; ++n) {
            __builtin_amdgcn_s_sleep(2);
            flag = poll(a, th);
            if (__all(flag >= want)) {
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                return;
            }
            if ((n & 255) == 255 &&
                __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
                break;
        }
        if (th.lane == 0) __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        th.gaveup = true;
    }

    // Buffer resource over the plane at byte offset `off` of a field (an
    // empty range if !valid).  The host admits a wave pass only for fields
    // below 2 GiB, so plane offsets are 32-bit (one scalar multiply per plane
    // instead of a 64-bit one per resource).
    __device__ static __forceinline__ __amdgpu_buffer_rsrc_t wplane(const float *field, uint32_t off,
                                                                    bool valid, uint32_t sxy4)
    {
        const char *base = (const char *)field + (valid ? off : 0u);
        return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, valid ? (int)sxy4 : 0, 0x00020000);
    }

    // Issue the loads of iteration i: head plane i of u^n; level 1's plane
    // c1 = i - M (ring of u^n, u^{n-1}, q); level 2's plane c2 = i - 2M - E
    // (the level-1 ring from the neighbours).
    __device__ static __forceinline__ void load(const SweepArgs &a, const Thread &th, Pre &P, int i)
    {
        const int c1 = i - M, c2 = i - 2 * M - E;
        const bool v0 = i < a.nx, v1 = (unsigned)c1 < (unsigned)a.nx, v2 = (unsigned)c2 < (unsigned)a.nx;
        const uint32_t sxy4 = (uint32_t)a.sxy * 4u;
        const uint32_t o0 = (uint32_t)i * sxy4, o1 = (uint32_t)c1 * sxy4, o2 = (uint32_t)c2 * sxy4;
        const auto rh = wplane(a.u0, o0, v0, sxy4);
#pragma unroll
        for (int r = 0; r < PY; ++r) P.head[r] = bload(rh, th.bo[r]);
        const auto rc = wplane(a.u0, o1, v1, sxy4);
#pragma unroll
        for (int s = 0; s < HS; ++s) P.h0[s] = bload(rc, th.hb[s]);
        const auto rm = wplane(a.um, o1, v1, sxy4);
        const auto rq1 = wplane(a.q, o1, v1, sxy4);
#pragma unroll
        for (int r = 0; r < PY; ++r) {
            P.um[r] = bload<kStream>(rm, th.bo[r]);
            P.q1[r] = bload<kStream>(rq1, th.bo[r]);
        }
        const auto r1 = wplane(a.o2, o2, v2, sxy4);
#pragma unroll
        for (int s = 0; s < HS; ++s) P.h1[s] = bload<kCoherent>(r1, th.hb[s]);
        {
            // lane k < 2 kTab: slot k % kTab of plane c1 (k < kTab) or c2;
            // other lanes and planes outside the grid read 0
            const int l = th.lane, k = l < kTab ? l : l - kTab;
            const int c = l < kTab ? c1 : c2;
            const bool v = l < 2 * kTab && (unsigned)c < (unsigned)a.nx;
            const auto rt = span_rsrc(a.ptab, (int64_t)a.nx * kPlaneTab * 4, true);
            P.tab = (int)__builtin_amdgcn_raw_buffer_load_b32(
                rt, v ? (uint32_t)(c * kPlaneTab + k) * 4u : kOutside, 0, 0);
        }
    }

    // One level's update at plane c: the untiled kernel's operation order.
    // q[r][CJ +- k] are the x neighbours, S the LDS plane (own rows from the
    // queue centre), up the level two below, then the point entries.
    template <int CJ>
    __device__ static __forceinline__ void update(const SweepArgs &a, const Thread &th,
                                                  const float (&qq)[PY][QX], const float *S,
                                                  const float (&up)[PY], const float (&qv)[PY], float pxv,
                                                  bool need, int step, int ib, int ie, float (&out)[PY])
    {
        const int lane = th.lane, wv = th.wv;
        float colv[PY + 2 * M];
#pragma unroll
        for (int j = 0; j < M; ++j) {
            colv[j] = S[(wv * PY - M + j + M) * LW + lane + M];
            colv[M + PY + j] = S[(wv * PY + PY + j + M) * LW + lane + M];
        }
#pragma unroll
        for (int r = 0; r < PY; ++r) colv[M + r] = qq[r][CJ];
#pragma unroll
        for (int r = 0; r < PY; ++r) {
            const float uc = qq[r][CJ];
            const float *row = S + (wv * PY + r + M) * LW + lane + M;
            float lap = 0.0f;
#pragma unroll
            for (int k = 1; k <= M; ++k) {
                const float xs = qq[r][CJ - k] + qq[r][CJ + k];
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
            const float eta = qv[r] * (pxv + th.pyz[r]);
            const float num = fmaf(qv[r], lap, fmaf(eta - 1.0f, up[r], 2.0f * uc));
            out[r] = (need && th.din[r]) ? damped(num, eta) : 0.0f;
        }
        // point entries of the plane, in table order (entries at one node are
        // applied in that order)
        if (need && ib < ie) {
            const float *arow = a.amp + (a.abase + (int64_t)a.adir * step) * a.inj.stride;
            for (int j = ib; j < ie; ++j) {
                const uint32_t p = (uint32_t)a.inj.yz[j] * 4u;
                const float sc = a.inj.scale[j];
                const float w = arow[a.inj.id[j]];
#pragma unroll
                for (int r = 0; r < PY; ++r)
                    if (th.din[r] && th.bo[r] == p) out[r] = fmaf(sc, w, out[r]);
            }
        }
    }

    // Receivers on plane c of the level producing step `step`.  The first
    // entry's node y0 and output slot d0 come with the per-plane table: a load
    // here would wait for every prefetch issued before it, so a plane with a
    // single entry is recorded without one.
    __device__ static __forceinline__ void record(const SweepArgs &a, const Thread &th, int step, int rb,
                                                  int re, int y0, int d0, const float (&val)[PY])
    {
        if (rb >= re) return;
        const int64_t row = a.rbase + (int64_t)a.rdir * step;
        const bool ent = a.rec.etr != nullptr;
        float *orow = ent ? a.rec.etr + row * a.rec.cnt : a.rec_out + row * a.rec.stride;
        const float rs = ent ? 1.0f : a.rscale;
        {
            const uint32_t p = (uint32_t)y0 * 4u;
#pragma unroll
            for (int r = 0; r < PY; ++r)
                if (th.din[r] && th.bo[r] == p) orow[d0] = val[r] * rs;
        }
        for (int j = rb + 1; j < re; ++j) {
            const uint32_t p = (uint32_t)a.rec.yz[j] * 4u;
            const int dst = ent ? j : a.rec.id[j];
#pragma unroll
            for (int r = 0; r < PY; ++r)
                if (th.din[r] && th.bo[r] == p) orow[dst] = val[r] * rs;
        }
    }

    // One iteration: publish both LDS planes, barrier, progress counter,
    // level 1 at c1 = i - M, level 2 at c2 = i - 2M - E.
    template <int PH>
    __device__ static __forceinline__ void step(const SweepArgs &a, Smem &sm, const Thread &th,
                                                float (&qa)[PY][QX], float (&qb)[PY][QX], float (&qq)[PY][QQX],
                                                const Pre &P, int i)
    {
        static_assert(PH + Q < QX && PH + QQ < QQX, "a phase's push lands beyond the queue slots");
        static_assert(PH + 1 + 2 * M < QX, "level 2's window beyond the queue slots");
        const int par = i & 1;
        const int c1 = i - M, c2 = i - 2 * M - E;
        float *S0 = sm.s0[par], *S1 = sm.s1[par];
#pragma unroll
        for (int s = 0; s < HS; ++s) {
            int row, col;
            if (halo_pos(threadIdx.x + s * NT, row, col)) {
                S0[row * LW + col] = P.h0[s];
                S1[row * LW + col] = P.h1[s];
            }
        }
        // own rows: u^n at c1 (window entry Q - M before this iteration's
        // push) and level 1 at c2 (entry M + 1 of its window before the push)
#pragma unroll
        for (int r = 0; r < PY; ++r) {
            S0[(th.wv * PY + r + M) * LW + th.lane + M] = qa[r][PH + Q - M];
            S1[(th.wv * PY + r + M) * LW + th.lane + M] = qb[r][PH + M + 1];
        }
        __syncthreads();
        // every wave has waited for this iteration's loads, issued D
        // iterations ago, after its stores of iteration i - D - 1: those
        // stores, and all before them, are complete (stored every P-th
        // iteration; the readers' slack covers the rest).  Nothing is
        // stored while i - D < 1: a negative count would read as a huge one
        // in the counter's low word, i.e. as every plane of the pass stored
        // (the first iteration is i = M, below D for M < D).
        if (threadIdx.x == 0 && (i & (PUB - 1)) == 0 && i > D)
            __hip_atomic_store(a.prog + (int64_t)kWaveProgStride * th.tile,
                               ((uint64_t)a.epoch << 32) | (uint32_t)(i - D), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);

        // level 1 at c1: push the head plane and q at c1, update from the
        // u^n queue
#pragma unroll
        for (int r = 0; r < PY; ++r) {
            qa[r][PH + Q] = P.head[r];
            qq[r][PH + QQ] = P.q1[r];
        }
        const bool n1 = (unsigned)c1 < (unsigned)a.nx, n2 = (unsigned)c2 < (unsigned)a.nx;
        float o1v[PY];
        // the entry ranges are read back only for planes that hold points
        const int f1 = tab<1, kFl>(P.tab), f2 = tab<2, kFl>(P.tab);
        int ib = 0, ie = 0;
        if (f1 & 1) {
            ib = tab<1, kIb>(P.tab);
            ie = tab<1, kIe>(P.tab);
        }
        update<PH + Q - M>(a, th, qa, S0, P.um, P.q1, __int_as_float(tab<1, kPx>(P.tab)), n1, a.step0, ib,
                          ie, o1v);
        if (n1 && (f1 & 2))
            record(a, th, a.step0, tab<1, kRb>(P.tab), tab<1, kRe>(P.tab), tab<1, kRy>(P.tab), tab<1, kRd>(P.tab),
                   o1v);
        const uint32_t sxy4 = (uint32_t)a.sxy * 4u;
        {
            const auto rw = wplane(a.o2, (uint32_t)c1 * sxy4, n1, sxy4);
#pragma unroll
            for (int r = 0; r < PY; ++r) bstore<kCoherent>(rw, th.bo[r], o1v[r]);
        }
#pragma unroll
        for (int r = 0; r < PY; ++r) qb[r][PH + Q] = o1v[r];

        // level 2 at c2: update from the level-1 window (centre entry M); the
        // level below it is u^n at c2, entry 0 of the u^n window, and q at c2
        // entry 0 of the q window
        float up[PY], q2[PY], o2v[PY];
#pragma unroll
        for (int r = 0; r < PY; ++r) {
            up[r] = qa[r][PH + 1];
            q2[r] = qq[r][PH + 1];
        }
        ib = ie = 0;
        if (f2 & 1) {
            ib = tab<2, kIb>(P.tab);
            ie = tab<2, kIe>(P.tab);
        }
        update<PH + 1 + M>(a, th, qb, S1, up, q2, __int_as_float(tab<2, kPx>(P.tab)), n2, a.step0 + 1, ib, ie,
                           o2v);
        if (n2 && (f2 & 2))
            record(a, th, a.step0 + 1, tab<2, kRb>(P.tab), tab<2, kRe>(P.tab), tab<2, kRy>(P.tab),
                   tab<2, kRd>(P.tab), o2v);
        const auto ro = wplane(a.o1, (uint32_t)c2 * sxy4, n2, sxy4);
#pragma unroll
        for (int r = 0; r < PY; ++r) bstore<kStream>(ro, th.bo[r], o2v[r]);
    }
};

template <int M, int PY, int NW, bool ISO>
__global__ __launch_bounds__(64 * NW) void k_wave(SweepArgs a)
{
    using K = WaveKernel<M, PY, NW, ISO>;
    __shared__ typename K::Smem sm;
    K::run(a, sm);
}

template <int M, int PY, int NW>
bool wave_launch(const SweepArgs &a, hipStream_t s)
{
    const dim3 grid(a.ntz * a.nty), block(64 * NW);
    if (a.w.iso) hipLaunchKernelGGL((k_wave<M, PY, NW, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_wave<M, PY, NW, false>), grid, block, 0, s, a);
    return true;
}

template <int M, int PY, int NW>
int wave_occupancy(bool iso)
{
    int n = 0;
    const void *fn = iso ? reinterpret_cast<const void *>(&k_wave<M, PY, NW, true>)
                         : reinterpret_cast<const void *>(&k_wave<M, PY, NW, false>);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, 64 * NW, 0) == hipSuccess ? n : 0;
}

}  // namespace fdw
