// fd_internal.h -- structures shared by the HIP kernels and the host planner of
// libfdwave.so.  Not part of the public ABI (include/fdwave.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdw {

constexpr int kMaxM = 8;     // space order up to 16
constexpr int kMaxLx = 512;  // planes per workgroup chunk (per-plane tables live in LDS)

// FP32 stencil weights w{x,y,z}[k-1] = c_k / h_a^2 for k = 1..M (zero for an
// absent axis), computed once on the host in FP64 and rounded to FP32.  The
// centre weight c_0 = -2 sum_k c_k is not stored: every kernel evaluates
// sum_k w_k (u(-k) + u(+k) - 2 u_c).
// When every present axis has the same weights ("isotropic"), kernels use the
// cheaper, equally cancellation-free form
//   lap = sum_k w_k ((sx + sy) + sz - 2 d u_c)      (cc = -2 d, d present axes)
// with s_a = u(-k e_a) + u(+k e_a); otherwise sum_k sum_a w_{a,k} (s_a - 2 u_c).
struct Weights {
    float wx[kMaxM];
    float wy[kMaxM];
    float wz[kMaxM];
    float cc;
    int iso;
};

// Grid nodes of a point set, bucketed by x (CSR): entries of plane x are
// [xptr[x], xptr[x+1]), ordered by (y, z, original index).
struct PointTable {
    const int32_t *xptr;  // [nx + 1]
    const int32_t *xe;    // [cnt] x of each entry
    const int32_t *yz;    // [cnt] y * nz + z
    const int32_t *id;    // [cnt] original point index (column of amp / record arrays)
    const float *scale;   // [cnt] injection scale (sources only), else nullptr
    const float *wt;      // [cnt] interpolation weight of each entry (1 on grid nodes)
    float *etr;           // recording of points between nodes: [rows][cnt], the value
                          // at every entry, summed per point after the sweep; nullptr:
                          // one entry per point, written straight to the trace
    const int32_t *box;   // [nx][4] bounding box of each plane's entries: min y, max y,
                          // min z, max z (empty plane: min > max)
    int32_t stride;       // number of original points (row length of amp / record)
    int32_t cnt;          // number of entries
};

// Arguments of one pass of T levels (T = 1 for a plain step).
struct SweepArgs {
    int nx, ny, nz;
    int nzp;          // row pitch of every internal field: nz rounded up to 32 floats
    int64_t sxy;      // ny * nzp (one x-plane)
    Weights w;
    const float *q;   // v^2 dt^2
    const float *px;  // sponge profile / (2 dt) along x, y, z  (damp * v^2 dt / 2 = q * (px + (py + pz)))
    const float *py;
    const float *pz;
    const float *u0;  // u^n
    const float *um;  // u^{n-1}
    float *o1;        // receives u^{n+T}   (T = 1: may alias um)
    float *o2;        // receives u^{n+T-1} (T >= 2)
    // injection: level t (1..T) produces step s = step0 + t - 1; amplitude row
    // abase + adir * s.
    PointTable inj;
    const float *amp;
    int64_t abase;
    int adir;
    int step0;
    // recording: row rbase + rdir * s, value scaled by rscale.
    PointTable rec;
    float *rec_out;
    int64_t rbase;
    int rdir;
    float rscale;
    // gradient support: field slot dslot0 + ddir * (t - 1) of d2 (N floats each).
    float *d2;
    int64_t dslot0;
    int ddir;
    float *g;         // the image's partial sums (FP32, N) over at most kImageFlush
                      // steps, then added into the FP64 image
    const float *bs;  // Born: scattering coefficient 2 dv / v (N); d2 slot dslot0 holds
                      // the background's second difference
    const float *u0b; // fused Born: the perturbation's u^n and u^{n-1} (o2 receives
    const float *umb; // its u^{n+1}, and may alias umb)
    // tiling of the launch
    int lx;           // planes per workgroup along x
    int ntz, nty, ntx;
    // XCD-aware tile order: workgroup b runs on XCD b % 8; with remap != 0 the
    // tiles are cut into super-tiles of all ntz x gy x gx tiles, dealt to the
    // XCDs round-robin, so that neighbouring tiles share one XCD's L2.
    int remap;
    int gx, gy;
    // alt != 0: workgroups of odd x-chunks stream x downward, so the planes two
    // neighbouring chunks both read are read at the same time (both at the
    // chunks' ends or both at their starts).
    int alt;
    // ntl != 0: u^{n-1}, q and the gradient fields are loaded non-temporally
    // (single-pass launches; a grouped launch takes the policy as an argument).
    int ntl;
    // ps != 0: the point entries of every chunk fit in LDS and are staged there
    // (single-pass launches; a grouped launch takes the choice as an argument).
    int ps;
    // Chunk placement along x: chunk bx starts at plane xoff + bx * xstride
    // (xstride 0: lx) and spans lx planes.
    int xoff, xstride;
    // split != 0 (two-level plain passes): the first phase of a pass split into
    // upright and inverted trapezoids along x.  Chunks tile x without overlap:
    // level 1 is computed on the chunk's own planes and stored there in full,
    // level 2 on them less M planes at each end another chunk shares; the
    // second phase, a single-level pass over the 2M planes around each shared
    // end, fills level 2 in those gaps.
    int split;
    // Passes without redundant halos (fd_wave.h): per-tile progress counters
    // ((epoch << 32) | iterations completed), the pass's epoch (distinct for
    // every pass of a sweep; the counters start at 0), and the error word a
    // wait that runs out sets.
    uint64_t *prog;
    int *err;
    uint32_t epoch;
    // Per-plane scalars of those passes, [nx][8]: the sponge profile px (as
    // bits), the plane's source entry range [ib, ie), its receiver entry range
    // [rb, re), flags (bit 0: sources, bit 1: receivers on the plane), and the
    // first receiver entry's node (rec.yz[rb]) and output slot (rb when the
    // receivers interpolate, else rec.id[rb]).
    const int32_t *ptab;
};
constexpr int kPlaneTab = 8;  // int32 slots per plane of SweepArgs::ptab

// The imaging condition's sum over time steps is carried in FP32 over at most
// this many consecutive adjoint steps and then added into the FP64 image: the
// FP32 partial sum costs at most this many roundings of its own magnitude
// (about 4e-6 relative, against the ~1e-7 of the FP32 wavefields' terms
// themselves), and reading and writing 4 instead of 8 bytes per point and step
// takes 8 of the imaging pass's 36 bytes per point-step (the flush costs 24
// bytes per point once per block).
constexpr int kImageFlush = 64;

// Point entries x time levels a workgroup can stage in LDS, the configurations
// that can (the others would spill registers), and the table size below which
// the walk in memory is kept (a lone source costs it nothing).
constexpr int kPtsCap = 512;
constexpr int kStageMin = 32;
constexpr bool points_stageable(int M, int T, int PY, int NW) { return NW < 16 && PY <= 4 && M * T < 16; }

// kBorn: the perturbation wavefield of Born modelling, whose update carries
// the volume source s * d2 inside the division: (num + s d2) / (1 + eta), with
// s = 2 dv / v and d2 the background's second difference at the same step
// (single-step passes only).
// kBornFused: background (u0/um -> o1, sources injected) and perturbation
// (u0b/umb -> o2, receivers recorded) of Born modelling in one pass, the
// perturbation's source formed from the background's new level in registers.
enum Mode { kPlain = 0, kSaveD2 = 1, kImaging = 2, kBorn = 3, kBornFused = 4 };

// The damped update's division u = num / (1 + eta), taken only where eta != 0
// (the sponge), as num times the hardware reciprocal of 1 + eta (v_rcp_f32,
// within 1 ulp; 1 + eta >= 1, so no denormal can occur).  Every kernel calls
// this one helper, so all variants round identically; it replaces the
// ten-instruction IEEE division sequence.
__device__ __forceinline__ float damped(float num, float eta)
{
    return (eta != 0.0f) ? num * __builtin_amdgcn_rcpf(1.0f + eta) : num;
}

// One shot's pass in a grouped launch: its arguments and the index of its
// first tile in the launch's flat tile range (entries sorted by tile0).
struct GroupEntry {
    SweepArgs a;
    int32_t tile0;
    int32_t pad[3];
};

// Stream/time-block kernel configuration (compile-time template parameters).
struct KernelKey {
    int M, T, PY, NW, mode;
};

// Launcher for the templated streaming kernel; returns false when no
// instantiation matches the key.  With list == nullptr the kernel runs the
// tiles of `a`; otherwise it walks the `total` tiles of the nlist entries
// with `grid` workgroups, persistently if grid < total (iso selects the Laplacian form).
bool launch_stream(const KernelKey &key, const SweepArgs &a, hipStream_t s);
// Traces of points between nodes from their recorded entry values:
// out[row][p] = rscale * sum over the entries k of point p (pptr/pent, corner
// order) of wt[k] * etr[row][k].
hipError_t launch_gather(const float *etr, int64_t rows, int cnt, const int32_t *pptr,
                         const int32_t *pent, const float *wt, int npts, float *out, float rscale,
                         hipStream_t s);
bool launch_stream_grouped(const KernelKey &key, bool iso, bool ntl, bool ps,
                           const GroupEntry *list, int nlist, int total, int grid, hipStream_t s);
// Resident workgroups per CU of a configuration's single-pass or grouped kernel
// (0 if not compiled).
int stream_occupancy(const KernelKey &key, bool iso, bool grouped);
// Tile sizes (core rows / columns) for a key.
int stream_core_rows(const KernelKey &key);
int stream_core_cols(const KernelKey &key);
// Whether a configuration is compiled for the isotropic / anisotropic form, and
// whether its grouped batch kernel is.
bool stream_has(const KernelKey &key, bool iso);
bool stream_has_group(const KernelKey &key, bool iso);

// Two-level passes without redundant halos (fd_wave.h): whether a tile shape
// (PY rows per thread, NW waves) is compiled for radius M, its launcher (one
// workgroup per (y, z) tile of a.ntz x a.nty) and its resident workgroups per
// CU (0 if not compiled).
bool wave_has(int M, int PY, int NW);
// Spacing of the progress counters in uint64 elements: one counter per 256
// bytes, so no two workgroups' counters share a cache line (counters packed
// into a few lines, stored and polled by every workgroup each iteration,
// serialised those accesses and cut the 512^3 so-8 rate from 260 to 81 GPts/s).
constexpr int kWaveProgStride = 32;
bool launch_wave(int M, int PY, int NW, const SweepArgs &a, hipStream_t s);
int wave_occupancy(int M, int PY, int NW, bool iso);

// Naive (untiled) kernels.
hipError_t launch_naive_step(int M, const SweepArgs &a, hipStream_t s);  // form from a.w.iso
hipError_t launch_inject(const SweepArgs &a, float *field, int step, hipStream_t s);
hipError_t launch_record(const SweepArgs &a, const float *field, int step, hipStream_t s);
hipError_t launch_entry_x(const PointTable &t, int nx, int32_t *xe, hipStream_t s);
hipError_t launch_save_d2(const SweepArgs &a, const float *unew, const float *ucur,
                          const float *uprev, float *d2, hipStream_t s);
hipError_t launch_imaging(const SweepArgs &a, const float *lam, const float *d2, float *g,
                          hipStream_t s);
// The FP64 image g += the partial sums part, which are then cleared.
hipError_t launch_flush_image(float *part, double *g, int64_t n, hipStream_t s);

// Preparation / reduction kernels.
// q = v^2 dt^2 from the dense caller layout (rows of nz) into the padded
// internal layout (rows of nzp, padding zero).
hipError_t launch_born_coef(const float *v, const float *dv, float *s, int64_t rows, int nz, int nzp,
                            hipStream_t st);
hipError_t launch_make_q(const float *v, float *q, int64_t rows, int nz, int nzp, double dt2,
                         hipStream_t s);
// Copy rows of nz floats between layouts of row pitch spitch and dpitch (the
// destination's padding, if any, is zeroed).
hipError_t launch_repitch(float *dst, int dpitch, const float *src, int spitch, int64_t rows,
                          int nz, hipStream_t s);
hipError_t launch_vstats(const float *v, int64_t n, float *partial /*[3*nb]*/, int nb,
                         hipStream_t s);
hipError_t launch_scales(const SweepArgs &a, const PointTable &t, float *scale, float alpha,
                         hipStream_t s);
hipError_t launch_residual(const float *d, const float *dobs, float *res, int64_t n,
                           double *partial, int nb, hipStream_t s);
hipError_t launch_grad_v(const double *g, const float *v, float *grad_v, int64_t rows, int nz,
                         int nzp, hipStream_t s);
hipError_t launch_zero(void *p, int64_t bytes, hipStream_t s);
hipError_t launch_copy(float *dst, const float *src, int64_t n, hipStream_t s);

}  // namespace fdw
