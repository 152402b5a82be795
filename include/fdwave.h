/*
 * fdwave.h -- C ABI of the MI355X (gfx950) acoustic finite-difference sweep
 * library, libfdwave.so.
 *
 * The library advances the damped, second-order-in-time acoustic wave equation
 *     m u_tt + damp u_t - Lap(u) = source,    m = 1 / v^2,
 * with the leapfrog update of the paper's Devito-generated stencil (Sec. 6.3.1,
 * Fig. "acoustic_devito"; the same update is the body of the time-tiled loop of
 * Sec. 5.5, Fig. "tiled_256"):
 *     u^{n+1} = ((dt damp - 2m) u^{n-1} + 4m u^n + 2 dt^2 L_h u^n) / (dt damp + 2m)
 * where L_h is the star Laplacian of space order so (2, 4, ..., 16), whose
 * weights are the closed-form central second-difference coefficients.  Points
 * outside the grid are zero (the paper's never-written ghost cells).  The GPU
 * evaluates the same update in the algebraically equal form
 *     u^{n+1} = (2 u^n + (eta - 1) u^{n-1} + q L_h u^n) / (1 + eta),
 *     q = v^2 dt^2,  eta = dt damp v^2 / 2,
 * in FP32 with one fixed per-point operation order shared by every kernel
 * variant, so that the untiled, space-tiled and time-blocked kernels return
 * bit-identical fields.
 *
 * Time blocking (the paper's contribution, Secs. 5.2-5.4 and 7.1): a kernel may
 * advance T >= 2 time levels per pass over HBM.  Legality comes from skewing
 * each level by the stencil radius M = so/2 (Sec. 5.2: skew by the largest
 * negative dependence distance), which the streaming kernels realise as a lag
 * of M planes per level along the streamed axis plus an overlapped halo of
 * M (T - 1) cells in the two tiled axes.
 *
 * Readings the paper leaves open (it only names source and receiver loops and
 * a damp array, Sec. 6.2 shell log and Sec. 6.3.1):
 *   * sources are injected in the step producing u^{n+1}:
 *       u^{n+1}(s) += 2 dt^2 w[n][s] / (dt damp(s) + 2 m(s));
 *   * receivers record the new level on grid nodes: d[n][r] = u^{n+1}(r);
 *   * a point between grid nodes acts through multilinear interpolation over
 *     the nodes of its cell (fd_points.pos), or Kaiser-windowed sinc
 *     interpolation (Hicks 2002) over 2r nodes per axis (fd_points.interp = r):
 *     a receiver reads the weighted sum, a source adds to each node its
 *     weight's share, which keeps the two rules above as the single-node case
 *     and the adjoint an exact transpose;
 *   * sponge: damp(i) = sum_a d0_a (delta_a / L)^2 with delta_a the number of
 *     cells into the outer L-cell layer of axis a (0 in the interior and at the
 *     layer's inner edge) and d0_a = 1.5 ln(1000) / (vref L h_a)  [s/m^2];
 *   * stability: v_max^2 dt^2 S sum_a 1/h_a^2 <= 4 with S = -c_0 - 2 sum_k (-1)^k c_k,
 *     the largest eigenvalue of -h^2 L_h along one axis (the symbol at the Nyquist
 *     wavenumber); for equal spacing this is the Courant bound
 *     v_max dt / h <= 2 / sqrt(ndim S).
 *
 * Memory layout of every field: dense FP32, C order over the ndim axes, the
 * last axis contiguous (the paper's z loop is the innermost, vectorised one).
 * A 3-D grid has axes (x, y, z); 2-D grids are treated as 3-D with a unit
 * middle axis, 1-D grids as 3-D with two unit leading axes.
 *
 * Ownership: the caller owns every buffer.  Device pointers must stay valid
 * until the work enqueued on `stream` has completed.  The library never
 * allocates device memory on these paths: all scratch lives in the caller's
 * workspace (size from fd_workspace_size).  Host pointers (point indices) are
 * read during the call only.
 *
 * Streams: every call enqueues its work on `stream` (a hipStream_t; NULL is
 * the default stream) and returns without waiting, except (i) the stability
 * check, which reads back max(v) (skip it with FD_FLAG_NO_CFL_CHECK), (ii) the
 * upload of the point tables in each call's set-up, which waits for its copies
 * on `stream`, and (iii) fd_gradient when `misfit` is non-NULL, which waits for
 * the misfit.  The batched entry points fork the work of each space order onto
 * a stream of their own and join it back into `stream` before returning.
 *
 * Operations: fd_forward, fd_adjoint (its transpose), fd_gradient and fd_vjp
 * (adjoint-state derivatives with respect to v), fd_born (the linearised
 * forward map, fd_vjp's transpose), their batched forms for many shots,
 * fd_autotune (picks a kernel configuration for a grid) and fd_gradient_storage
 * (picks a gradient's checkpoint interval for a memory budget).
 *
 * Errors: every entry point returns 0 (FD_OK) or a negative FD_E* code; no
 * C++ exception crosses the ABI.  On error nothing further is enqueued, but
 * work enqueued before the failing check may still run.
 */
#ifndef FDWAVE_H
#define FDWAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
#define FD_OK 0
#define FD_EINVAL (-1)        /* bad descriptor, pointer, size or option */
#define FD_ECFL (-2)          /* dt beyond the leapfrog stability limit */
#define FD_EDOM (-3)          /* a source or receiver index outside the grid */
#define FD_EWORKSPACE (-4)    /* workspace NULL or smaller than fd_workspace_size */
#define FD_ENOMEM (-5)        /* a host-side allocation failed */
#define FD_EHIP (-6)          /* a HIP runtime call failed */
#define FD_ENONFINITE (-7)    /* v has a NaN/Inf/non-positive entry, or (with
                                 FD_FLAG_CHECK_FINITE) the traces are not finite */
#define FD_EUNSUPPORTED (-8)  /* no compiled kernel for the requested options */
#define FD_ESCRATCH (-9)      /* fd_forward_noalloc: the call needs more scratch than
                                 FD_NOALLOC_SCRATCH_BYTES */
#define FD_ESYNC (-10)        /* FD_VARIANT_WAVE: a workgroup waited too long for its
                                 neighbours (its launch did not run all workgroups at
                                 once, e.g. the device was shared); the outputs are
                                 undefined */

/* ------------------------------------------------------------------ variants */
#define FD_VARIANT_AUTO 0    /* autotuner / cached choice */
#define FD_VARIANT_NAIVE 1   /* untiled: one thread per point, neighbours from memory */
#define FD_VARIANT_STREAM 2  /* space-tiled: (y,z) tile per workgroup, x streamed
                                through a register queue, y/z neighbours via LDS */
#define FD_VARIANT_TBLOCK 3  /* time-blocked streaming: T levels per HBM pass */
#define FD_VARIANT_SPLIT 4   /* time-blocked, two levels per pass, with split tiles along
                                the streamed axis x (Pochoir-style trapezoids, paper
                                Sec. 2.5): chunks tile x without overlap, each computes
                                an upright trapezoid (level 1 on its planes, level 2 on
                                them less M at each shared end), and a second, single-
                                level phase fills the inverted trapezoids (level 2 on the
                                2M planes around each shared end); no plane of level 1 is
                                computed twice.  Passes with more than 32 receiver
                                entries use TBLOCK's overlapped chunks.  tblock must
                                be 0 or 2. */
#define FD_VARIANT_WAVE 5    /* time-blocked, two levels per pass, without redundant
                                halos (paper Secs. 5.2-5.5: each tile computes every
                                level on its own points only): a workgroup owns a
                                (y, z) tile of the whole x axis, level 2 trails level 1
                                by M + E planes, and level 2 reads level 1 on the ring
                                around its tile from the neighbouring workgroups once
                                their progress counters show it stored (device-coherent
                                exchange through the pass's u^{n+1} field).  tile[0] is
                                ignored (the whole axis), tile[1] / tile[2] choose the
                                tile's rows and rows per thread; tblock must be 0 or 2.
                                All of a pass's workgroups must fit on the device at once,
                                and each field must be below 2 GiB (FD_EUNSUPPORTED
                                otherwise; an automatic plan whose cached choice is this
                                variant falls back to the default then); the call waits for its
                                passes to finish and returns FD_ESYNC if a wait ran out.
                                Plain forward and adjoint passes only: gradient and Born
                                passes, passes whose point tables are injected or recorded
                                separately, batches and single-step tails use the other
                                variants' kernels; so do, when the plan is automatic (a
                                cached choice), passes with more than 64 injected entries
                                or more than 64 receiver entries beyond the first of each
                                x-plane (the workgroups holding them walk them through
                                memory, and their neighbours wait for them). */

/* ------------------------------------------------------------------ flags */
#define FD_FLAG_NO_CFL_CHECK 1u   /* skip the max(v) read-back and stability check */
#define FD_FLAG_CHECK_FINITE 2u   /* read back the traces and fail on NaN/Inf */
#define FD_FLAG_NO_XCD_REMAP 4u   /* keep the hardware workgroup order (for A/B timing) */
#define FD_FLAG_NO_X_ALTERNATE 8u /* stream every x-chunk upward (for A/B timing) */
/* Cache policy of the loads each point makes once per step (u^{n-1}, the
 * coefficient field q, and the gradient's fields).  By default they are
 * non-temporal in single-step passes when the fields a step re-reads (u^n,
 * u^{n-1}, q; the image's partial sums in a gradient) exceed 320 MiB, the share the
 * GPU's last-level cache keeps, and ordinary otherwise (time-blocked passes
 * share those loads between overlapping tiles); for a grouped batch launch
 * the fields of all its shots count.  The two flags force one policy (for A/B timing); setting
 * both is FD_EINVAL.  Results are identical either way. */
#define FD_FLAG_LOADS_STREAM 16u
#define FD_FLAG_LOADS_KEEP 32u

/* ------------------------------------------------------------------ ops for workspace sizing */
#define FD_OP_FORWARD 0
#define FD_OP_ADJOINT 1
#define FD_OP_GRADIENT 2
#define FD_OP_VJP 3
#define FD_OP_BORN 4

/* Grid: extents, spacing, space order and sponge. */
typedef struct fd_grid {
    int32_t ndim;         /* 1, 2 or 3 */
    int32_t space_order;  /* 2, 4, 6, ..., 16 */
    int64_t n[3];         /* points per axis (first ndim used), last axis contiguous;
                             1 <= n <= 2^20, and the product of the last two axes
                             of a 3-D grid (one plane) below 2^28 */
    double h[3];          /* spacing per axis in metres, > 0 */
    int32_t sponge;       /* sponge width L in cells, 0 = none (2 L <= n[a]) */
    int32_t reserved;     /* must be 0 */
    double sponge_vref;   /* velocity (m/s) setting the sponge strength, > 0 if sponge > 0 */
} fd_grid;

/* Time axis. */
typedef struct fd_time {
    int64_t nt;  /* number of steps, >= 0 */
    double dt;   /* step in seconds, > 0 */
} fd_time;

/* Point set (sources or receivers), on grid nodes (idx) or anywhere in the
 * grid (pos).  A point at a position acts through multilinear interpolation
 * over the 2^ndim nodes of the cell that holds it, with weights
 * w_c = prod_a (c_a ? f_a : 1 - f_a), f_a the fractional part of the position
 * (a position on the last node of an axis uses the cell below):
 *   receiver:  d[n] = sum_c w_c u^{n+1}(c)
 *   source:    u^{n+1}(c) += w_c 2 dt^2 w(n dt) / (2 m(c) + dt damp(c))
 * (the operator P and its transpose, so the adjoint and the gradient stay
 * exact transposes; an integer position is the same as the grid index, bit
 * for bit).  Exactly one of idx and pos is non-NULL when n > 0. */
typedef struct fd_points {
    int32_t n;           /* number of points, >= 0 */
    int32_t interp;      /* with pos: 0 multilinear over the cell (2^ndim nodes);
                            r in 1..8 Kaiser-windowed sinc of half-width r ((2r)^ndim
                            nodes, those outside the grid left out; the window shape
                            b(r) minimises the largest error of interpolating waves
                            of up to four points per wavelength).  0 with idx.
                            At most 2^27 nodes per point set (FD_EINVAL). */
    const int32_t *idx;  /* HOST, [n][ndim] grid indices, or NULL */
    const float *amp;    /* DEVICE, [nt][n] time samples: source wavelet (forward),
                            injected residual (adjoint), observed data or trace
                            cotangent (gradient / vjp); unused where not listed */
    const double *pos;   /* HOST, [n][ndim] positions in grid-index units
                            (0 <= pos_a <= n_a - 1, finite; FD_EDOM otherwise), or NULL */
} fd_points;

/* Execution options; zero-initialised options mean "automatic". */
typedef struct fd_options {
    int32_t variant;     /* FD_VARIANT_*; 0 = automatic */
    int32_t tile[3];     /* {planes per workgroup along x, tile rows along y,
                            rows per thread}; 0 = automatic */
    int32_t tblock;      /* time levels per pass for FD_VARIANT_TBLOCK (2..4); 0 = auto */
    int32_t ckpt_every;  /* gradient checkpoint interval k in steps; 0 = auto (50) */
    uint32_t flags;      /* FD_FLAG_* */
    int32_t reserved;    /* must be 0 */
} fd_options;

/*
 * Bytes of device workspace an operation needs (FD_OP_*).  src/rec give the
 * point counts (amp is not read); opts may be NULL.  Returns 0 on invalid input.
 */
size_t fd_workspace_size(const fd_grid *grid, const fd_time *time, const fd_points *src,
                         const fd_points *rec, const fd_options *opts, int op);

/*
 * Storage scheme of a gradient (op FD_OP_GRADIENT or FD_OP_VJP) for a memory
 * budget: the paper's choice between a saved (full) and a buffered time
 * dimension (Sec. 6.3.2), here between keeping every second difference and
 * checkpointing with recomputation.  Sets inout->ckpt_every (other fields are
 * kept) to
 *   nt, the whole time axis stored (no recomputation: two sweeps per step
 *       instead of three), when fd_workspace_size for it is <= budget; else
 *   the interval with the smallest workspace (every interval below nt
 *       recomputes the same nt steps, so the smallest footprint costs no time).
 * *ws_bytes (may be NULL) receives fd_workspace_size for the chosen interval.
 * Host-only: no device call, no allocation.  src/rec as in fd_workspace_size.
 * Returns FD_OK; FD_EWORKSPACE if even the smallest workspace exceeds budget
 * (*inout and *ws_bytes are still set to it); FD_EINVAL on a bad descriptor,
 * op, nt < 1 or inout == NULL.
 */
int fd_gradient_storage(const fd_grid *grid, const fd_time *time, const fd_points *src,
                        const fd_points *rec, int op, size_t budget, fd_options *inout,
                        size_t *ws_bytes);

/*
 * Forward sweep (Sec. 6.3.1 update, nt steps).
 *   v        DEVICE [N] velocity in m/s (read only).
 *   src      point sources; src->amp DEVICE [nt][ns] raw wavelet samples w[n].
 *   rec      receivers; positions only.
 *   rec_out  DEVICE [nt][nr] receiver traces d[n][r] = u^{n+1}(r); may be NULL if nr == 0.
 *   u_state  DEVICE [2][N] or NULL.  On entry (u^0, u^{-1}); on return
 *            (u^nt, u^{nt-1}).  NULL means a zero initial state and no state out.
 *   workspace/ws_bytes  DEVICE scratch of at least fd_workspace_size(..., FD_OP_FORWARD).
 *   opts     may be NULL.   stream  hipStream_t or NULL.
 * Returns FD_OK or FD_EINVAL / FD_EDOM / FD_ECFL / FD_ENONFINITE / FD_EWORKSPACE /
 * FD_EUNSUPPORTED / FD_EHIP.
 */
int fd_forward(const fd_grid *grid, const fd_time *time, const float *v,
               const fd_points *src, const fd_points *rec, float *rec_out, float *u_state,
               void *workspace, size_t ws_bytes, const fd_options *opts, void *stream);

/*
 * Adjoint sweep: the transpose of the linear map F: w -> d that fd_forward
 * realises for a zero initial state.  With step k written as
 *   A u^k - B u^{k-1} - C u^{k-2} = 2 dt^2 P_s^T w^{k-1},
 *   A = diag(2m + dt damp), B = 4m + 2 dt^2 L_h (symmetric), C = diag(dt damp - 2m),
 * the adjoint solves lambda^k = A^{-1}(B lambda^{k+1} + C lambda^{k+2} + P_r^T y[k-1])
 * backward from lambda^{nt+1} = lambda^{nt+2} = 0, i.e. the same stencil update
 * run in reversed time, and returns (F^T y)[k-1][s] = 2 dt^2 lambda^k(s).
 *   rec->amp DEVICE [nt][nr] the traces y injected at the receivers.
 *   src_out  DEVICE [nt][ns] result at the source positions (may be NULL if ns == 0).
 *   lam_state DEVICE [2][N] or NULL: on return (lambda^1, lambda^2).
 */
int fd_adjoint(const fd_grid *grid, const fd_time *time, const float *v,
               const fd_points *src, const fd_points *rec, float *src_out, float *lam_state,
               void *workspace, size_t ws_bytes, const fd_options *opts, void *stream);

/*
 * Gradient of the least-squares misfit J = 1/2 sum_{n,r} (d[n][r] - d_obs[n][r])^2
 * with respect to v, for a zero initial state:
 *   dJ/dm(x) = -2 sum_{k=1..nt} lambda^k(x) (u^k - 2u^{k-1} + u^{k-2})(x)   (zero-lag
 *   imaging condition, lambda from fd_adjoint's recurrence driven by the residual),
 *   dJ/dv = dJ/dm * (-2 / v^3).
 * Forward wavefields are checkpointed every ckpt_every steps (u^{jk}, u^{jk-1}) and
 * recomputed segment by segment (the paper's buffered vs saved time dimension,
 * Sec. 6.3.2, traded through recomputation).  With ckpt_every >= nt the whole
 * time axis is stored instead (workspace about nt fields): the forward sweep
 * saves every second difference and no recomputation runs, two sweeps instead
 * of three; results are identical.  The imaging sum is carried in FP32 over
 * blocks of 64 consecutive time steps (the same blocks for every checkpoint
 * interval) and accumulated in FP64 across the blocks.
 *   src->amp DEVICE [nt][ns] source wavelet; rec->amp DEVICE [nt][nr] observed data.
 *   grad_v   DEVICE [N] FP32 result.
 *   misfit   HOST double or NULL (non-NULL: the call waits for it).
 *   residual DEVICE [nt][nr] or NULL: receives d - d_obs.
 */
int fd_gradient(const fd_grid *grid, const fd_time *time, const float *v,
                const fd_points *src, const fd_points *rec, float *grad_v, double *misfit,
                float *residual, void *workspace, size_t ws_bytes, const fd_options *opts,
                void *stream);

/*
 * Vector-Jacobian product of the map v -> d (receiver traces, zero initial
 * state): grad_v = (dd/dv)^T y for the trace cotangent y = rec->amp DEVICE [nt][nr].
 * Same checkpointed adjoint-state computation as fd_gradient with the residual
 * replaced by y (this is what a reverse-mode autodiff backward needs).
 */
int fd_vjp(const fd_grid *grid, const fd_time *time, const float *v, const fd_points *src,
           const fd_points *rec, float *grad_v, void *workspace, size_t ws_bytes,
           const fd_options *opts, void *stream);

/*
 * Born (linearised) modelling: the traces dd = (dd/dv) dv of the map v -> d for
 * a velocity perturbation dv, zero initial state.  Differentiating the step with
 * respect to m = 1/v^2 (paper Sec. 6.3.1 update; dm = -2 dv / v^3) gives the
 * perturbation wavefield the same recurrence driven by the volume source
 * A^{-1} (-2 dm (u^k - 2u^{k-1} + u^{k-2})), u the background wavefield; each step
 * advances the background and the perturbation, whose update folds the source
 * in as (num + s d2) / (1 + eta), s = 2 dv / v, d2 the background's new second
 * difference: in one pass over both fields for space orders up to 8 (tiled
 * variants), else in two (the first saving d2).  fd_vjp is its transpose.
 *   dv       DEVICE [N] FP32 velocity perturbation (m/s).
 *   src->amp DEVICE [nt][ns] source wavelet of the background.
 *   rec_out  DEVICE [nt][nr] perturbed traces (may be NULL if nr == 0).
 * Workspace: fd_workspace_size(..., FD_OP_BORN) (ten fields and the tables).
 * Errors as fd_forward; FD_EINVAL if dv is NULL.
 */
int fd_born(const fd_grid *grid, const fd_time *time, const float *v, const float *dv,
            const fd_points *src, const fd_points *rec, float *rec_out, void *workspace,
            size_t ws_bytes, const fd_options *opts, void *stream);

/*
 * Autotuner, the counterpart of the auto-tuned spatial blocking that the
 * paper's control runs use (Devito's block-size search, Sec. 6.6.1): times
 * candidate kernels (variant, tile, time-block depth) for a
 * few steps at this grid's real shape (zero state, no points) on `stream`,
 * writes the fastest into *inout (fields left 0 are searched, set fields are
 * kept) and caches it in-process and, if the environment variable
 * FD_AUTOTUNE_CACHE names a file, in that file keyed by (ndim, n, so, arch,
 * Laplacian form: "iso" for equal spacing on every axis, else "aniso").
 * Automatic plans (variant 0) of every operation on a grid with that key take
 * the cached choice from then on.
 * Synchronises the stream.  workspace must hold
 * fd_workspace_size(grid, time, NULL, NULL, NULL, FD_OP_FORWARD) for time->nt = 8.
 */
int fd_autotune(const fd_grid *grid, const fd_time *time, fd_options *inout, void *workspace,
                size_t ws_bytes, void *stream);

/*
 * fd_forward without a workspace, for callers that cannot allocate device
 * memory (code under graph capture, serving loops, harnesses that forbid
 * hipMalloc).  Arguments, results and errors as fd_forward; the scratch that
 * fd_forward carves from the caller's workspace (q, the spare fields, the point
 * tables) lives instead in a static device array of FD_NOALLOC_SCRATCH_BYTES
 * that every GPU the library runs on holds until the process ends.  The call
 * allocates nothing: it returns FD_ESCRATCH when
 * fd_workspace_size(grid, time, src, rec, opts, FD_OP_FORWARD) exceeds the
 * array (64 MiB: a 3-D grid of about 2.4e6 points with nz a multiple of 32, a
 * 2-D grid of 128 x 128 easily).  Every call on one GPU uses that GPU's one
 * array, which keeps the last call's contents (each call writes everything it
 * reads): calls that overlap on one GPU, on different streams or host
 * threads, race and must be serialised by the caller.
 */
#define FD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int fd_forward_noalloc(const fd_grid *grid, const fd_time *time, const float *v,
                       const fd_points *src, const fd_points *rec, float *rec_out,
                       float *u_state, const fd_options *opts, void *stream);

/* One shot of a batch (all pointers as in fd_forward / fd_gradient). */
typedef struct fd_shot {
    fd_grid grid;
    fd_time time;
    const float *v;       /* DEVICE [N] */
    fd_points src;        /* amp: DEVICE [nt][ns] wavelet */
    fd_points rec;        /* amp: DEVICE [nt][nr] observed data (gradient) */
    float *rec_out;       /* DEVICE [nt][nr] traces (forward) or NULL */
    float *grad_v;        /* DEVICE [N] (gradient) or NULL */
    double misfit;        /* out (gradient) */
    fd_options opts;      /* per-shot options (variant/tile/tblock; 0 = auto) */
} fd_shot;

/* Workspace for a batch: the sum over shots of fd_workspace_size, each rounded
 * up to 256 bytes, plus the device table of grouped-launch entries.  0 for no
 * shots, an invalid shot or an op other than FORWARD / GRADIENT. */
size_t fd_batch_workspace_size(int nshots, const fd_shot *shots, int op);

/*
 * Batched forward sweeps over shots of uneven grid size and space order.
 * All shots' time blocks are issued as grouped launches: one launch per
 * (space order, time-block depth) class per pass covers the tiles of every shot
 * in that class, each workgroup finding its shot and tile in a device table.  With
 * flags & FD_BATCH_GRAPH the whole sequence is captured once into a hipGraph
 * and replayed.  Synchronises the stream (stability checks and graph build).
 */
#define FD_BATCH_GRAPH 1u
int fd_forward_batch(int nshots, fd_shot *shots, void *workspace, size_t ws_bytes,
                     uint32_t batch_flags, void *stream);

/* Batched least-squares gradients (each shot as fd_gradient); misfits in shots[i].misfit. */
int fd_gradient_batch(int nshots, fd_shot *shots, void *workspace, size_t ws_bytes,
                      uint32_t batch_flags, void *stream);

/*
 * Autotuner of a batch, the grouped launches' counterpart of fd_autotune (the
 * auto-tuned blocking of the paper's control runs, Sec. 6.6.1): for each class
 * of shots of one space order whose options are automatic (variant 0), times
 * a few steps of the class's grouped forward launches under every grouped
 * kernel shape compiled for it (tile rows, rows per thread, time-block depth
 * 1..4) and two chunk lengths, and writes the fastest into the options of
 * every shot of the class (one shared kernel keeps the class's passes in one
 * grouped launch per round; the shots' flags and ckpt_every are kept).  Shots
 * with explicit options are left as they are.  The timing runs sweep the shots
 * with their sources only (no receiver or gradient buffer is written).
 * workspace: at least fd_batch_workspace_size(nshots, shots, FD_OP_FORWARD)
 * bytes (a gradient batch's workspace is larger).  Synchronises the stream.
 */
int fd_batch_autotune(int nshots, fd_shot *shots, void *workspace, size_t ws_bytes, void *stream);

/* Static text for a status code. */
const char *fd_strerror(int code);

/* ABI version (major * 100 + minor). */
int fd_version(void);

/* Writes the kernel configuration the last call on this thread used into *out
 * (variant, tile, tblock actually run).  Returns FD_OK, or FD_EINVAL if none. */
int fd_last_config(fd_options *out);

#ifdef __cplusplus
}
#endif
#endif /* FDWAVE_H */
