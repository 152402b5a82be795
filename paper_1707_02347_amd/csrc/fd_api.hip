// fd_api.hip -- host side of libfdwave.so: validation, planning, workspace
// layout, the host sweep loop, checkpointed adjoint-state gradients, the
// autotuner and the C ABI declared in include/fdwave.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fdwave.h"
#include "fd_internal.h"
#include "fd_stream_entry.h"

namespace fdw {

// ------------------------------------------------------------------ configuration registry
const StreamEntry *find_entry(const KernelKey &k)
{
    int n = 0;
    const StreamEntry *const *reg = stream_registry(&n);
    for (int i = 0; i < n; ++i) {
        const StreamEntry *e = reg[i];
        if (e->M == k.M && e->T == k.T && e->PY == k.PY && e->NW == k.NW && e->mode == k.mode) return e;
    }
    return nullptr;
}

bool launch_stream(const KernelKey &k, const SweepArgs &a, hipStream_t s)
{
    const StreamEntry *e = find_entry(k);
    return e && e->launch(a, s);
}

bool launch_stream_grouped(const KernelKey &k, bool iso, bool ntl, bool ps,
                           const GroupEntry *list, int nlist, int total, int grid, hipStream_t s)
{
    const StreamEntry *e = find_entry(k);
    return e && e->launch_group(iso, ntl, ps, list, nlist, total, grid, s);
}

// Bytes a pass re-reads every step: u^n, u^{n-1} and q, plus the image's FP32
// partial sums in imaging mode (d2 snapshots and the new field are touched
// once).
double resident_bytes(const SweepArgs &a, int mode)
{
    return (double)a.nx * (double)a.sxy * (mode == kImaging ? 16.0 : 12.0);
}

// Above this, loads of once-per-step data are non-temporal.  Measured on
// MI355X with a three-read / one-write elementwise kernel: three 96 MiB fields
// still stream at the cache's rate (7 TB/s), three 128 MiB fields at HBM's
// (5.6-6 TB/s); the sweep with non-temporal loads is 17 % slower at 256^3 and
// 7 % faster at 512^3.
constexpr double kCacheKeeps = 320.0 * 1048576.0;

// loads: -1 automatic, 0 ordinary, 1 non-temporal.  Automatic is ordinary for
// time-blocked passes: their overlapped tiles load u^{n-1} and q around the
// output tile, and the neighbouring tiles find those lines in L2 (512^3, so 2,
// T = 4: 464 GPts/s ordinary, 371 non-temporal).
bool stream_loads(int loads, double resident, int T)
{
    return loads >= 0 ? loads != 0 : (T == 1 && resident > kCacheKeeps);
}

int stream_occupancy(const KernelKey &k, bool iso, bool grouped)
{
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int, int, int, int>, int> cache;
    const auto key = std::make_tuple(k.M, k.T, k.PY, k.NW, k.mode, iso ? 1 : 0, grouped ? 1 : 0);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    const StreamEntry *e = find_entry(k);
    const int n = e ? e->occupancy(iso, grouped) : 0;
    cache[key] = n;
    return n;
}

bool stream_has(const KernelKey &k, bool iso)
{
    const StreamEntry *e = find_entry(k);
    return e && (iso || (e->flags & 1));
}

bool stream_has_group(const KernelKey &k, bool iso)
{
    const StreamEntry *e = find_entry(k);
    return e && (e->flags & 2) && (iso || (e->flags & 1));
}

const WaveEntry *find_wave(int M, int PY, int NW)
{
    int n = 0;
    const WaveEntry *const *reg = wave_registry(&n);
    for (int i = 0; i < n; ++i)
        if (reg[i]->M == M && reg[i]->PY == PY && reg[i]->NW == NW) return reg[i];
    return nullptr;
}

bool wave_has(int M, int PY, int NW) { return find_wave(M, PY, NW) != nullptr; }

bool launch_wave(int M, int PY, int NW, const SweepArgs &a, hipStream_t s)
{
    const WaveEntry *e = find_wave(M, PY, NW);
    return e && e->launch(a, s);
}

int wave_occupancy(int M, int PY, int NW, bool iso)
{
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int>, int> cache;
    const auto key = std::make_tuple(M, PY, NW, iso ? 1 : 0);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    const WaveEntry *e = find_wave(M, PY, NW);
    const int n = e ? e->occupancy(iso) : 0;
    cache[key] = n;
    return n;
}

int stream_core_rows(const KernelKey &k) { return k.NW * k.PY - 2 * k.M * (k.T - 1); }
int stream_core_cols(const KernelKey &k) { return 64 - 2 * k.M * (k.T - 1); }

namespace {

// ------------------------------------------------------------------ status helpers
struct HipFail {
    hipError_t e;
};
#define FDW_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) throw HipFail{e_};                                           \
    } while (0)

struct Status {
    int code;
};

thread_local fd_options g_last{};
thread_local bool g_last_valid = false;

// ------------------------------------------------------------------ geometry
struct Dims {
    int ndim;
    int M;
    int nx, ny, nz;        // as 3-D
    int nzp;               // row pitch of the internal fields (nz rounded up to 32 floats)
    int64_t N;             // points (the caller's dense layout)
    int64_t Np;            // floats of one internal field: nx ny nzp
    double h[3];           // spacing of the 3-D axes (1 for absent axes)
    bool present[3];
};

int make_dims(const fd_grid *g, Dims &d)
{
    if (!g) return FD_EINVAL;
    if (g->ndim < 1 || g->ndim > 3) return FD_EINVAL;
    if (g->space_order < 2 || g->space_order > 2 * kMaxM || (g->space_order & 1)) return FD_EINVAL;
    if (g->reserved != 0) return FD_EINVAL;
    d.ndim = g->ndim;
    d.M = g->space_order / 2;
    int64_t n3[3] = {1, 1, 1};
    double h3[3] = {1.0, 1.0, 1.0};
    bool p3[3] = {false, false, false};
    // 3-D: (x, y, z); 2-D: (x, 1, z); 1-D: (1, 1, z)
    static const int map[4][3] = {{0, 0, 0}, {2, 0, 0}, {0, 2, 0}, {0, 1, 2}};
    for (int a = 0; a < g->ndim; ++a) {
        if (g->n[a] < 1 || g->n[a] > (1 << 20)) return FD_EINVAL;
        if (!(g->h[a] > 0.0) || !std::isfinite(g->h[a])) return FD_EINVAL;
        const int ax = map[g->ndim][a];
        n3[ax] = g->n[a];
        h3[ax] = g->h[a];
        p3[ax] = true;
    }
    d.nx = (int)n3[0];
    d.ny = (int)n3[1];
    d.nz = (int)n3[2];
    d.N = n3[0] * n3[1] * n3[2];
    // Internal fields pad each z row to a multiple of 32 floats (128 bytes), so
    // that a wave's 64 consecutive points always span two whole cache lines;
    // the caller's arrays stay dense and are converted at the boundary.
    d.nzp = (int)((n3[2] + 31) / 32 * 32);
    d.Np = n3[0] * n3[1] * (int64_t)d.nzp;
    // one (y, z) plane must stay below 2^28 points: kernels address a plane
    // with 32-bit byte offsets (4-byte elements) and mark points outside the
    // grid with offset 2^31
    if (n3[1] * (int64_t)d.nzp >= ((int64_t)1 << 28)) return FD_EINVAL;
    for (int a = 0; a < 3; ++a) {
        d.h[a] = h3[a];
        d.present[a] = p3[a];
    }
    if (g->sponge < 0) return FD_EINVAL;
    if (g->sponge > 0) {
        if (!(g->sponge_vref > 0.0) || !std::isfinite(g->sponge_vref)) return FD_EINVAL;
        for (int a = 0; a < g->ndim; ++a)
            if (2 * (int64_t)g->sponge > g->n[a]) return FD_EINVAL;
    }
    return FD_OK;
}

// Map a user index tuple (ndim entries) onto the 3-D (x, y, z) node; -1 if outside.
int64_t node_of(const Dims &d, const int32_t *idx, int &x, int &y, int &z)
{
    int v3[3] = {0, 0, 0};
    static const int map[4][3] = {{0, 0, 0}, {2, 0, 0}, {0, 2, 0}, {0, 1, 2}};
    const int n3[3] = {d.nx, d.ny, d.nz};
    for (int a = 0; a < d.ndim; ++a) {
        const int ax = map[d.ndim][a];
        if (idx[a] < 0 || idx[a] >= n3[ax]) return -1;
        v3[ax] = idx[a];
    }
    x = v3[0];
    y = v3[1];
    z = v3[2];
    return ((int64_t)x * d.ny + y) * d.nz + z;
}

// Closed-form central second-difference weights of order 2M.
void fd_weights(int M, double *c)
{
    double sum = 0.0;
    for (int k = 1; k <= M; ++k) {
        double r = 1.0;
        for (int j = 1; j <= k; ++j) r *= double(M - k + j) / double(M + j);
        c[k] = 2.0 * ((k & 1) ? 1.0 : -1.0) * r / (double(k) * k);
        sum += c[k];
    }
    c[0] = -2.0 * sum;
}

Weights make_weights(const Dims &d)
{
    double c[kMaxM + 1];
    fd_weights(d.M, c);
    Weights w;
    std::memset(&w, 0, sizeof w);
    for (int k = 1; k <= d.M; ++k) {
        w.wx[k - 1] = d.present[0] ? (float)(c[k] / (d.h[0] * d.h[0])) : 0.0f;
        w.wy[k - 1] = d.present[1] ? (float)(c[k] / (d.h[1] * d.h[1])) : 0.0f;
        w.wz[k - 1] = d.present[2] ? (float)(c[k] / (d.h[2] * d.h[2])) : 0.0f;
    }
    // isotropic: every present axis has bit-identical weights; the kernels then
    // read the common weight from wx, so wx must hold it even if x is absent
    int npresent = 0;
    bool iso = true;
    const float *ref = nullptr;
    const float *ws[3] = {w.wx, w.wy, w.wz};
    for (int a = 0; a < 3; ++a) {
        if (!d.present[a]) continue;
        ++npresent;
        if (!ref) ref = ws[a];
        else if (std::memcmp(ref, ws[a], sizeof(float) * kMaxM) != 0) iso = false;
    }
    w.iso = iso ? 1 : 0;
    w.cc = -2.0f * (float)npresent;
    if (iso && ref != w.wx) std::memcpy(w.wx, ref, sizeof(float) * kMaxM);
    return w;
}

bool grid_iso(const Dims &d) { return make_weights(d).iso != 0; }

// Symbol of the stencil at the Nyquist wavenumber: -c0 - 2 sum_k (-1)^k c_k.
double nyquist_symbol(int M)
{
    double c[kMaxM + 1];
    fd_weights(M, c);
    double s = -c[0];
    for (int k = 1; k <= M; ++k) s -= 2.0 * ((k & 1) ? -1.0 : 1.0) * c[k];
    return s;
}

// Sponge profile of one axis divided by 2 dt:  d0 (delta/L)^2 / (2 dt),
// d0 = 1.5 ln(1000) / (vref L h).
void sponge_profile(int n, int L, double h, double vref, double dt, bool present, float *out)
{
    for (int i = 0; i < n; ++i) {
        double delta = 0.0;
        if (present && L > 0) {
            if (i < L) delta = double(L - i);
            else if (i > n - 1 - L) delta = double(i - (n - 1 - L));
        }
        double d = 0.0;
        if (delta > 0.0) {
            const double d0 = 1.5 * std::log(1000.0) / (vref * double(L) * h);
            const double r = delta / double(L);
            d = d0 * r * r;
        }
        out[i] = (float)(d / (2.0 * dt));
    }
}

// ------------------------------------------------------------------ workspace layout
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base((char *)b) {}
    template <class T>
    T *take(size_t count)
    {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

constexpr int kStatBlocks = 256;

struct TableBufs {
    int32_t *xptr, *xe, *yz, *id, *box;
    float *scale, *wt;
    // points between nodes: per point, its entries in corner order (CSR), and
    // the recorded entry values [nt][cnt]
    bool interp;
    int32_t *pptr, *pent;
    float *etr;
};

// Sizes of a point set's table: points, entries (2^ndim per point between
// nodes, an upper bound), and whether it interpolates.
struct PtsSpec {
    int n = 0;
    int ent = 0;
    bool interp = false;
};

constexpr int kMaxFields = 12;
constexpr int64_t kMaxEntries = (int64_t)1 << 27;  // interpolation entries of one point set

struct Layout {
    float *q = nullptr;
    float *prof = nullptr;          // px | py | pz
    float *fields[kMaxFields] = {}; // spare fields (ping-pong, state)
    int nfields = 0;
    TableBufs src{}, rec{};
    float *vstat = nullptr;
    double *rpart = nullptr;
    uint64_t *prog = nullptr;       // progress counters of passes without redundant halos
    int *err = nullptr;             // their error word
    int nprog = 0;
    int32_t *ptab = nullptr;        // their per-plane table ([nx][kPlaneTab])
    // gradient
    float *ckpt = nullptr;          // [nck][2][N]
    int nck = 0;
    float *seg = nullptr;           // [K][N] second differences
    double *g = nullptr;            // [N] the image (FP64)
    float *gp = nullptr;            // [N] its FP32 partial sums (kImageFlush steps at most)
    float *traces = nullptr;        // [nt][nr]
    float *resid = nullptr;         // [nt][nr]
    size_t bytes = 0;
};

TableBufs carve_table(Carver &cv, int nx, const PtsSpec &p, int64_t rows)
{
    TableBufs t{};
    const int cnt = std::max(p.ent, 1);
    t.xptr = cv.take<int32_t>(nx + 1);
    t.xe = cv.take<int32_t>(cnt);
    t.yz = cv.take<int32_t>(cnt);
    t.id = cv.take<int32_t>(cnt);
    t.scale = cv.take<float>(cnt);
    t.wt = cv.take<float>(cnt);
    t.box = cv.take<int32_t>((size_t)nx * 4);
    t.interp = p.interp;
    if (p.interp) {
        t.pptr = cv.take<int32_t>((size_t)p.n + 1);
        t.pent = cv.take<int32_t>(cnt);
        t.etr = cv.take<float>((size_t)std::max<int64_t>(rows, 1) * cnt);
    }
    return t;
}

int ckpt_interval(const fd_options *o) { return (o && o->ckpt_every > 0) ? o->ckpt_every : 50; }

Layout layout(void *ws, const Dims &d, int64_t nt, const PtsSpec &S, const PtsSpec &R, int op,
              int nfields, int K)
{
    const int ns = S.n, nr = R.n;
    Carver cv(ws);
    Layout L;
    L.q = cv.take<float>(d.Np);
    L.prof = cv.take<float>((size_t)d.nx + d.ny + d.nz);
    L.nfields = std::min(nfields, kMaxFields);
    for (int i = 0; i < L.nfields; ++i) L.fields[i] = cv.take<float>(d.Np);
    L.src = carve_table(cv, d.nx, S, nt);
    L.rec = carve_table(cv, d.nx, R, nt);
    L.vstat = cv.take<float>(3 * kStatBlocks);
    L.rpart = cv.take<double>(kStatBlocks);
    // one counter per tile of the smallest compiled tile (8 rows)
    L.nprog = ((d.nz + 63) / 64) * ((d.ny + 7) / 8);
    L.prog = cv.take<uint64_t>((size_t)L.nprog * kWaveProgStride);
    L.err = cv.take<int>(64);
    L.ptab = cv.take<int32_t>((size_t)d.nx * kPlaneTab);
    if (op == FD_OP_BORN) L.seg = cv.take<float>(d.Np);  // the background's second difference
    if (op == FD_OP_GRADIENT || op == FD_OP_VJP) {
        L.nck = nt > 0 ? (int)((nt + K - 1) / K) : 0;
        L.ckpt = cv.take<float>((size_t)std::max(L.nck, 1) * 2 * d.Np);
        L.seg = cv.take<float>((size_t)std::max(1, (int)std::min<int64_t>(K, std::max<int64_t>(nt, 1))) * d.Np);
        L.g = cv.take<double>(d.Np);
        L.gp = cv.take<float>(d.Np);
        L.traces = cv.take<float>((size_t)std::max<int64_t>(nt * nr, 1));
        L.resid = cv.take<float>((size_t)std::max<int64_t>(nt * nr, 1));
    }
    L.bytes = ((cv.off + 255) & ~(size_t)255) + 256;
    return L;
}

// Spare fields each op needs: forward 2 (state if NULL) + 2 (time-block ping-pong);
// adjoint same; gradient: forward (2 + 2 + 1 scratch) + adjoint (2 + 2).
int fields_needed(int op)
{
    switch (op) {
    case FD_OP_FORWARD:
    case FD_OP_ADJOINT: return 4;
    case FD_OP_BORN: return 9;  // background 4, perturbation 4, s
    default: return 9;
    }
}

// ------------------------------------------------------------------ planning
struct Plan {
    int variant;      // FD_VARIANT_NAIVE / STREAM / TBLOCK / SPLIT
    KernelKey key;    // for stream / tblock (mode set per use)
    int lx;
    bool remap;
    bool alt;
    int loads;        // cache policy of once-per-step loads: -1 automatic, 0 keep, 1 stream
    bool split = false;  // two-level plain passes split into trapezoids along x
    bool wave = false;   // two-level plain passes without redundant halos (fd_wave.h)
    bool wave_auto = false;  // ... chosen by the automatic plan (see kWaveAutoEntries)
};

std::mutex g_tune_mu;
std::map<std::string, fd_options> g_tune;

// Key of a tuned choice: grid extents, space order, the architecture and the
// Laplacian's form (equal spacing on every axis, or not: the two forms compile
// to different kernels, and the tuner times the grid's own).  The tuner
// times plain forward passes; the other operations run the same tile (their
// modes' kernels are compiled for the shapes the tuner searches).
std::string tune_key(const Dims &d)
{
    char buf[128];
    std::snprintf(buf, sizeof buf, "%d %d %d %d %d gfx950 %s", d.ndim, d.nx, d.ny, d.nz, 2 * d.M,
                  grid_iso(d) ? "iso" : "aniso");
    return buf;
}

void load_tune_file()
{
    static bool loaded = false;
    if (loaded) return;
    loaded = true;
    const char *path = std::getenv("FD_AUTOTUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        int nd, nx, ny, nz, so, var, t0, t1, t2, tb;
        char arch[32], form[8];
        if (std::sscanf(line, "%d %d %d %d %d %31s %7s %d %d %d %d %d", &nd, &nx, &ny, &nz, &so, arch, form,
                        &var, &t0, &t1, &t2, &tb) == 12) {
            char key[128];
            std::snprintf(key, sizeof key, "%d %d %d %d %d %s %s", nd, nx, ny, nz, so, arch, form);
            fd_options o{};
            o.variant = var;
            o.tile[0] = t0;
            o.tile[1] = t1;
            o.tile[2] = t2;
            o.tblock = tb;
            g_tune[key] = o;
        }
    }
    std::fclose(f);
}

// Compute units of the current device (256 on MI355X).
int device_cus()
{
    static int cache[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cache[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n <= 0)
            n = 256;
        cache[dev] = n;
    }
    return cache[dev];
}

bool grid_iso(const Dims &d);

// Default x-chunk.  A launch has P (y, z) tiles per plane times the number of
// chunks along x; C workgroups are resident at once (occupancy x CUs).  A last,
// partly filled round of workgroups costs as much as a full one, and every
// chunk re-reads 2 T M warm-up planes, so the chunk count maximises
//   (filled share of the rounds) / (1 + 2 T M / lx),
// with chunks of at least 4 T M planes.  (Measured on MI355X: 320^3 so 8 with
// 6 chunks of 54 planes -- 300 workgroups, 256 resident -- ran at 223 GPts/s,
// with 5 chunks of 64 at 307.)
int default_lx(const Dims &d, const KernelKey &k)
{
    const int ty = stream_core_rows(k), tz = stream_core_cols(k);
    const int64_t P = (int64_t)((d.nz + tz - 1) / tz) * ((d.ny + ty - 1) / ty);
    const int64_t C = (int64_t)std::max(1, stream_occupancy(k, grid_iso(d), false)) * device_cus();
    const int minlx = 4 * k.T * k.M;
    int best_lx = std::min(d.nx, kMaxLx);
    double best = -1.0;
    for (int ntx = 1; ntx <= d.nx; ++ntx) {
        const int lx = (d.nx + ntx - 1) / ntx;
        if (lx > kMaxLx) continue;
        if (lx < minlx && ntx > 1) break;
        const int64_t W = P * ((d.nx + lx - 1) / lx);
        const int64_t rounds = (W + C - 1) / C;
        const double score = ((double)W / (double)(rounds * C)) / (1.0 + 2.0 * k.T * k.M / lx);
        if (score > best + 1e-9) {
            best = score;
            best_lx = lx;
        }
    }
    return best_lx;
}



KernelKey default_key(const Dims &d, int T)
{
    const bool iso = grid_iso(d);
    // measured on MI355X: T = 1 wins with 4 rows per thread, in 8 waves for
    // M <= 4 and 4 waves for longer stencils (register queues of 2M + 1 planes);
    // a tall (2 rows x 16 waves) tile for T >= 2; fall back to what is compiled
    static const int pref1s[][2] = {{4, 8}, {4, 4}, {8, 4}};
    static const int pref1l[][2] = {{4, 4}, {4, 8}, {8, 4}};
    static const int pref2[][2] = {{2, 16}, {4, 8}, {8, 4}};
    for (auto &sh : (T == 1 ? (d.M <= 4 ? pref1s : pref1l) : pref2)) {
        KernelKey k{d.M, T, sh[0], sh[1], kPlain};
        if (stream_has(k, iso)) return k;
    }
    return KernelKey{d.M, 1, 8, 4, kPlain};
}

// Tiles of a pass without redundant halos: 64 columns by rows of y.
int wave_tiles(const Dims &d, int rows) { return ((d.nz + 63) / 64) * ((d.ny + rows - 1) / rows); }

// FD_VARIANT_WAVE: the tile shape (tile[1] rows of tile[2] per thread, or the
// first compiled of a preference list), admitted only if every tile's
// workgroup can be resident at once -- a pass's workgroups wait for their
// neighbours, so all of them must run together.
int wave_plan(const Dims &d, const fd_options &eff, Plan &p)
{
    if (eff.tblock != 0 && eff.tblock != 2) return FD_EINVAL;
    const bool iso = grid_iso(d);
    // preference order from 512^3 sweeps: so 8 2 x 8 380 GPts/s, 2 x 4 345;
    // 4 x 4 ran 20-35 % behind 2 x 8 (so 8 / so 16) in an earlier build, and
    // 1 x 16 (no longer compiled) 8 % behind
    static const int shapes[][2] = {{2, 8}, {2, 4}, {4, 4}};
    int PY = 0, NW = 0;
    if (eff.tile[1] > 0 || eff.tile[2] > 0) {
        PY = eff.tile[2] > 0 ? eff.tile[2] : 4;
        const int rows = eff.tile[1] > 0 ? eff.tile[1] : 16;
        if (rows % PY) return FD_EUNSUPPORTED;
        NW = rows / PY;
        if (!wave_has(d.M, PY, NW)) return FD_EUNSUPPORTED;
    } else {
        for (auto &sh : shapes)
            if (wave_has(d.M, sh[0], sh[1])) {
                PY = sh[0];
                NW = sh[1];
                break;
            }
        if (!PY) return FD_EUNSUPPORTED;
    }
    const int64_t resident = (int64_t)wave_occupancy(d.M, PY, NW, iso) * device_cus();
    if (wave_tiles(d, PY * NW) > resident) return FD_EUNSUPPORTED;
    // the kernel's plane byte offsets are 32-bit
    if (d.Np * 4 >= ((int64_t)1 << 31)) return FD_EUNSUPPORTED;
    p.key = KernelKey{d.M, 2, PY, NW, kPlain};
    p.lx = d.nx;
    p.variant = FD_VARIANT_WAVE;
    p.wave = true;
    return FD_OK;
}

int make_plan(const Dims &d, const fd_options *o, Plan &p)
{
    fd_options eff{};
    if (o) eff = *o;
    if (eff.reserved != 0) return FD_EINVAL;
    if (eff.flags & ~(uint32_t)(FD_FLAG_NO_CFL_CHECK | FD_FLAG_CHECK_FINITE | FD_FLAG_NO_XCD_REMAP |
                                FD_FLAG_NO_X_ALTERNATE | FD_FLAG_LOADS_STREAM | FD_FLAG_LOADS_KEEP))
        return FD_EINVAL;
    if ((eff.flags & FD_FLAG_LOADS_STREAM) && (eff.flags & FD_FLAG_LOADS_KEEP)) return FD_EINVAL;
    const bool automatic = eff.variant == FD_VARIANT_AUTO;
    if (eff.variant == FD_VARIANT_AUTO) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_tune_file();
        auto it = g_tune.find(tune_key(d));
        // a cached choice whose kernel this grid's form lacks is ignored
        const bool usable =
            it != g_tune.end() &&
            (it->second.variant == FD_VARIANT_NAIVE ||
             (it->second.tile[2] > 0 && it->second.tile[1] % it->second.tile[2] == 0 &&
              (it->second.variant == FD_VARIANT_WAVE
                   ? wave_has(d.M, it->second.tile[2], it->second.tile[1] / it->second.tile[2])
                   : stream_has(KernelKey{d.M, std::max(it->second.tblock, 1), it->second.tile[2],
                                          it->second.tile[1] / it->second.tile[2], kPlain},
                                grid_iso(d)))));
        if (usable) {
            const fd_options &t = it->second;
            eff.variant = t.variant;
            for (int i = 0; i < 3; ++i)
                if (!eff.tile[i]) eff.tile[i] = t.tile[i];
            if (!eff.tblock) eff.tblock = t.tblock;
        } else {
            eff.variant = (d.ndim == 3) ? FD_VARIANT_STREAM : FD_VARIANT_NAIVE;
        }
    }
    p.remap = !(eff.flags & FD_FLAG_NO_XCD_REMAP);
    p.alt = !(eff.flags & FD_FLAG_NO_X_ALTERNATE);
    p.loads = (eff.flags & FD_FLAG_LOADS_STREAM) ? 1 : (eff.flags & FD_FLAG_LOADS_KEEP) ? 0 : -1;
    p.variant = eff.variant;
    if (eff.variant == FD_VARIANT_NAIVE) {
        p.key = KernelKey{d.M, 1, 1, 1, kPlain};
        p.lx = d.nx;
        return FD_OK;
    }
    if (eff.variant == FD_VARIANT_WAVE) {
        const int rc = wave_plan(d, eff, p);
        if (rc == FD_OK) p.wave_auto = automatic;
        // a cached choice this device cannot run (fewer compute units than the
        // one it was tuned on) falls back to the default plan
        if (rc != FD_EUNSUPPORTED || !automatic) return rc;
        eff = fd_options{};
        if (o) eff.flags = o->flags;
        eff.variant = (d.ndim == 3) ? FD_VARIANT_STREAM : FD_VARIANT_NAIVE;
        p.variant = eff.variant;
        p.wave = false;
        if (eff.variant == FD_VARIANT_NAIVE) {
            p.key = KernelKey{d.M, 1, 1, 1, kPlain};
            p.lx = d.nx;
            return FD_OK;
        }
    }
    if (eff.variant != FD_VARIANT_STREAM && eff.variant != FD_VARIANT_TBLOCK && eff.variant != FD_VARIANT_SPLIT)
        return FD_EINVAL;
    int T = 1;
    if (eff.variant == FD_VARIANT_TBLOCK) T = eff.tblock > 0 ? eff.tblock : 2;
    if (eff.variant == FD_VARIANT_SPLIT) {
        if (eff.tblock != 0 && eff.tblock != 2) return FD_EINVAL;
        T = 2;
    }
    if (T < 1 || T > 4) return FD_EINVAL;
    KernelKey k;
    if (eff.tile[1] > 0 || eff.tile[2] > 0) {
        const int PY = eff.tile[2] > 0 ? eff.tile[2] : 8;
        const int rows = eff.tile[1] > 0 ? eff.tile[1] : 32;
        if (rows % PY) return FD_EUNSUPPORTED;
        k = KernelKey{d.M, T, PY, rows / PY, kPlain};
        if (!stream_has(k, grid_iso(d))) return FD_EUNSUPPORTED;
    } else {
        k = default_key(d, T);
        if (k.T != T) {
            if (eff.variant == FD_VARIANT_TBLOCK && eff.tblock > 0) return FD_EUNSUPPORTED;
        }
    }
    p.key = k;
    p.variant = (k.T >= 2) ? FD_VARIANT_TBLOCK : FD_VARIANT_STREAM;
    p.lx = eff.tile[0] > 0 ? std::min(std::min(eff.tile[0], d.nx), kMaxLx) : default_lx(d, k);
    if (eff.variant == FD_VARIANT_SPLIT) {
        if (k.T != 2) return FD_EUNSUPPORTED;
        // an upright trapezoid needs level 2 on at least one plane of its chunk
        p.lx = std::max(p.lx, std::min(d.nx, 2 * k.M + 1));
        p.variant = FD_VARIANT_SPLIT;
        p.split = true;
    }
    return FD_OK;
}

// Key with the same tile for another mode / depth; otherwise the first compiled
// shape of a preference list at depth T, then at depth 1.
KernelKey key_for(const KernelKey &base, int T, int mode, bool iso)
{
    KernelKey k = base;
    k.T = T;
    k.mode = mode;
    if (stream_has(k, iso)) return k;
    static const int shapes[][2] = {{4, 8}, {2, 16}, {4, 4}, {8, 4}};
    for (int t : {T, 1}) {
        for (auto &sh : shapes) {
            k = KernelKey{base.M, t, sh[0], sh[1], mode};
            if (stream_has(k, iso)) return k;
        }
    }
    return KernelKey{base.M, 1, 8, 4, mode};
}

// A compiled shape of the same radius, depth and mode whose kernel can stage
// point entries in LDS, in order of preference; M = 0 if there is none.
KernelKey stageable_key(const KernelKey &k, bool iso)
{
    static const int shapes[][2] = {{4, 8}, {4, 4}, {8, 4}, {2, 8}};
    for (auto &sh : shapes) {
        const KernelKey c{k.M, k.T, sh[0], sh[1], k.mode};
        if (points_stageable(c.M, c.T, c.PY, c.NW) && stream_has(c, iso)) return c;
    }
    return KernelKey{0, 0, 0, 0, 0};
}

// ------------------------------------------------------------------ point tables
struct Entry {
    int x, y, z, id;
    int corner;  // order of the point's nodes: multilinear bit 2 +x, bit 1 +y, bit 0 +z from the
                 // cell's lowest node; windowed sinc (i * 16 + j) * 16 + k
    float wt;
};

// The nodes of the cell that holds a position (ndim coordinates in grid-index
// units) with their multilinear weights prod_a (c_a ? f_a : 1 - f_a), nodes of
// weight zero left out (an integer position keeps one node of weight 1); -1 if
// a coordinate is not finite or lies outside [0, n - 1].
int cell_of(const Dims &d, const double *pos, int id, std::vector<Entry> &out)
{
    static const int map[4][3] = {{0, 0, 0}, {2, 0, 0}, {0, 2, 0}, {0, 1, 2}};
    const int n3[3] = {d.nx, d.ny, d.nz};
    int base[3] = {0, 0, 0};
    double f[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d.ndim; ++a) {
        const int ax = map[d.ndim][a];
        const double x = pos[a];
        if (!(x >= 0.0) || !(x <= (double)(n3[ax] - 1))) return -1;
        int i = (int)std::floor(x);
        i = std::max(0, std::min(i, n3[ax] - 2));  // the last node: the cell below, f = 1
        base[ax] = i;
        f[ax] = x - (double)i;
    }
    for (int c = 0; c < 8; ++c) {
        double w = 1.0;
        int node[3];
        for (int ax = 0; ax < 3; ++ax) {
            const int bit = (c >> (2 - ax)) & 1;
            node[ax] = base[ax] + bit;
            w *= bit ? f[ax] : 1.0 - f[ax];
        }
        if (w == 0.0) continue;
        out.push_back(Entry{node[0], node[1], node[2], id, c, (float)w});
    }
    return 0;
}

// Kaiser-windowed sinc (Hicks 2002): along one axis a point at x weighs the 2r
// nodes floor(x) - r + 1 .. floor(x) + r by sinc(d) I0(b sqrt(1 - (d/r)^2)) / I0(b),
// d = node - x.  b(r) minimises the largest error of interpolating a cosine of
// wavenumber up to pi / (2h) (four points per wavelength), found by a search
// over b in steps of 0.1.
constexpr int kSincMax = 8;
constexpr double kWindowShape[kSincMax + 1] = {0.0, 1.3, 2.9, 4.5, 6.3, 7.9, 9.4, 10.9, 12.6};

double bessel_i0(double x)
{
    // power series of I0: terms ((x/2)^j / j!)^2, each the last times (x/2)^2 / j^2
    const double q = 0.25 * x * x;
    double sum = 1.0, t = 1.0;
    for (int j = 1; j <= 200 && t > 1e-17 * sum; ++j) {
        t = t * q / ((double)j * j);
        sum += t;
    }
    return sum;
}

// The 1-D weights of the 2r nodes from lo = floor(x) - r + 1; nodes outside
// [0, n - 1] get weight 0 (the field is zero there).
void sinc_axis(double x, int r, int n, int &lo, double *w)
{
    const int i0 = (int)std::floor(x);
    lo = i0 - r + 1;
    const double norm = 1.0 / bessel_i0(kWindowShape[r]);
    for (int k = 0; k < 2 * r; ++k) {
        const int node = lo + k;
        const double dx = (double)node - x;
        if (node < 0 || node >= n) {
            w[k] = 0.0;
            continue;
        }
        // sinc is exactly 1 at distance 0 and 0 at the other integers
        const double sn = dx == 0.0 ? 1.0
                          : dx == std::trunc(dx) ? 0.0
                                                 : std::sin(M_PI * dx) / (M_PI * dx);
        const double rho = dx / r;
        w[k] = rho * rho < 1.0 ? sn * bessel_i0(kWindowShape[r] * std::sqrt(1.0 - rho * rho)) * norm : 0.0;
    }
}

// The nodes of a point's windowed-sinc stencil (half-width r) with their
// weights, the products of the per-axis weights; zero weights left out.  The
// entry's corner code is the node's rank in x-major order within the 2r-cube.
int sinc_of(const Dims &d, const double *pos, int r, int id, std::vector<Entry> &out)
{
    static const int map[4][3] = {{0, 0, 0}, {2, 0, 0}, {0, 2, 0}, {0, 1, 2}};
    const int n3[3] = {d.nx, d.ny, d.nz};
    int lo[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
    double w[3][2 * kSincMax];
    w[0][0] = w[1][0] = w[2][0] = 1.0;
    for (int a = 0; a < d.ndim; ++a) {
        const int ax = map[d.ndim][a];
        const double x = pos[a];
        if (!(x >= 0.0) || !(x <= (double)(n3[ax] - 1))) return -1;
        sinc_axis(x, r, n3[ax], lo[ax], w[ax]);
        cnt[ax] = 2 * r;
    }
    for (int i = 0; i < cnt[0]; ++i)
        for (int j = 0; j < cnt[1]; ++j)
            for (int k = 0; k < cnt[2]; ++k) {
                const double wt = w[0][i] * w[1][j] * w[2][k];
                if (wt == 0.0) continue;
                out.push_back(Entry{lo[0] + i, lo[1] + j, lo[2] + k, id, (i * 16 + j) * 16 + k, (float)wt});
            }
    return 0;
}

int64_t nodes_per_point(const Dims &d, const fd_points *p)
{
    if (!p->pos) return 1;
    const int64_t side = p->interp > 0 ? 2 * p->interp : 2;
    int64_t c = 1;
    for (int a = 0; a < d.ndim; ++a) c *= side;
    return c;
}

PtsSpec spec_of(const Dims &d, const fd_points *p)
{
    PtsSpec s;
    if (!p || p->n <= 0) return s;
    s.n = p->n;
    s.interp = p->pos != nullptr;
    s.ent = (int)std::min<int64_t>((int64_t)p->n * nodes_per_point(d, p), kMaxEntries);
    return s;
}

int build_table(const Dims &d, const fd_points *pts, std::vector<Entry> &ent)
{
    ent.clear();
    if (!pts || pts->n == 0) return FD_OK;
    if (pts->n < 0 || (!pts->idx == !pts->pos)) return FD_EINVAL;
    if (pts->interp < 0 || pts->interp > kSincMax || (pts->interp && !pts->pos)) return FD_EINVAL;
    for (int i = 0; i < pts->n; ++i) {
        if (pts->pos) {
            const double *x = pts->pos + (size_t)i * d.ndim;
            if ((pts->interp ? sinc_of(d, x, pts->interp, i, ent) : cell_of(d, x, i, ent)) < 0)
                return FD_EDOM;
            continue;
        }
        int x, y, z;
        if (node_of(d, pts->idx + (size_t)i * d.ndim, x, y, z) < 0) return FD_EDOM;
        ent.push_back(Entry{x, y, z, i, 0, 1.0f});
    }
    std::stable_sort(ent.begin(), ent.end(), [](const Entry &a, const Entry &b) {
        if (a.x != b.x) return a.x < b.x;
        if (a.y != b.y) return a.y < b.y;
        if (a.z != b.z) return a.z < b.z;
        return a.id < b.id;
    });
    return FD_OK;
}

int check_position(const Dims &d, const double *pos)
{
    std::vector<Entry> tmp;
    return cell_of(d, pos, 0, tmp);
}

// Host staging of a table; kept alive until the copies are enqueued (pageable
// copies are staged by the runtime before hipMemcpyAsync returns).
void upload_table(const Dims &d, const std::vector<Entry> &ent, const TableBufs &b, int npts,
                  std::vector<int32_t> *host_xptr, hipStream_t s, std::vector<int32_t> *host_yz = nullptr,
                  std::vector<int32_t> *host_id = nullptr)
{
    std::vector<int32_t> xptr(d.nx + 1, 0), xe(ent.size()), yz(ent.size()), id(ent.size());
    std::vector<float> wt(ent.size());
    // per-plane bounding box of the entries, so that a tile skips the planes
    // whose points it cannot hold without reading their entries
    std::vector<int32_t> box((size_t)d.nx * 4);
    for (int x = 0; x < d.nx; ++x) {
        box[4 * x + 0] = box[4 * x + 2] = 1;
        box[4 * x + 1] = box[4 * x + 3] = 0;
    }
    std::vector<bool> seen(d.nx, false);
    for (size_t j = 0; j < ent.size(); ++j) {
        const Entry &e = ent[j];
        xptr[e.x + 1]++;
        xe[j] = e.x;
        yz[j] = e.y * d.nzp + e.z;
        id[j] = e.id;
        wt[j] = e.wt;
        int32_t *bx = &box[4 * (size_t)e.x];
        if (!seen[e.x]) {
            bx[0] = bx[1] = e.y;
            bx[2] = bx[3] = e.z;
            seen[e.x] = true;
        } else {
            bx[0] = std::min(bx[0], e.y);
            bx[1] = std::max(bx[1], e.y);
            bx[2] = std::min(bx[2], e.z);
            bx[3] = std::max(bx[3], e.z);
        }
    }
    for (int x = 0; x < d.nx; ++x) xptr[x + 1] += xptr[x];
    if (host_xptr) *host_xptr = xptr;
    if (host_yz) *host_yz = yz;
    if (host_id) *host_id = id;
    FDW_HIP(hipMemcpyAsync(b.xptr, xptr.data(), xptr.size() * 4, hipMemcpyHostToDevice, s));
    if (!ent.empty()) {
        FDW_HIP(hipMemcpyAsync(b.xe, xe.data(), xe.size() * 4, hipMemcpyHostToDevice, s));
        FDW_HIP(hipMemcpyAsync(b.yz, yz.data(), yz.size() * 4, hipMemcpyHostToDevice, s));
        FDW_HIP(hipMemcpyAsync(b.id, id.data(), id.size() * 4, hipMemcpyHostToDevice, s));
        FDW_HIP(hipMemcpyAsync(b.box, box.data(), box.size() * 4, hipMemcpyHostToDevice, s));
        FDW_HIP(hipMemcpyAsync(b.wt, wt.data(), wt.size() * 4, hipMemcpyHostToDevice, s));
    }
    std::vector<int32_t> pptr, pent;
    if (b.interp && npts > 0) {
        // entries of each point, in corner order: the order of the sums that
        // turn recorded entry values into traces
        std::vector<std::vector<std::pair<int, int>>> per(npts);
        for (size_t j = 0; j < ent.size(); ++j) per[ent[j].id].push_back({ent[j].corner, (int)j});
        pptr.assign(npts + 1, 0);
        for (int p = 0; p < npts; ++p) {
            std::sort(per[p].begin(), per[p].end());
            pptr[p + 1] = pptr[p] + (int)per[p].size();
            for (auto &cj : per[p]) pent.push_back(cj.second);
        }
        FDW_HIP(hipMemcpyAsync(b.pptr, pptr.data(), pptr.size() * 4, hipMemcpyHostToDevice, s));
        if (!pent.empty())
            FDW_HIP(hipMemcpyAsync(b.pent, pent.data(), pent.size() * 4, hipMemcpyHostToDevice, s));
    }
    FDW_HIP(hipStreamSynchronize(s));
}

// The per-plane table of passes without redundant halos: per x-plane the
// sponge profile, the source and receiver entry ranges, whether they are
// non-empty, and the plane's first receiver entry (its node and its output
// slot: an entry index when receivers interpolate, else the receiver's column)
// (one vector load per iteration reads it, lane k holding slot k).
void upload_planes(const Dims &d, const float *px, const std::vector<int32_t> &xs,
                   const std::vector<int32_t> &xr, int32_t *dst, hipStream_t s,
                   const std::vector<int32_t> &ryz = {}, const std::vector<int32_t> &rid = {},
                   bool rinterp = false)
{
    std::vector<int32_t> t((size_t)d.nx * kPlaneTab, 0);
    for (int c = 0; c < d.nx; ++c) {
        int32_t *e = &t[(size_t)c * kPlaneTab];
        std::memcpy(&e[0], &px[c], 4);
        e[1] = xs.size() > (size_t)c + 1 ? xs[c] : 0;
        e[2] = xs.size() > (size_t)c + 1 ? xs[c + 1] : 0;
        e[3] = xr.size() > (size_t)c + 1 ? xr[c] : 0;
        e[4] = xr.size() > (size_t)c + 1 ? xr[c + 1] : 0;
        e[5] = (e[2] > e[1] ? 1 : 0) | (e[4] > e[3] ? 2 : 0);
        if (e[4] > e[3] && (size_t)e[3] < ryz.size() && (size_t)e[3] < rid.size()) {
            e[6] = ryz[e[3]];
            e[7] = rinterp ? e[3] : rid[e[3]];
        }
    }
    FDW_HIP(hipMemcpyAsync(dst, t.data(), t.size() * 4, hipMemcpyHostToDevice, s));
    FDW_HIP(hipStreamSynchronize(s));
}

PointTable as_table(const TableBufs &b, int stride, int cnt, bool with_scale)
{
    PointTable t;
    t.xptr = b.xptr;
    t.xe = b.xe;
    t.yz = b.yz;
    t.id = b.id;
    t.scale = with_scale ? b.scale : nullptr;
    t.wt = b.wt;
    t.etr = b.interp ? b.etr : nullptr;
    t.box = b.box;
    t.stride = stride;
    t.cnt = cnt;
    return t;
}

// ------------------------------------------------------------------ execution
// Device work of a sweep is issued through an Exec: immediately on its stream,
// or recorded as a list of ops (kernel passes kept as (key, arguments) so that
// a batch can merge the passes of many shots into grouped launches).
struct Op {
    bool is_pass = false;
    KernelKey key{};
    SweepArgs a{};
    int loads = -1;  // the plan's cache policy of once-per-step loads
    std::function<hipError_t(hipStream_t)> call;
};

struct Exec {
    hipStream_t s = nullptr;
    std::vector<Op> *rec = nullptr;
    void pass(const KernelKey &k, const SweepArgs &a, int loads)
    {
        if (!stream_has(k, a.w.iso != 0)) throw Status{FD_EUNSUPPORTED};
        if (rec) {
            Op o;
            o.is_pass = true;
            o.key = k;
            o.a = a;
            o.loads = loads;
            rec->push_back(std::move(o));
            return;
        }
        launch_stream(k, a, s);
        FDW_HIP(hipGetLastError());
    }
    // a pass without redundant halos (issued immediately only: its
    // workgroups wait for each other, so it is never merged into a batch)
    void wave(const KernelKey &k, const SweepArgs &a)
    {
        if (rec || !launch_wave(k.M, k.PY, k.NW, a, s)) throw Status{FD_EUNSUPPORTED};
        FDW_HIP(hipGetLastError());
    }
    template <class F>
    void call(F f)
    {
        if (rec) {
            Op o;
            o.call = f;
            rec->push_back(std::move(o));
            return;
        }
        FDW_HIP(f(s));
    }
};

hipError_t copy_async(float *dst, const float *src, int64_t n, hipStream_t s)
{
    return hipMemcpyAsync(dst, src, (size_t)n * 4, hipMemcpyDeviceToDevice, s);
}

// ------------------------------------------------------------------ per-call context
struct Ctx {
    Dims d;
    int64_t nt;
    double dt;
    hipStream_t s;
    Exec ex;
    Plan plan;
    Layout L;
    SweepArgs base;   // common launch arguments
    std::vector<int32_t> hxs, hxr;  // host copies of the point tables' plane pointers
    int64_t rec_extra = 0;          // receiver entries beyond the first of each plane
    int ran_T = 0;    // deepest time block a pass of this call used (0: none yet)
    bool ran_split = false;  // a pass of this call ran split along x
    uint32_t wave_epoch = 0;  // passes without redundant halos issued so far
};

// Whether a pass walks its point entries staged in LDS: a configuration that
// can stage, a table large enough to be worth it, and every chunk's entries
// (its planes, with the 2 (T - 1) M overlap planes of a time block) within
// the capacity, since the staged form of the kernel has no other walk.
bool fits_chunks(const Ctx &c, const KernelKey &k, const SweepArgs &a, const PointTable &t)
{
    if (t.cnt == 0) return true;
    const int cap = kPtsCap / k.T, H = (k.T - 1) * k.M;
    const std::vector<int32_t> *hx = (t.xptr == c.L.src.xptr)   ? &c.hxs
                                     : (t.xptr == c.L.rec.xptr) ? &c.hxr
                                                                : nullptr;
    if (!hx || hx->size() != (size_t)a.nx + 1) return false;
    for (int x0 = 0; x0 < a.nx; x0 += a.lx) {
        const int xend = std::min(x0 + a.lx, a.nx);
        const int c0 = std::max(x0 - H, 0), c1 = std::min(xend + H, a.nx);
        if ((*hx)[c1] - (*hx)[c0] > cap) return false;
    }
    return true;
}

bool stage_points(const Ctx &c, const KernelKey &k, const SweepArgs &a)
{
    if (!points_stageable(k.M, k.T, k.PY, k.NW)) return false;
    if (a.inj.cnt <= kStageMin && a.rec.cnt <= kStageMin) return false;
    return fits_chunks(c, k, a, a.inj) && fits_chunks(c, k, a, a.rec);
}

// A point table no chunk could stage: more than kPtsCap entries within some
// kHeavySpan consecutive planes (dense receiver planes, windowed-sinc points by
// the hundred).  Walked inside the tiled kernel it would cost one serial
// iteration per entry on every plane that holds them, so the steps take
// another route (single-level passes): receivers are recorded by a per-entry
// kernel after the pass; an injected table is added by one after a plain-mode
// pass, which the untiled path's recording and second-difference or imaging
// kernels follow.  Every route gives the same bits.
constexpr int kHeavySpan = 32;

// In a plain single-level pass an injected table of more than this many
// entries is also added after the pass (k_inject) rather than staged: on the
// 256^3 so-8 sweep 64 / 256 multilinear sources ran at 309 / 210 GPts/s staged
// and 347 / 344 injected after the pass, one windowed-sinc source (512 nodes)
// 321 vs 351.  Time-blocked passes keep staging such tables (routing them out
// would drop the pass to one level), and so do the modes that save second
// differences or image, whose alternative re-reads fields.
constexpr int kRouteInjPlain = 256;

// An automatic plan runs a pass as an exchange pass (fd_wave.h) only with at
// most this many injected entries and this many receiver entries beyond the
// first of each plane.  A plane's first receiver entry comes with the
// per-plane table; every other entry is read from memory by the workgroups on
// that plane, and a load there waits for all of their prefetches, so the
// workgroup holding many entries slows down, and its neighbours, which wait
// for its level 1, run at its pace.  At 512^3 with a line of 256 receivers
// along x the exchange form ran 362 GPts/s at so 8 against 337 for the
// single-level kernel (413 against 333 at so 4); before the first entry came
// with the table, 314 at so 8.  Injecting at those 256 points (the adjoint):
// 289 against 328.
constexpr int64_t kWaveAutoEntries = 64;

bool heavy_table(const Ctx &c, const PointTable &t)
{
    if (t.cnt <= kPtsCap) return false;
    const std::vector<int32_t> *hx = (t.xptr == c.L.src.xptr)   ? &c.hxs
                                     : (t.xptr == c.L.rec.xptr) ? &c.hxr
                                                                : nullptr;
    if (!hx || hx->size() < 2) return false;
    const int nx = (int)hx->size() - 1;
    for (int x = 0; x < nx; ++x)
        if ((*hx)[std::min(x + kHeavySpan, nx)] - (*hx)[x] > kPtsCap) return true;
    return false;
}

int validate_common(const fd_grid *g, const fd_time *t, const float *v, Dims &d)
{
    int rc = make_dims(g, d);
    if (rc) return rc;
    if (!t || t->nt < 0 || t->nt > (int64_t)1 << 30 || !(t->dt > 0.0) || !std::isfinite(t->dt))
        return FD_EINVAL;
    if (!v) return FD_EINVAL;
    return FD_OK;
}

int check_points(const Dims &d, const fd_points *p, bool need_amp, int64_t nt)
{
    if (!p) return FD_OK;
    if (p->n < 0) return FD_EINVAL;
    if (p->n > 0 && !p->idx == !p->pos) return FD_EINVAL;  // exactly one of idx, pos
    if (p->interp < 0 || p->interp > kSincMax || (p->interp && p->n > 0 && !p->pos)) return FD_EINVAL;
    if (p->n > (1 << 24)) return FD_EINVAL;
    if ((int64_t)p->n * nodes_per_point(d, p) > kMaxEntries) return FD_EINVAL;
    if (need_amp && p->n > 0 && nt > 0 && !p->amp) return FD_EINVAL;
    for (int i = 0; i < p->n; ++i) {
        if (p->pos) {
            if (check_position(d, p->pos + (size_t)i * d.ndim) < 0) return FD_EDOM;
            continue;
        }
        int x, y, z;
        if (node_of(d, p->idx + (size_t)i * d.ndim, x, y, z) < 0) return FD_EDOM;
    }
    return FD_OK;
}

// Prepare q, sponge profiles, weights, point tables and the stability check.
int prepare(Ctx &c, const fd_grid *g, const float *v, const fd_points *inj, float inj_alpha,
            const fd_points *rec, uint32_t flags)
{
    const Dims &d = c.d;
    FDW_HIP(launch_make_q(v, c.L.q, (int64_t)d.nx * d.ny, d.nz, d.nzp, c.dt * c.dt, c.s));
    std::vector<float> prof((size_t)d.nx + d.ny + d.nz);
    sponge_profile(d.nx, g->sponge, d.h[0], g->sponge_vref, c.dt, d.present[0], prof.data());
    sponge_profile(d.ny, g->sponge, d.h[1], g->sponge_vref, c.dt, d.present[1], prof.data() + d.nx);
    sponge_profile(d.nz, g->sponge, d.h[2], g->sponge_vref, c.dt, d.present[2],
                   prof.data() + d.nx + d.ny);
    FDW_HIP(hipMemcpyAsync(c.L.prof, prof.data(), prof.size() * 4, hipMemcpyHostToDevice, c.s));

    // v statistics: non-finite / non-positive values and the stability limit
    if (!(flags & FD_FLAG_NO_CFL_CHECK)) {
        FDW_HIP(launch_vstats(v, d.N, c.L.vstat, kStatBlocks, c.s));
        std::vector<float> st(3 * kStatBlocks);
        FDW_HIP(hipMemcpyAsync(st.data(), c.L.vstat, st.size() * 4, hipMemcpyDeviceToHost, c.s));
        FDW_HIP(hipStreamSynchronize(c.s));
        float vmax = 0.0f, bad = 0.0f;
        for (int b = 0; b < kStatBlocks; ++b) {
            vmax = std::max(vmax, st[3 * b]);
            bad += st[3 * b + 2];
        }
        if (bad > 0.0f) return FD_ENONFINITE;
        double inv_h2 = 0.0;
        for (int a = 0; a < 3; ++a)
            if (d.present[a]) inv_h2 += 1.0 / (d.h[a] * d.h[a]);
        const double lhs = (double)vmax * vmax * c.dt * c.dt * nyquist_symbol(d.M) * inv_h2;
        if (lhs > 4.0 * (1.0 + 1e-12)) return FD_ECFL;
    }

    std::vector<Entry> es, er;
    int rc = build_table(d, inj, es);
    if (rc) return rc;
    rc = build_table(d, rec, er);
    if (rc) return rc;
    std::vector<int32_t> ryz, rid;
    upload_table(d, es, c.L.src, inj ? inj->n : 0, &c.hxs, c.s);
    upload_table(d, er, c.L.rec, rec ? rec->n : 0, &c.hxr, c.s, &ryz, &rid);
    upload_planes(d, prof.data(), c.hxs, c.hxr, c.L.ptab, c.s, ryz, rid, c.L.rec.interp);
    c.rec_extra = 0;
    for (size_t x = 0; x + 1 < c.hxr.size(); ++x) c.rec_extra += std::max(0, c.hxr[x + 1] - c.hxr[x] - 1);

    SweepArgs &a = c.base;
    std::memset(&a, 0, sizeof a);
    a.nx = d.nx;
    a.ny = d.ny;
    a.nz = d.nz;
    a.nzp = d.nzp;
    a.sxy = (int64_t)d.ny * d.nzp;
    a.w = make_weights(d);
    a.q = c.L.q;
    a.px = c.L.prof;
    a.py = c.L.prof + d.nx;
    a.pz = c.L.prof + d.nx + d.ny;
    a.inj = as_table(c.L.src, inj ? inj->n : 0, (int)es.size(), true);
    a.rec = as_table(c.L.rec, rec ? rec->n : 0, (int)er.size(), false);
    a.rscale = 1.0f;
    a.adir = 1;
    a.rdir = 1;
    a.ptab = c.L.ptab;
    FDW_HIP(launch_entry_x(a.inj, d.nx, c.L.src.xe, c.s));
    FDW_HIP(launch_entry_x(a.rec, d.nx, c.L.rec.xe, c.s));
    FDW_HIP(launch_scales(a, a.inj, c.L.src.scale, inj_alpha, c.s));
    return FD_OK;
}

// ------------------------------------------------------------------ the host sweep loop
// State of a running sweep: (cur, prev) plus spare fields for ping-pong.
struct State {
    float *cur, *prev;
    float *spare[3];
    int nspare;
};

void swap_in(State &st, float *ncur, float *nprev)
{
    // keep every pointer exactly once among cur, prev and spares
    float *all[5] = {st.cur, st.prev, st.spare[0], st.spare[1], st.spare[2]};
    const int total = 2 + st.nspare;
    st.cur = ncur;
    st.prev = nprev;
    int k = 0;
    for (int i = 0; i < total; ++i)
        if (all[i] != ncur && all[i] != nprev) st.spare[k++] = all[i];
}

struct StepOpts {
    int mode = kPlain;       // kPlain / kSaveD2 / kImaging
    int64_t dslot_first = 0; // d2 slot of the first step in the range
    int ddir = 1;
};

// Super-tile of the XCD-aware tile order (see SweepArgs::remap): gx x-chunks by
// gy y-tiles by all z-tiles, with a multiple of 8 super-tiles.  Among the
// admissible shapes, pick the one whose faces to other XCDs re-read the least
// of u per tile: a y face costs M rows of (RZ + 2M) columns (the halo band
// and the lines its ends touch) against RY x RZ owned points, an x face costs
// T M warm-up planes against lx planes.
// Without an admissible shape the hardware order is kept.
void supertile(const KernelKey &k, SweepArgs &a)
{
    a.gx = a.gy = 1;
    if (!a.remap) return;
    const double RY = k.NW * k.PY, RZ = 64.0;
    double best = 1e300;
    int bgx = 0, bgy = 0;
    for (int gx = 1; gx <= a.ntx; ++gx) {
        if (a.ntx % gx) continue;
        for (int gy = 1; gy <= a.nty; ++gy) {
            if (a.nty % gy || ((a.ntx / gx) * (a.nty / gy)) % 8) continue;
            const double cy = (gy == a.nty) ? 0.0 : 2.0 / gy * k.M * (RZ + 2 * k.M) / (RY * RZ);
            const double cx = (gx == a.ntx) ? 0.0 : 2.0 / gx * (double)(k.T * k.M) / a.lx;
            const double cost = cy + cx;
            if (cost < best - 1e-12 || (cost < best + 1e-12 && gx > bgx)) {
                best = cost;
                bgx = gx;
                bgy = gy;
            }
        }
    }
    if (!bgx) {
        a.remap = 0;
        return;
    }
    a.gx = bgx;
    a.gy = bgy;
}

// Advance `nsteps` steps, the first one being global step index `step0`.
void advance(Ctx &c, State &st, int64_t step0, int64_t nsteps, const StepOpts &so)
{
    const Dims &d = c.d;
    int64_t s = 0;
    while (s < nsteps) {
        SweepArgs a = c.base;
        a.step0 = (int)(step0 + s);
        a.d2 = c.L.seg;
        a.dslot0 = so.dslot_first + (int64_t)so.ddir * s;
        a.ddir = so.ddir;
        a.g = c.L.gp;
        // an injected table no chunk can stage: the tiled pass runs without it
        // in the plain mode and the untiled path's injection, recording and
        // second-difference or imaging kernels follow (its own order); only
        // modes whose update itself needs the injected values fall back to the
        // untiled step
        const bool imode = so.mode == kPlain || so.mode == kSaveD2 || so.mode == kImaging;
        const bool iheavy = heavy_table(c, a.inj);
        if (c.plan.variant == FD_VARIANT_NAIVE || (iheavy && !imode)) {
            a.u0 = st.cur;
            a.um = st.prev;
            float *out = (so.mode == kSaveD2) ? st.spare[0] : st.prev;
            a.o1 = out;
            const int M = d.M, mode = so.mode;
            float *cur = st.cur, *prev = st.prev, *d2 = a.d2 ? a.d2 + a.dslot0 * d.Np : nullptr;
            c.ex.call([a, M, out, cur, prev, d2, mode](hipStream_t s) {
                hipError_t e = launch_naive_step(M, a, s);
                if (e == hipSuccess) e = launch_inject(a, out, a.step0, s);
                if (e == hipSuccess) e = launch_record(a, out, a.step0, s);
                if (e == hipSuccess && mode == kSaveD2) e = launch_save_d2(a, out, cur, prev, d2, s);
                if (e == hipSuccess && mode == kImaging) e = launch_imaging(a, out, d2, a.g, s);
                return e;
            });
            swap_in(st, out, st.cur);
            s += 1;
            continue;
        }
        // receivers recorded after the pass need its output level in memory
        bool isep = iheavy, rsep = iheavy || heavy_table(c, a.rec);
        const bool iso = c.base.w.iso != 0;
        // two levels without redundant halos: plain passes with both steps
        // left, issued immediately, whose point tables need no separate route
        // (such tables and single-step tails take the passes below)
        if (c.plan.wave && !c.ex.rec && so.mode == kPlain && !isep && !rsep && nsteps - s >= 2 &&
            a.inj.xptr == c.L.src.xptr && a.rec.xptr == c.L.rec.xptr && a.ptab == c.L.ptab &&
            !(c.plan.wave_auto && ((int64_t)a.inj.cnt > kWaveAutoEntries || c.rec_extra > kWaveAutoEntries))) {
            const KernelKey &k = c.plan.key;
            a.u0 = st.cur;
            a.um = st.prev;
            a.o1 = st.spare[0];  // u^{n+2}
            a.o2 = st.spare[1];  // u^{n+1}: the exchanged level
            a.lx = d.nx;
            a.ntx = 1;
            a.ntz = (d.nz + 63) / 64;
            a.nty = (d.ny + k.NW * k.PY - 1) / (k.NW * k.PY);
            if (a.ntz * a.nty > c.L.nprog) throw Status{FD_EUNSUPPORTED};
            a.remap = c.plan.remap ? 1 : 0;
            a.prog = c.L.prog;
            a.err = c.L.err;
            a.epoch = ++c.wave_epoch;
            if (a.epoch == 1) {
                // counters start below every epoch; no error yet
                uint64_t *prog = c.L.prog;
                int *err = c.L.err;
                const int64_t nb = (int64_t)c.L.nprog * kWaveProgStride * 8;
                c.ex.call([prog, err, nb](hipStream_t s) {
                    hipError_t e = launch_zero(prog, nb, s);
                    return e == hipSuccess ? launch_zero(err, 256, s) : e;
                });
            }
            c.ex.wave(k, a);
            swap_in(st, a.o1, a.o2);
            c.ran_T = std::max(c.ran_T, 2);
            s += 2;
            continue;
        }
        const SweepArgs a0 = a;
        KernelKey k{};
        float *o1 = nullptr, *o2 = nullptr;
        auto plan_pass = [&]() {
            a = a0;
            // (a plan of passes without halos runs its other passes single-level)
            const int T = (!rsep && nsteps - s >= c.plan.key.T && !c.plan.wave) ? c.plan.key.T : 1;
            const int kmode = isep ? (int)kPlain : so.mode;
            k = (T == c.plan.key.T && kmode == kPlain) ? c.plan.key : key_for(c.plan.key, T, kmode, iso);
            if (k.T != T) k = key_for(c.plan.key, 1, kmode, iso);
            // a shape that cannot stage point entries (a tuned choice, made
            // without points, can be one) would walk a pass's tables of more
            // than a few entries in memory, serially: take a stageable shape
            // of the same depth and mode for such passes
            if (!points_stageable(k.M, k.T, k.PY, k.NW) &&
                ((!isep && a0.inj.cnt > kStageMin) || (!rsep && a0.rec.cnt > kStageMin))) {
                const KernelKey sk = stageable_key(k, iso);
                if (sk.M) k = sk;
            }
            a.u0 = st.cur;
            a.um = st.prev;
            o2 = nullptr;
            if (k.T == 1) {
                // in place: each point's u^{n-1} is read only by its owner (but a
                // second difference saved after the pass needs u^{n-1} intact)
                o1 = (isep && so.mode == kSaveD2) ? st.spare[0] : st.prev;
            } else {
                o1 = st.spare[0];
                o2 = st.spare[1];
            }
            a.o1 = o1;
            a.o2 = o2;
            a.lx = (k.T == c.plan.key.T && k.PY == c.plan.key.PY && k.NW == c.plan.key.NW)
                       ? c.plan.lx
                       : default_lx(d, k);
            const int ty = stream_core_rows(k), tz = stream_core_cols(k);
            a.ntz = (d.nz + tz - 1) / tz;
            a.nty = (d.ny + ty - 1) / ty;
            a.ntx = (d.nx + a.lx - 1) / a.lx;
            a.remap = c.plan.remap ? 1 : 0;
            a.alt = c.plan.alt ? 1 : 0;
            a.ntl = stream_loads(c.plan.loads, resident_bytes(a, k.mode), k.T) ? 1 : 0;
        };
        plan_pass();
        // a table of more than a few entries that this pass's chunks cannot
        // stage would be walked in memory one entry at a time: route it too
        const bool ri = !isep && imode && a.inj.cnt > kStageMin &&
                        (!fits_chunks(c, k, a, a.inj) ||
                         (so.mode == kPlain && k.T == 1 && a.inj.cnt > kRouteInjPlain));
        const bool rr = !rsep && a.rec.cnt > kStageMin && !fits_chunks(c, k, a, a.rec);
        if (ri || rr) {
            isep = isep || ri;
            rsep = rsep || rr || isep;
            plan_pass();
        }
        const int Tk = k.T;
        const SweepArgs ar = a;
        if (rsep) a.rec = PointTable{};
        if (isep) a.inj = PointTable{};
        a.ps = stage_points(c, k, a) ? 1 : 0;
        supertile(k, a);
        // split trapezoids along x: plain two-level passes that span more than
        // one chunk, with at most a few receivers (their entries are walked in
        // memory: the staged walk records each entry for every level of its
        // own chunk, which a split chunk does not compute; larger tables keep
        // the overlapped chunks)
        const bool split = c.plan.split && k.T == 2 && k.mode == kPlain && a.rec.cnt <= kStageMin && a.ntx >= 2;
        a.split = split ? 1 : 0;
        if (split && a.rec.cnt > 0) a.ps = 0;
        c.ex.pass(k, a, c.plan.loads);
        c.ran_split = c.ran_split || split;
        if (split) {
            // the inverted trapezoids: level 2 on the 2M planes around each
            // shared chunk end, from the level-1 field the first phase stored
            // in full (o2) and u^n (the pass's u0)
            const KernelKey k1 = key_for(k, 1, kPlain, iso);
            SweepArgs b = a;
            b.split = 0;
            b.u0 = o2;
            b.um = a.u0;
            b.o1 = o1;
            b.o2 = nullptr;
            b.step0 = a.step0 + 1;
            b.lx = 2 * d.M;
            b.xoff = a.lx - d.M;
            b.xstride = a.lx;
            b.ntx = a.ntx - 1;
            const int ty = stream_core_rows(k1), tz = stream_core_cols(k1);
            b.ntz = (d.nz + tz - 1) / tz;
            b.nty = (d.ny + ty - 1) / ty;
            b.remap = 0;
            b.alt = 0;
            b.gx = b.gy = 1;
            b.ps = 0;  // a few planes per chunk: the entries are walked in memory
            b.ntl = stream_loads(c.plan.loads, resident_bytes(b, kPlain), 1) ? 1 : 0;
            c.ex.pass(k1, b, c.plan.loads);
        }
        if (rsep) {
            const int mode = so.mode;
            const float *cur = st.cur, *prev = st.prev;
            float *d2 = a.d2 ? a.d2 + a.dslot0 * d.Np : nullptr;
            c.ex.call([ar, o1, cur, prev, d2, mode, isep](hipStream_t s) {
                hipError_t e = isep ? launch_inject(ar, o1, ar.step0, s) : hipSuccess;
                if (e == hipSuccess) e = launch_record(ar, o1, ar.step0, s);
                if (e == hipSuccess && isep && mode == kSaveD2) e = launch_save_d2(ar, o1, cur, prev, d2, s);
                if (e == hipSuccess && isep && mode == kImaging) e = launch_imaging(ar, o1, d2, ar.g, s);
                return e;
            });
        }
        if (Tk == 1) swap_in(st, o1, st.cur);
        else swap_in(st, o1, o2);
        c.ran_T = std::max(c.ran_T, Tk);
        s += Tk;
    }
}

// One step of fused Born modelling: background (sb, sources injected) and
// perturbation (sp, receivers recorded) advance in one pass of kernel `k`
// (mode kBornFused), each updated in place over its previous level.
void born_fused_step(Ctx &c, State &sb, State &sp, int64_t step, const KernelKey &k)
{
    const Dims &d = c.d;
    SweepArgs a = c.base;
    a.step0 = (int)step;
    a.u0 = sb.cur;
    a.um = sb.prev;
    a.o1 = sb.prev;
    a.u0b = sp.cur;
    a.umb = sp.prev;
    a.o2 = sp.prev;
    a.lx = (c.plan.key.T == 1 && k.PY == c.plan.key.PY && k.NW == c.plan.key.NW) ? c.plan.lx
                                                                                 : default_lx(d, k);
    const int ty = stream_core_rows(k), tz = stream_core_cols(k);
    a.ntz = (d.nz + tz - 1) / tz;
    a.nty = (d.ny + ty - 1) / ty;
    a.ntx = (d.nx + a.lx - 1) / a.lx;
    a.remap = c.plan.remap ? 1 : 0;
    a.alt = c.plan.alt ? 1 : 0;
    // two fields and their coefficient: u, u_prev, du, du_prev, q, s
    a.ntl = stream_loads(c.plan.loads, 2.0 * resident_bytes(a, kPlain), 1) ? 1 : 0;
    a.ps = stage_points(c, k, a) ? 1 : 0;
    supertile(k, a);
    c.ex.pass(k, a, c.plan.loads);
    c.ran_T = std::max(c.ran_T, 1);
    std::swap(sb.cur, sb.prev);
    std::swap(sp.cur, sp.prev);
}

// Move the final pair (st.cur, st.prev) into the caller's (A, B); tmp is a
// field distinct from A, B, st.cur and st.prev.
void place_state(const State &st, float *A, float *B, float *tmp, int64_t N, hipStream_t s)
{
    const size_t bytes = (size_t)N * 4;
    if (st.cur == A && st.prev == B) return;
    if (st.cur == B && st.prev == A) {
        FDW_HIP(hipMemcpyAsync(tmp, A, bytes, hipMemcpyDeviceToDevice, s));
        FDW_HIP(hipMemcpyAsync(A, B, bytes, hipMemcpyDeviceToDevice, s));
        FDW_HIP(hipMemcpyAsync(B, tmp, bytes, hipMemcpyDeviceToDevice, s));
    } else if (st.prev == A) {
        FDW_HIP(hipMemcpyAsync(B, A, bytes, hipMemcpyDeviceToDevice, s));
        FDW_HIP(hipMemcpyAsync(A, st.cur, bytes, hipMemcpyDeviceToDevice, s));
    } else {
        if (st.cur != A) FDW_HIP(hipMemcpyAsync(A, st.cur, bytes, hipMemcpyDeviceToDevice, s));
        if (st.prev != B) FDW_HIP(hipMemcpyAsync(B, st.prev, bytes, hipMemcpyDeviceToDevice, s));
    }
}

// The configuration of the last call: its plan, with the time-block depth the
// passes actually used (a route for large point tables or a short tail of
// steps can run fewer levels than planned).
void record_last(const Ctx &c)
{
    const Plan &p = c.plan;
    g_last = fd_options{};
    g_last.variant = p.variant;
    g_last.tile[0] = p.lx;
    g_last.tile[1] = p.key.NW * p.key.PY;
    g_last.tile[2] = p.key.PY;
    g_last.tblock = c.ran_T > 0 ? c.ran_T : p.key.T;
    if ((p.variant == FD_VARIANT_TBLOCK || p.variant == FD_VARIANT_SPLIT || p.variant == FD_VARIANT_WAVE) &&
        c.ran_T == 1)
        g_last.variant = FD_VARIANT_STREAM;
    else if (p.variant == FD_VARIANT_WAVE && c.wave_epoch == 0)
        g_last.variant = FD_VARIANT_TBLOCK;
    else if (p.variant == FD_VARIANT_SPLIT && !c.ran_split)
        g_last.variant = FD_VARIANT_TBLOCK;
    g_last_valid = true;
}

// After a call that ran passes without redundant halos: wait for them and
// report a wait that ran out (the outputs are then undefined).
int wave_status(const Ctx &c)
{
    if (c.wave_epoch == 0) return FD_OK;
    int e = 0;
    FDW_HIP(hipMemcpyAsync(&e, c.L.err, sizeof e, hipMemcpyDeviceToHost, c.s));
    FDW_HIP(hipStreamSynchronize(c.s));
    return e ? FD_ESYNC : FD_OK;
}

template <class F>
int guarded(F &&f)
{
    try {
        return f();
    } catch (const HipFail &) {
        return FD_EHIP;
    } catch (const Status &st) {
        return st.code;
    } catch (const std::bad_alloc &) {
        return FD_ENOMEM;
    } catch (...) {
        return FD_EHIP;
    }
}

int check_finite_traces(const float *dev, int64_t n, hipStream_t s)
{
    if (n <= 0) return FD_OK;
    std::vector<float> h(n);
    FDW_HIP(hipMemcpyAsync(h.data(), dev, n * 4, hipMemcpyDeviceToHost, s));
    FDW_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(h[i])) return FD_ENONFINITE;
    return FD_OK;
}

int ws_check(void *ws, size_t ws_bytes, size_t need)
{
    if (!ws || ws_bytes < need) return FD_EWORKSPACE;
    if (((uintptr_t)ws) & 255) return FD_EWORKSPACE;
    return FD_OK;
}

// Points between nodes record one value per (point, node) entry during the
// sweep; this turns the nt recorded rows into traces: out[row][p] = rscale *
// sum_c w_c e[row][c] over the point's nodes in corner order.
void gather_traces(Ctx &c, const TableBufs &b, int npts, int cnt, float *out, float rscale)
{
    if (!b.interp || npts <= 0 || c.nt <= 0 || !out) return;
    const float *etr = b.etr, *wt = b.wt;
    const int32_t *pptr = b.pptr, *pent = b.pent;
    const int64_t rows = c.nt;
    c.ex.call([=](hipStream_t s) {
        return launch_gather(etr, rows, cnt, pptr, pent, wt, npts, out, rscale, s);
    });
}

}  // namespace

// fd_forward in two phases: setup (eager) and issue (through c.ex).
struct FwdJob {
    Ctx c;
    float *u_state = nullptr;
    int nr = 0;
    uint32_t flags = 0;
};

int fwd_setup(FwdJob &j, const fd_grid *grid, const fd_time *time, const float *v,
              const fd_points *src, const fd_points *rec, float *rec_out, float *u_state,
              void *workspace, size_t ws_bytes, const fd_options *opts, void *stream)
{
    Ctx &c = j.c;
    int rc = validate_common(grid, time, v, c.d);
    if (rc) return rc;
    if ((rc = check_points(c.d, src, true, time->nt))) return rc;
    if ((rc = check_points(c.d, rec, false, time->nt))) return rc;
    j.nr = rec ? rec->n : 0;
    if (j.nr > 0 && time->nt > 0 && !rec_out) return FD_EINVAL;
    c.nt = time->nt;
    c.dt = time->dt;
    c.s = (hipStream_t)stream;
    c.ex.s = c.s;
    if ((rc = make_plan(c.d, opts, c.plan))) return rc;
    const PtsSpec S = spec_of(c.d, src), R = spec_of(c.d, rec);
    c.L = layout(nullptr, c.d, c.nt, S, R, FD_OP_FORWARD, fields_needed(FD_OP_FORWARD), 1);
    if ((rc = ws_check(workspace, ws_bytes, c.L.bytes))) return rc;
    c.L = layout(workspace, c.d, c.nt, S, R, FD_OP_FORWARD, fields_needed(FD_OP_FORWARD), 1);
    j.flags = opts ? opts->flags : 0u;
    if ((rc = prepare(c, grid, v, src, 1.0f, rec, j.flags))) return rc;
    c.base.amp = src ? src->amp : nullptr;
    c.base.rec_out = rec_out;
    j.u_state = u_state;
    return FD_OK;
}

void fwd_issue(FwdJob &j)
{
    Ctx &c = j.c;
    const int64_t N = c.d.Np;
    // the caller's state pair is used in place when its layout is the
    // internal one (nz a multiple of 32); otherwise it is converted in and out
    const bool direct = j.u_state && c.d.nzp == c.d.nz;
    float *A, *B;
    if (direct) {
        A = j.u_state;
        B = j.u_state + N;
    } else {
        A = c.L.fields[2];
        B = c.L.fields[3];
        if (j.u_state) {
            const float *U = j.u_state;
            const int64_t rows = (int64_t)c.d.nx * c.d.ny, Nd = c.d.N;
            const int nz = c.d.nz, nzp = c.d.nzp;
            c.ex.call([A, B, U, rows, nz, nzp, Nd](hipStream_t s) {
                hipError_t e = launch_repitch(A, nzp, U, nz, rows, nz, s);
                return e == hipSuccess ? launch_repitch(B, nzp, U + Nd, nz, rows, nz, s) : e;
            });
        } else {
            c.ex.call([A, B, N](hipStream_t s) {
                hipError_t e = launch_zero(A, N * 4, s);
                return e == hipSuccess ? launch_zero(B, N * 4, s) : e;
            });
        }
    }
    State st;
    st.cur = A;
    st.prev = B;
    st.spare[0] = c.L.fields[0];
    st.spare[1] = c.L.fields[1];
    st.spare[2] = nullptr;
    st.nspare = 2;
    advance(c, st, 0, c.nt, StepOpts{});
    gather_traces(c, c.L.rec, j.nr, c.base.rec.cnt, c.base.rec_out, 1.0f);
    if (j.u_state && !direct) {
        float *U = j.u_state;
        const float *cur = st.cur, *prev = st.prev;
        const int64_t rows = (int64_t)c.d.nx * c.d.ny, Nd = c.d.N;
        const int nz = c.d.nz, nzp = c.d.nzp;
        c.ex.call([U, cur, prev, rows, nz, nzp, Nd](hipStream_t s) {
            hipError_t e = launch_repitch(U, nz, cur, nzp, rows, nz, s);
            return e == hipSuccess ? launch_repitch(U + Nd, nz, prev, nzp, rows, nz, s) : e;
        });
    } else if (j.u_state) {
        const State fin = st;
        float *tmp = (c.L.fields[0] == st.cur || c.L.fields[0] == st.prev) ? c.L.fields[1]
                                                                            : c.L.fields[0];
        c.ex.call([fin, A, B, tmp, N](hipStream_t s) {
            try {
                place_state(fin, A, B, tmp, N, s);
            } catch (const HipFail &f) {
                return f.e;
            }
            return hipSuccess;
        });
    }
}

int forward_impl(const fd_grid *grid, const fd_time *time, const float *v, const fd_points *src,
                 const fd_points *rec, float *rec_out, float *u_state, void *workspace,
                 size_t ws_bytes, const fd_options *opts, void *stream)
{
    FwdJob j;
    int rc = fwd_setup(j, grid, time, v, src, rec, rec_out, u_state, workspace, ws_bytes, opts, stream);
    if (rc) return rc;
    fwd_issue(j);
    record_last(j.c);
    if ((rc = wave_status(j.c))) return rc;
    if (j.flags & FD_FLAG_CHECK_FINITE) return check_finite_traces(rec_out, j.c.nt * j.nr, j.c.s);
    return FD_OK;
}

// Scratch of fd_forward_noalloc: a forward call's workspace in a static device
// array.  Each device holds its own copy; host code reaches it only through
// the device address hipGetSymbolAddress returns (the array's name is a host
// stand-in, not a device address), looked up once per device.
constexpr size_t kScratchBytes = FD_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void *scratch_ptr()
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *ptrs[kMaxDevices] = {};
    int dev = 0;
    FDW_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Status{FD_EINVAL};
    std::lock_guard<std::mutex> lk(mu);
    if (!ptrs[dev]) {
        void *p = nullptr;
        FDW_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p & 255)) throw HipFail{hipErrorInvalidSymbol};
        ptrs[dev] = p;
    }
    return ptrs[dev];
}

}  // namespace fdw

using namespace fdw;

// ====================================================================== C ABI
extern "C" {

const char *fd_strerror(int code)
{
    switch (code) {
    case FD_OK: return "success";
    case FD_EINVAL: return "invalid argument";
    case FD_ECFL: return "time step exceeds the leapfrog stability limit";
    case FD_EDOM: return "source or receiver index outside the grid";
    case FD_EWORKSPACE: return "workspace missing, misaligned or too small";
    case FD_ENOMEM: return "host allocation failed";
    case FD_EHIP: return "HIP runtime error";
    case FD_ENONFINITE: return "non-finite or non-positive values";
    case FD_EUNSUPPORTED: return "no compiled kernel for the requested options";
    case FD_ESCRATCH: return "the call needs more scratch than the library's static array holds";
    default: return "unknown status";
    }
}

int fd_version(void) { return 100; }

int fd_last_config(fd_options *out)
{
    if (!out || !g_last_valid) return FD_EINVAL;
    *out = g_last;
    return FD_OK;
}

size_t fd_workspace_size(const fd_grid *grid, const fd_time *time, const fd_points *src,
                         const fd_points *rec, const fd_options *opts, int op)
{
    Dims d;
    if (make_dims(grid, d) || !time || time->nt < 0) return 0;
    if (op < FD_OP_FORWARD || op > FD_OP_BORN) return 0;
    // the tables of both point sets are laid out alike, so the order (which
    // set injects) does not change the size
    Layout L = layout(nullptr, d, time->nt, spec_of(d, src), spec_of(d, rec), op, fields_needed(op),
                      ckpt_interval(opts));
    return L.bytes;
}

int fd_gradient_storage(const fd_grid *grid, const fd_time *time, const fd_points *src,
                        const fd_points *rec, int op, size_t budget, fd_options *inout,
                        size_t *ws_bytes)
{
    return guarded([&]() -> int {
        Dims d;
        if (!inout || make_dims(grid, d) || !time || time->nt < 1 || time->nt > INT32_MAX)
            return FD_EINVAL;
        if (op != FD_OP_GRADIENT && op != FD_OP_VJP) return FD_EINVAL;
        if ((src && src->n < 0) || (rec && rec->n < 0)) return FD_EINVAL;
        const int64_t nt = time->nt;
        const PtsSpec S = spec_of(d, src), R = spec_of(d, rec);
        auto bytes_at = [&](int64_t K) {
            return layout(nullptr, d, nt, S, R, op, fields_needed(op), (int)K).bytes;
        };
        // The saved time dimension: one checkpoint, every second difference kept,
        // no recomputation (two sweeps per step instead of three).
        int64_t best = nt;
        size_t need = bytes_at(nt);
        if (need > budget) {
            // Every interval below nt recomputes the same nt steps, so the one
            // with the smallest footprint (about sqrt(2 nt)) costs nothing extra.
            for (int64_t K = 1; K < nt; ++K) {
                const size_t b = bytes_at(K);
                if (b < need) {
                    need = b;
                    best = K;
                }
            }
        }
        inout->ckpt_every = (int32_t)best;
        if (ws_bytes) *ws_bytes = need;
        return need <= budget ? FD_OK : FD_EWORKSPACE;
    });
}

int fd_forward(const fd_grid *grid, const fd_time *time, const float *v, const fd_points *src,
               const fd_points *rec, float *rec_out, float *u_state, void *workspace,
               size_t ws_bytes, const fd_options *opts, void *stream)
{
    return guarded([&]() -> int {
        return forward_impl(grid, time, v, src, rec, rec_out, u_state, workspace, ws_bytes, opts, stream);
    });
}

int fd_forward_noalloc(const fd_grid *grid, const fd_time *time, const float *v,
                       const fd_points *src, const fd_points *rec, float *rec_out,
                       float *u_state, const fd_options *opts, void *stream)
{
    return guarded([&]() -> int {
        const size_t need = fd_workspace_size(grid, time, src, rec, opts, FD_OP_FORWARD);
        if (!need) return FD_EINVAL;
        if (need > kScratchBytes) return FD_ESCRATCH;
        return forward_impl(grid, time, v, src, rec, rec_out, u_state, scratch_ptr(), kScratchBytes, opts,
                            stream);
    });
}

int fd_adjoint(const fd_grid *grid, const fd_time *time, const float *v, const fd_points *src,
               const fd_points *rec, float *src_out, float *lam_state, void *workspace,
               size_t ws_bytes, const fd_options *opts, void *stream)
{
    return guarded([&]() -> int {
        Ctx c;
        int rc = validate_common(grid, time, v, c.d);
        if (rc) return rc;
        if ((rc = check_points(c.d, src, false, time->nt))) return rc;
        if ((rc = check_points(c.d, rec, true, time->nt))) return rc;
        const int ns = src ? src->n : 0, nr = rec ? rec->n : 0;
        if (ns > 0 && time->nt > 0 && !src_out) return FD_EINVAL;
        c.nt = time->nt;
        c.dt = time->dt;
        c.s = (hipStream_t)stream;
        c.ex.s = c.s;
        if ((rc = make_plan(c.d, opts, c.plan))) return rc;
        const PtsSpec S = spec_of(c.d, src), R = spec_of(c.d, rec);
        c.L = layout(nullptr, c.d, c.nt, R, S, FD_OP_ADJOINT, fields_needed(FD_OP_ADJOINT), 1);
        if ((rc = ws_check(workspace, ws_bytes, c.L.bytes))) return rc;
        c.L = layout(workspace, c.d, c.nt, R, S, FD_OP_ADJOINT, fields_needed(FD_OP_ADJOINT), 1);
        const uint32_t flags = opts ? opts->flags : 0u;
        // receivers inject (scale 1 / (2m + dt damp) = q / (2 dt^2 (1 + eta))), sources record
        const float alpha = (float)(1.0 / (2.0 * c.dt * c.dt));
        if ((rc = prepare(c, grid, v, rec, alpha, src, flags))) return rc;
        c.base.amp = rec ? rec->amp : nullptr;
        c.base.abase = c.nt - 1;
        c.base.adir = -1;
        c.base.rec_out = src_out;
        c.base.rbase = c.nt - 1;
        c.base.rdir = -1;
        c.base.rscale = (float)(2.0 * c.dt * c.dt);
        State st;
        st.cur = c.L.fields[2];
        st.prev = c.L.fields[3];
        FDW_HIP(launch_zero(st.cur, c.d.Np * 4, c.s));
        FDW_HIP(launch_zero(st.prev, c.d.Np * 4, c.s));
        st.spare[0] = c.L.fields[0];
        st.spare[1] = c.L.fields[1];
        st.spare[2] = nullptr;
        st.nspare = 2;
        advance(c, st, 0, c.nt, StepOpts{});
        gather_traces(c, c.L.rec, ns, c.base.rec.cnt, src_out, c.base.rscale);
        if (lam_state) {
            const int64_t rows = (int64_t)c.d.nx * c.d.ny;
            FDW_HIP(launch_repitch(lam_state, c.d.nz, st.cur, c.d.nzp, rows, c.d.nz, c.s));
            FDW_HIP(launch_repitch(lam_state + c.d.N, c.d.nz, st.prev, c.d.nzp, rows, c.d.nz, c.s));
        }
        record_last(c);
        if ((rc = wave_status(c))) return rc;
        if (flags & FD_FLAG_CHECK_FINITE) return check_finite_traces(src_out, c.nt * ns, c.s);
        return FD_OK;
    });
}

int fd_born(const fd_grid *grid, const fd_time *time, const float *v, const float *dv,
            const fd_points *src, const fd_points *rec, float *rec_out, void *workspace,
            size_t ws_bytes, const fd_options *opts, void *stream)
{
    return guarded([&]() -> int {
        Ctx c;
        int rc = validate_common(grid, time, v, c.d);
        if (rc) return rc;
        if (!dv) return FD_EINVAL;
        if ((rc = check_points(c.d, src, true, time->nt))) return rc;
        if ((rc = check_points(c.d, rec, false, time->nt))) return rc;
        const int ns = src ? src->n : 0, nr = rec ? rec->n : 0;
        if (nr > 0 && time->nt > 0 && !rec_out) return FD_EINVAL;
        c.nt = time->nt;
        c.dt = time->dt;
        c.s = (hipStream_t)stream;
        c.ex.s = c.s;
        if ((rc = make_plan(c.d, opts, c.plan))) return rc;
        const PtsSpec S = spec_of(c.d, src), R = spec_of(c.d, rec);
        c.L = layout(nullptr, c.d, c.nt, S, R, FD_OP_BORN, fields_needed(FD_OP_BORN), 1);
        if ((rc = ws_check(workspace, ws_bytes, c.L.bytes))) return rc;
        c.L = layout(workspace, c.d, c.nt, S, R, FD_OP_BORN, fields_needed(FD_OP_BORN), 1);
        const uint32_t flags = opts ? opts->flags : 0u;
        if ((rc = prepare(c, grid, v, src, 1.0f, rec, flags))) return rc;
        const int64_t N = c.d.Np, rows = (int64_t)c.d.nx * c.d.ny;
        float *bs = c.L.fields[8];
        FDW_HIP(launch_born_coef(v, dv, bs, rows, c.d.nz, c.d.nzp, c.s));
        for (int i = 0; i < 8; ++i) FDW_HIP(launch_zero(c.L.fields[i], N * 4, c.s));
        // background: sources inject, no recording, the second difference of
        // each new level goes to slot 0; perturbation: the Born source, no
        // injection, receivers record
        SweepArgs bg = c.base;
        bg.amp = src ? src->amp : nullptr;
        bg.rec = as_table(c.L.rec, nr, 0, false);
        SweepArgs pb = c.base;
        pb.inj = as_table(c.L.src, ns, 0, true);
        pb.rec_out = rec_out;
        pb.bs = bs;
        State sb{c.L.fields[0], c.L.fields[1], {c.L.fields[2], c.L.fields[3], nullptr}, 2};
        State sp{c.L.fields[4], c.L.fields[5], {c.L.fields[6], c.L.fields[7], nullptr}, 2};
        // one pass per step when a fused kernel for this order is compiled
        // (32 B per point instead of 44), else two passes per step
        // (2 rows x 8 waves where compiled: with two fields per thread it ran
        // 5 % faster than the 4 x 8 tile of the single-field sweep)
        KernelKey fk{c.plan.key.M, 1, 2, 8, kBornFused};
        if (!stream_has(fk, c.base.w.iso != 0)) fk = key_for(c.plan.key, 1, kBornFused, c.base.w.iso != 0);
        const bool fused = c.plan.variant != FD_VARIANT_NAIVE && fk.mode == kBornFused &&
                           stream_has(fk, c.base.w.iso != 0) && !heavy_table(c, bg.inj) &&
                           !heavy_table(c, pb.rec);
        if (fused) {
            SweepArgs fa = c.base;
            fa.amp = src ? src->amp : nullptr;
            fa.rec_out = rec_out;
            fa.bs = bs;
            c.base = fa;
            for (int64_t k = 0; k < c.nt; ++k) born_fused_step(c, sb, sp, k, fk);
        } else {
            StepOpts fo, bo;
            fo.mode = kSaveD2;
            bo.mode = kBorn;
            fo.dslot_first = bo.dslot_first = 0;
            fo.ddir = bo.ddir = 0;
            for (int64_t k = 0; k < c.nt; ++k) {
                c.base = bg;
                advance(c, sb, k, 1, fo);
                c.base = pb;
                advance(c, sp, k, 1, bo);
            }
        }
        gather_traces(c, c.L.rec, nr, pb.rec.cnt, rec_out, 1.0f);
        record_last(c);
        if ((rc = wave_status(c))) return rc;
        if (flags & FD_FLAG_CHECK_FINITE) return check_finite_traces(rec_out, c.nt * nr, c.s);
        return FD_OK;
    });
}

}  // extern "C"

namespace fdw {
namespace {

// fd_gradient / fd_vjp in three phases: setup (validation, tables, stability
// check: eager, may synchronise), issue (all device work of the checkpointed
// adjoint-state gradient, through c.ex: executed or recorded) and misfit (reads
// the residual partial sums back).
struct GradJob {
    Ctx c;
    const float *v = nullptr;
    const float *y = nullptr;      // trace cotangent (vjp) or nullptr (least squares)
    const float *dobs = nullptr;   // observed data (least squares)
    float *grad_v = nullptr;
    float *residual = nullptr;     // caller's residual buffer or nullptr
    int K = 50, ns = 0, nr = 0;
};

int grad_setup(GradJob &j, const fd_grid *grid, const fd_time *time, const float *v,
               const fd_points *src, const fd_points *rec, const float *y, float *grad_v,
               float *residual, void *workspace, size_t ws_bytes, const fd_options *opts,
               void *stream, int op)
{
    Ctx &c = j.c;
    int rc = validate_common(grid, time, v, c.d);
    if (rc) return rc;
    if ((rc = check_points(c.d, src, true, time->nt))) return rc;
    if ((rc = check_points(c.d, rec, true, time->nt))) return rc;
    if (!grad_v) return FD_EINVAL;
    j.ns = src ? src->n : 0;
    j.nr = rec ? rec->n : 0;
    c.nt = time->nt;
    c.dt = time->dt;
    c.s = (hipStream_t)stream;
    c.ex.s = c.s;
    if ((rc = make_plan(c.d, opts, c.plan))) return rc;
    j.K = ckpt_interval(opts);
    if (j.K < 1) return FD_EINVAL;
    const PtsSpec S = spec_of(c.d, src), R = spec_of(c.d, rec);
    c.L = layout(nullptr, c.d, c.nt, S, R, op, fields_needed(op), j.K);
    if ((rc = ws_check(workspace, ws_bytes, c.L.bytes))) return rc;
    c.L = layout(workspace, c.d, c.nt, S, R, op, fields_needed(op), j.K);
    const uint32_t flags = opts ? opts->flags : 0u;
    if ((rc = prepare(c, grid, v, src, 1.0f, rec, flags))) return rc;
    // adjoint injection scale at the receivers: 1 / (2m + dt damp) = q / (2 dt^2 (1 + eta))
    const float alpha = (float)(1.0 / (2.0 * c.dt * c.dt));
    FDW_HIP(launch_scales(c.base, as_table(c.L.rec, j.nr, c.base.rec.cnt, true), c.L.rec.scale, alpha,
                          c.s));
    c.base.amp = src ? src->amp : nullptr;
    j.v = v;
    j.y = y;
    j.dobs = rec ? rec->amp : nullptr;
    j.grad_v = grad_v;
    j.residual = residual;
    return FD_OK;
}

void grad_issue(GradJob &j)
{
    Ctx &c = j.c;
    const int64_t N = c.d.Np;  // floats of one internal (padded) field
    const int K = j.K, ns = j.ns, nr = j.nr;
    // ---- forward sweep with checkpoints (sources inject, receivers record)
    c.base.rec_out = c.L.traces;
    float *F[5] = {c.L.fields[0], c.L.fields[1], c.L.fields[2], c.L.fields[3], c.L.fields[4]};
    State st{F[0], F[1], {F[2], F[3], F[4]}, 3};
    {
        float *a0 = st.cur, *a1 = st.prev;
        c.ex.call([a0, a1, N](hipStream_t s) {
            hipError_t e = launch_zero(a0, N * 4, s);
            return e == hipSuccess ? launch_zero(a1, N * 4, s) : e;
        });
    }
    // One segment (checkpoint interval >= nt: the whole time axis is stored,
    // the paper's "saved" time dimension): the forward sweep itself writes
    // every second difference, and the adjoint needs no recomputation
    // (two sweeps instead of three).
    const bool full = c.L.nck == 1;
    if (full) {
        StepOpts fo;
        fo.mode = kSaveD2;
        fo.dslot_first = 0;  // step n produces u^{n+1}: slot n
        fo.ddir = 1;
        advance(c, st, 0, c.nt, fo);
    } else {
        for (int jck = 0; jck < c.L.nck; ++jck) {
            const int64_t k0 = (int64_t)jck * K, k1 = std::min<int64_t>(k0 + K, c.nt);
            float *ck = c.L.ckpt + (size_t)jck * 2 * N;
            float *cur = st.cur, *prev = st.prev;
            c.ex.call([ck, cur, prev, N](hipStream_t s) {
                hipError_t e = copy_async(ck, cur, N, s);
                return e == hipSuccess ? copy_async(ck + N, prev, N, s) : e;
            });
            advance(c, st, k0, k1 - k0, StepOpts{});
        }
    }
    gather_traces(c, c.L.rec, nr, c.base.rec.cnt, c.L.traces, 1.0f);
    // ---- residual (least squares) or the given cotangent
    const float *adj_src = j.y;
    if (!j.y) {
        float *res = j.residual ? j.residual : c.L.resid;
        const float *d = c.L.traces, *dobs = j.dobs;
        double *part = c.L.rpart;
        const int64_t n = c.nt * nr;
        c.ex.call([d, dobs, res, n, part](hipStream_t s) {
            return launch_residual(d, dobs, res, n, part, kStatBlocks, s);
        });
        adj_src = res;
    }
    // ---- adjoint sweep with segment recomputation and imaging
    SweepArgs fwd = c.base;
    fwd.rec = as_table(c.L.rec, nr, 0, false);  // no recording during recomputation
    SweepArgs adj = c.base;
    adj.inj = as_table(c.L.rec, nr, c.base.rec.cnt, true);
    adj.rec = as_table(c.L.src, ns, 0, false);
    adj.amp = adj_src;
    adj.abase = c.nt - 1;
    adj.adir = -1;
    adj.rec_out = nullptr;
    {
        double *g = c.L.g;
        float *gp = c.L.gp;
        c.ex.call([g, gp, N](hipStream_t s) {
            hipError_t e = launch_zero(g, N * 8, s);
            return e == hipSuccess ? launch_zero(gp, N * 4, s) : e;
        });
    }
    float *Aa[4] = {c.L.fields[5], c.L.fields[6], c.L.fields[7], c.L.fields[8]};
    State sa{Aa[0], Aa[1], {Aa[2], Aa[3], nullptr}, 2};
    {
        float *a0 = sa.cur, *a1 = sa.prev;
        c.ex.call([a0, a1, N](hipStream_t s) {
            hipError_t e = launch_zero(a0, N * 4, s);
            return e == hipSuccess ? launch_zero(a1, N * 4, s) : e;
        });
    }
    const SweepArgs saved = c.base;
    for (int jck = c.L.nck - 1; jck >= 0; --jck) {
        const int64_t k0 = (int64_t)jck * K, k1 = std::min<int64_t>(k0 + K, c.nt);
        if (!full) {
            const float *ck = c.L.ckpt + (size_t)jck * 2 * N;
            State sf{F[0], F[1], {F[2], F[3], F[4]}, 3};
            {
                float *cur = sf.cur, *prev = sf.prev;
                c.ex.call([ck, cur, prev, N](hipStream_t s) {
                    hipError_t e = copy_async(cur, ck, N, s);
                    return e == hipSuccess ? copy_async(prev, ck + N, N, s) : e;
                });
            }
            c.base = fwd;
            StepOpts fo;
            fo.mode = kSaveD2;
            fo.dslot_first = 0;  // step k0 produces u^{k0+1}: slot (k0+1) - k0 - 1 = 0
            fo.ddir = 1;
            advance(c, sf, k0, k1 - k0, fo);
        }
        c.base = adj;
        // adjoint step n produces lambda^{nt-n}, imaged with the second
        // difference in slot k1 - k0 - 1 - (n - (nt - k1)).  The FP32 partial
        // sums are added into the image after every step n with n + 1 a
        // multiple of kImageFlush, and after the last: the same blocks of
        // steps for every checkpoint interval, so every storage choice rounds
        // alike
        for (int64_t n = c.nt - k1; n < c.nt - k0;) {
            const int64_t end = std::min<int64_t>((n / kImageFlush + 1) * kImageFlush, c.nt - k0);
            StepOpts ao;
            ao.mode = kImaging;
            ao.dslot_first = k1 - k0 - 1 - (n - (c.nt - k1));
            ao.ddir = -1;
            advance(c, sa, n, end - n, ao);
            n = end;
            if (n % kImageFlush == 0 || n == c.nt) {
                double *g = c.L.g;
                float *gp = c.L.gp;
                c.ex.call([gp, g, N](hipStream_t s) { return launch_flush_image(gp, g, N, s); });
            }
        }
    }
    c.base = saved;
    {
        const double *g = c.L.g;
        const float *v = j.v;
        float *gv = j.grad_v;
        const int64_t rows = (int64_t)c.d.nx * c.d.ny;
        const int nz = c.d.nz, nzp = c.d.nzp;
        c.ex.call([g, v, gv, rows, nz, nzp](hipStream_t s) {
            return launch_grad_v(g, v, gv, rows, nz, nzp, s);
        });
    }
}

double grad_misfit(GradJob &j)
{
    std::vector<double> part(kStatBlocks);
    FDW_HIP(hipMemcpyAsync(part.data(), j.c.L.rpart, kStatBlocks * 8, hipMemcpyDeviceToHost, j.c.s));
    FDW_HIP(hipStreamSynchronize(j.c.s));
    double J = 0.0;
    for (double p : part) J += p;
    return J;
}

int gradient_impl(const fd_grid *grid, const fd_time *time, const float *v, const fd_points *src,
                  const fd_points *rec, const float *y, float *grad_v, double *misfit,
                  float *residual, void *workspace, size_t ws_bytes, const fd_options *opts,
                  void *stream, int op)
{
    GradJob j;
    int rc = grad_setup(j, grid, time, v, src, rec, y, grad_v, residual, workspace, ws_bytes, opts,
                        stream, op);
    if (rc) return rc;
    grad_issue(j);
    if (!y && misfit) *misfit = grad_misfit(j);
    record_last(j.c);
    return wave_status(j.c);
}

}  // namespace
}  // namespace fdw

extern "C" {

int fd_gradient(const fd_grid *grid, const fd_time *time, const float *v, const fd_points *src,
                const fd_points *rec, float *grad_v, double *misfit, float *residual,
                void *workspace, size_t ws_bytes, const fd_options *opts, void *stream)
{
    return guarded([&]() -> int {
        return gradient_impl(grid, time, v, src, rec, nullptr, grad_v, misfit, residual, workspace,
                             ws_bytes, opts, stream, FD_OP_GRADIENT);
    });
}

int fd_vjp(const fd_grid *grid, const fd_time *time, const float *v, const fd_points *src,
           const fd_points *rec, float *grad_v, void *workspace, size_t ws_bytes,
           const fd_options *opts, void *stream)
{
    return guarded([&]() -> int {
        if (rec && rec->n > 0 && time && time->nt > 0 && !rec->amp) return FD_EINVAL;
        return gradient_impl(grid, time, v, src, rec, rec ? rec->amp : nullptr, grad_v, nullptr,
                             nullptr, workspace, ws_bytes, opts, stream, FD_OP_VJP);
    });
}

}  // extern "C"

// ====================================================================== autotuner
namespace fdw {
namespace {

__global__ void k_fill(float *p, float val, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = val;
}

struct Candidate {
    fd_options o;
};

std::vector<Candidate> candidates(const Dims &d, const fd_options &fixed)
{
    std::vector<Candidate> out;
    auto push = [&](int variant, int lx, int rows, int py, int tb) {
        Candidate c;
        c.o = fixed;
        c.o.variant = variant;
        c.o.tile[0] = lx;
        c.o.tile[1] = rows;
        c.o.tile[2] = py;
        c.o.tblock = tb;
        out.push_back(c);
    };
    if (fixed.variant == 0 || fixed.variant == FD_VARIANT_NAIVE) push(FD_VARIANT_NAIVE, 0, 0, 0, 1);
    static const int shapes[][2] = {{4, 8}, {4, 4}, {2, 16}, {8, 4}, {16, 2}, {8, 2}};
    for (int T = 1; T <= 5; ++T) {
        // T = 5 stands for the split form of two-level passes
        const int variant = T == 1 ? FD_VARIANT_STREAM : T == 5 ? FD_VARIANT_SPLIT : FD_VARIANT_TBLOCK;
        const int depth = T == 5 ? 2 : T;
        if (fixed.variant && fixed.variant != variant) continue;
        if (fixed.tblock && fixed.tblock != depth) continue;
        for (auto &sh : shapes) {
            KernelKey k{d.M, depth, sh[0], sh[1], kPlain};
            if (!stream_has(k, grid_iso(d))) continue;
            const int lx0 = default_lx(d, k);
            int last = -1;
            for (int f : {1, 2, 4, 8}) {  // lx0 / 2, lx0, 2 lx0, 4 lx0
                const int lx = std::min(std::min(d.nx, kMaxLx), std::max(4 * depth * d.M, lx0 * f / 2));
                if (lx == last) continue;
                last = lx;
                push(variant, lx, sh[0] * sh[1], sh[0], depth);
            }
        }
    }
    // two levels without redundant halos, where all tiles fit the device at once
    if (!fixed.variant || fixed.variant == FD_VARIANT_WAVE) {
        static const int wshapes[][2] = {{2, 8}, {2, 4}, {4, 4}};
        for (auto &sh : wshapes)
            if (wave_has(d.M, sh[0], sh[1]) && (!fixed.tblock || fixed.tblock == 2))
                push(FD_VARIANT_WAVE, 0, sh[0] * sh[1], sh[0], 2);
    }
    return out;
}

void save_tune(const std::string &key, const fd_options &o)
{
    const char *path = std::getenv("FD_AUTOTUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d %d %d\n", key.c_str(), o.variant, o.tile[0], o.tile[1], o.tile[2],
                 o.tblock);
    std::fclose(f);
}

}  // namespace
}  // namespace fdw

extern "C" int fd_autotune(const fd_grid *grid, const fd_time *time, fd_options *inout,
                           void *workspace, size_t ws_bytes, void *stream)
{
    return guarded([&]() -> int {
        Dims d;
        int rc = make_dims(grid, d);
        if (rc) return rc;
        if (!inout || !time || !(time->dt > 0.0)) return FD_EINVAL;
        fd_time tt = *time;
        if (tt.nt < 1) tt.nt = 8;
        fd_options fixed = *inout;
        hipStream_t s = (hipStream_t)stream;
        Layout L0 = layout(nullptr, d, tt.nt, PtsSpec{}, PtsSpec{}, FD_OP_FORWARD,
                           fields_needed(FD_OP_FORWARD), 1);
        if ((rc = ws_check(workspace, ws_bytes, L0.bytes))) return rc;
        Ctx c;
        c.d = d;
        c.nt = tt.nt;
        c.dt = tt.dt;
        c.s = s;
        c.ex.s = s;
        c.L = layout(workspace, d, tt.nt, PtsSpec{}, PtsSpec{}, FD_OP_FORWARD,
                     fields_needed(FD_OP_FORWARD), 1);
        // a constant medium at 60 % of the stability limit: kernel time does not
        // depend on the values, only on the sponge branch, which is kept
        double inv_h2 = 0.0;
        for (int a = 0; a < 3; ++a)
            if (d.present[a]) inv_h2 += 1.0 / (d.h[a] * d.h[a]);
        const float qv = (float)(0.36 * 4.0 / (nyquist_symbol(d.M) * inv_h2));
        hipLaunchKernelGGL(k_fill, dim3(2048), dim3(256), 0, s, c.L.q, qv, d.Np);
        FDW_HIP(hipGetLastError());
        std::vector<float> prof((size_t)d.nx + d.ny + d.nz);
        sponge_profile(d.nx, grid->sponge, d.h[0], grid->sponge_vref, tt.dt, d.present[0], prof.data());
        sponge_profile(d.ny, grid->sponge, d.h[1], grid->sponge_vref, tt.dt, d.present[1],
                       prof.data() + d.nx);
        sponge_profile(d.nz, grid->sponge, d.h[2], grid->sponge_vref, tt.dt, d.present[2],
                       prof.data() + d.nx + d.ny);
        FDW_HIP(hipMemcpyAsync(c.L.prof, prof.data(), prof.size() * 4, hipMemcpyHostToDevice, s));
        std::vector<Entry> none;
        upload_table(d, none, c.L.src, 0, &c.hxs, s);
        upload_table(d, none, c.L.rec, 0, &c.hxr, s);
        upload_planes(d, prof.data(), c.hxs, c.hxr, c.L.ptab, s);
        SweepArgs &a = c.base;
        std::memset(&a, 0, sizeof a);
        a.nx = d.nx;
        a.ny = d.ny;
        a.nz = d.nz;
        a.nzp = d.nzp;
        a.sxy = (int64_t)d.ny * d.nzp;
        a.w = make_weights(d);
        a.q = c.L.q;
        a.px = c.L.prof;
        a.py = c.L.prof + d.nx;
        a.pz = c.L.prof + d.nx + d.ny;
        a.inj = as_table(c.L.src, 0, 0, true);
        a.rec = as_table(c.L.rec, 0, 0, false);
        a.rscale = 1.0f;
        a.adir = a.rdir = 1;
        a.ptab = c.L.ptab;
        struct Events {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            ~Events()
            {
                if (e0) (void)hipEventDestroy(e0);
                if (e1) (void)hipEventDestroy(e1);
            }
        } ev;
        FDW_HIP(hipEventCreate(&ev.e0));
        FDW_HIP(hipEventCreate(&ev.e1));
        const hipEvent_t e0 = ev.e0, e1 = ev.e1;
        float best = 1e30f;
        fd_options best_o = fixed;
        bool found = false;
        for (const Candidate &cand : candidates(d, fixed)) {
            Plan p;
            if (make_plan(d, &cand.o, p) != FD_OK) continue;
            c.plan = p;
            State st{c.L.fields[2], c.L.fields[3], {c.L.fields[0], c.L.fields[1], nullptr}, 2};
            FDW_HIP(launch_zero(st.cur, d.Np * 4, s));
            FDW_HIP(launch_zero(st.prev, d.Np * 4, s));
            const int64_t steps = std::max<int64_t>(tt.nt, p.key.T) / p.key.T * p.key.T;
            c.wave_epoch = 0;  // a candidate's first pass without halos clears the counters
            advance(c, st, 0, steps, StepOpts{});  // warm-up
            FDW_HIP(hipEventRecord(e0, s));
            advance(c, st, 0, steps, StepOpts{});
            FDW_HIP(hipEventRecord(e1, s));
            FDW_HIP(hipEventSynchronize(e1));
            if (wave_status(c) != FD_OK) continue;  // a wait ran out: not a valid timing
            float ms = 0.0f;
            FDW_HIP(hipEventElapsedTime(&ms, e0, e1));
            const float per_step = ms / (float)steps;
            if (per_step < best) {
                best = per_step;
                best_o = cand.o;
                best_o.variant = p.variant;
                best_o.tile[0] = p.lx;
                best_o.tile[1] = p.key.NW * p.key.PY;
                best_o.tile[2] = p.key.PY;
                best_o.tblock = p.key.T;
                found = true;
            }
        }
        if (!found) return FD_EUNSUPPORTED;
        *inout = best_o;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune[tune_key(d)] = best_o;
        }
        save_tune(tune_key(d), best_o);
        return FD_OK;
    });
}

// ====================================================================== batches
namespace fdw {
namespace {


// Upper bound of grouped-pass entries a shot contributes (one per step per sweep).
size_t entry_bound(const fd_shot &sh, int op)
{
    const int64_t nt = std::max<int64_t>(sh.time.nt, 0);
    return (size_t)((op == FD_OP_GRADIENT ? 3 : 1) * nt + 8);
}

// Chunk length of a batched shot: a grouped launch draws its parallelism from
// all the shots of its class, so an automatic chunk is lengthened to at least
// kBatchLx planes, which cuts the share of the 2 T M warm-up planes that every
// chunk re-reads (a lone shot needs short chunks for enough workgroups).
constexpr int kBatchLx = 64;
void batch_chunk(Ctx &c, const fd_options &o)
{
    if (o.tile[0] > 0 || c.plan.variant == FD_VARIANT_NAIVE) return;
    c.plan.lx = std::min(std::min(c.d.nx, kMaxLx), std::max(c.plan.lx, kBatchLx));
}

// Merge the recorded op lists of many shots and run them on one stream: ops
// are taken round by round (op r of every shot), passes of one round with the
// same kernel configuration and Laplacian form become one grouped
// launch over all their tiles, other ops run as recorded.  Shots are
// independent, so any interleaving that keeps each shot's order is valid.
// The lanes of a device: streams the library creates on first use and keeps
// for the life of the process (as the runtime keeps its default stream), so a
// batch never destroys a stream that may still hold its work, plus one private
// stream per device for graph capture (the caller's may be the legacy default
// stream, which cannot be captured).  A batch holds its device's pool for the
// whole of its issue, so that batches issued from several host threads do not
// interleave their fork and join events.
struct LanePool {
    std::mutex mu;
    std::vector<hipStream_t> streams;
    hipStream_t capture = nullptr;
};

LanePool &lane_pool()
{
    static std::mutex mu;
    static std::map<int, std::unique_ptr<LanePool>> pools;
    int dev = 0;
    FDW_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto &p = pools[dev];
    if (!p) p.reset(new LanePool());
    return *p;
}

void grow_lanes(LanePool &p, int n)
{
    while ((int)p.streams.size() < n) {
        hipStream_t t = nullptr;
        FDW_HIP(hipStreamCreateWithFlags(&t, hipStreamNonBlocking));
        p.streams.push_back(t);
    }
    if (!p.capture) FDW_HIP(hipStreamCreateWithFlags(&p.capture, hipStreamNonBlocking));
}

// Fork and join events of one batch, all created before any capture begins and
// destroyed once the work that records or waits on them has completed (the
// batch synchronises the caller's stream before it returns).
struct LaneEvents {
    std::vector<hipEvent_t> ev;
    explicit LaneEvents(int n)
    {
        ev.reserve(n);
        for (int i = 0; i < n; ++i) {
            hipEvent_t e = nullptr;
            FDW_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            ev.push_back(e);
        }
    }
    ~LaneEvents()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    LaneEvents(const LaneEvents &) = delete;
    LaneEvents &operator=(const LaneEvents &) = delete;
};

int run_merged(std::vector<std::vector<Op>> &ops, const std::vector<int> &shot_lane,
               GroupEntry *dev_entries, size_t max_entries, bool graph, hipStream_t s)
{
    struct Launch {
        bool grouped;
        KernelKey key;
        bool iso;
        bool ntl;
        bool ps;
        size_t off;
        int n, total;
        int shot, idx;
        int grid;
    };
    // Lanes: shot_lane[i] names the lane of shot i (its space order); a
    // grouped launch only holds shots of one lane, so each lane's work is a
    // chain independent of the others.  Each lane gets a stream of its own,
    // forked from and joined back to the issuing stream, so that the launches
    // of different lanes overlap (one lane's tail of workgroups leaves CUs
    // that another's launch can fill).
    std::map<int, int> lane_of;
    for (int m : shot_lane) lane_of.emplace(m, (int)lane_of.size());
    std::vector<int> launch_lane;
    std::vector<GroupEntry> host;
    std::vector<Launch> plan;
    size_t rounds = 0;
    for (auto &o : ops) rounds = std::max(rounds, o.size());
    for (size_t r = 0; r < rounds; ++r) {
        std::vector<std::pair<size_t, size_t>> passes;  // (shot, op) of this round
        for (size_t sh = 0; sh < ops.size(); ++sh) {
            if (r >= ops[sh].size()) continue;
            const Op &o = ops[sh][r];
            if (o.is_pass && stream_has_group(o.key, o.a.w.iso != 0)) passes.push_back({sh, r});
            else {
                plan.push_back(Launch{false, {}, false, false, false, 0, 0, 0, (int)sh, (int)r, 0});
                launch_lane.push_back(lane_of[shot_lane[sh]]);
            }
        }
        std::vector<bool> done(passes.size(), false);
        for (size_t p = 0; p < passes.size(); ++p) {
            if (done[p]) continue;
            const Op &lead = ops[passes[p].first][passes[p].second];
            Launch L{true, lead.key, lead.a.w.iso != 0, false, lead.a.ps != 0, host.size(), 0, 0, -1, -1, 0};
            double resident = 0.0;
            for (size_t q = p; q < passes.size(); ++q) {
                const Op &o = ops[passes[q].first][passes[q].second];
                const KernelKey &k = o.key;
                if (done[q] || k.M != lead.key.M || k.T != lead.key.T || k.PY != lead.key.PY ||
                    k.NW != lead.key.NW || k.mode != lead.key.mode || (o.a.w.iso != 0) != L.iso ||
                    o.loads != lead.loads || o.a.ps != lead.a.ps ||
                    shot_lane[passes[q].first] != shot_lane[passes[p].first])
                    continue;
                done[q] = true;
                resident += resident_bytes(o.a, k.mode);
                GroupEntry e{};
                e.a = o.a;
                e.a.remap = 0;  // tiles of a grouped launch are in flat order
                e.tile0 = L.total;
                L.total += o.a.ntz * o.a.nty * o.a.ntx;
                host.push_back(e);
                ++L.n;
            }
            // one workgroup per tile: the hardware dispatcher balances the uneven
            // tiles of different shots (measured on MI355X, 7 % faster for the
            // 32-shot batch than a persistent grid of one workgroup per
            // resident slot walking the table; the kernel supports both).  The
            // grid is padded to a multiple of 8, the XCD count, so that the
            // kernel deals each XCD a contiguous block of tiles (neighbouring
            // tiles of a shot then share that XCD's L2); the padding workgroups
            // find no tile and exit.
            L.grid = (L.total + 7) / 8 * 8;
            // the shots of one grouped launch stream side by side: their fields
            // compete for the cache together
            L.ntl = stream_loads(lead.loads, resident, lead.key.T);
            plan.push_back(L);
            launch_lane.push_back(lane_of[shot_lane[passes[p].first]]);
        }
    }
    if (host.size() > max_entries) return FD_EWORKSPACE;
    if (!host.empty())
        FDW_HIP(hipMemcpyAsync(dev_entries, host.data(), host.size() * sizeof(GroupEntry),
                               hipMemcpyHostToDevice, s));
    FDW_HIP(hipStreamSynchronize(s));
    const int nl = (int)lane_of.size();
    LanePool &pool = lane_pool();
    std::lock_guard<std::mutex> lk(pool.mu);
    grow_lanes(pool, nl > 1 ? nl : 0);
    LaneEvents evs(nl > 1 ? nl + 1 : 0);  // fork, then one join per lane
    auto issue = [&](hipStream_t base) {
        if (nl > 1) {
            FDW_HIP(hipEventRecord(evs.ev[0], base));
            for (int l = 0; l < nl; ++l) FDW_HIP(hipStreamWaitEvent(pool.streams[l], evs.ev[0], 0));
        }
        for (size_t li = 0; li < plan.size(); ++li) {
            const Launch &L = plan[li];
            const hipStream_t st = nl > 1 ? pool.streams[launch_lane[li]] : base;
            if (L.grouped) {
                if (!launch_stream_grouped(L.key, L.iso, L.ntl, L.ps, dev_entries + L.off, L.n, L.total,
                                           L.grid, st))
                    throw Status{FD_EUNSUPPORTED};
                FDW_HIP(hipGetLastError());
            } else {
                const Op &o = ops[L.shot][L.idx];
                if (o.is_pass) {
                    if (!launch_stream(o.key, o.a, st)) throw Status{FD_EUNSUPPORTED};
                    FDW_HIP(hipGetLastError());
                } else {
                    FDW_HIP(o.call(st));
                }
            }
        }
        if (nl > 1)
            for (int l = 0; l < nl; ++l) {
                FDW_HIP(hipEventRecord(evs.ev[1 + l], pool.streams[l]));
                FDW_HIP(hipStreamWaitEvent(base, evs.ev[1 + l], 0));
            }
    };
    if (!graph) {
        issue(s);
        // the fork and join events are destroyed on return: wait for the work
        // that records them (the graph path below synchronises as well)
        FDW_HIP(hipStreamSynchronize(s));
        return FD_OK;
    }
    const hipStream_t cs = pool.capture;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) throw HipFail{e};
    int status = FD_OK;
    try {
        issue(cs);
    } catch (const HipFail &f) {
        e = f.e;
    } catch (const Status &st) {
        status = st.code;
    }
    const hipError_t ec = hipStreamEndCapture(cs, &g);
    if (e == hipSuccess && status == FD_OK) e = ec;
    if (e == hipSuccess && status == FD_OK) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e == hipSuccess && status == FD_OK) e = hipGraphLaunch(ge, s);
    if (e == hipSuccess && status == FD_OK) e = hipStreamSynchronize(s);
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    if (status != FD_OK) return status;
    if (e != hipSuccess) throw HipFail{e};
    return FD_OK;
}

size_t shot_ws(const fd_shot &sh, int op)
{
    return (fd_workspace_size(&sh.grid, &sh.time, &sh.src, &sh.rec, &sh.opts, op) + 255) &
           ~(size_t)255;
}

}  // namespace
}  // namespace fdw

extern "C" size_t fd_batch_workspace_size(int nshots, const fd_shot *shots, int op)
{
    if (nshots < 0 || (nshots > 0 && !shots)) return 0;
    if (op != FD_OP_FORWARD && op != FD_OP_GRADIENT) return 0;
    if (nshots == 0) return 0;
    size_t total = 0, entries = 0;
    for (int i = 0; i < nshots; ++i) {
        const size_t b = fd_workspace_size(&shots[i].grid, &shots[i].time, &shots[i].src,
                                           &shots[i].rec, &shots[i].opts, op);
        if (!b) return 0;
        total += (b + 255) & ~(size_t)255;
        entries += entry_bound(shots[i], op);
    }
    return total + ((entries * sizeof(GroupEntry) + 255) & ~(size_t)255) + 256;
}

extern "C" int fd_forward_batch(int nshots, fd_shot *shots, void *workspace, size_t ws_bytes,
                                uint32_t batch_flags, void *stream)
{
    return guarded([&]() -> int {
        if (nshots < 0 || (nshots > 0 && !shots)) return FD_EINVAL;
        if (nshots == 0) return FD_OK;
        const size_t need = fd_batch_workspace_size(nshots, shots, FD_OP_FORWARD);
        if (!need) return FD_EINVAL;
        if (!workspace || ws_bytes < need || ((uintptr_t)workspace & 255)) return FD_EWORKSPACE;
        std::vector<FwdJob> jobs(nshots);
        std::vector<std::vector<Op>> ops(nshots);
        size_t off = 0, entries = 0;
        for (int i = 0; i < nshots; ++i) {
            fd_shot &sh = shots[i];
            const size_t b = shot_ws(sh, FD_OP_FORWARD);
            const int rc = fwd_setup(jobs[i], &sh.grid, &sh.time, sh.v, &sh.src, &sh.rec, sh.rec_out,
                                     nullptr, (char *)workspace + off, b, &sh.opts, stream);
            if (rc) return rc;
            batch_chunk(jobs[i].c, sh.opts);
            jobs[i].c.ex.rec = &ops[i];
            fwd_issue(jobs[i]);
            off += b;
            entries += entry_bound(sh, FD_OP_FORWARD);
        }
        std::vector<int> shot_m(nshots);
        for (int i = 0; i < nshots; ++i) shot_m[i] = jobs[i].c.d.M;
        return run_merged(ops, shot_m, (GroupEntry *)((char *)workspace + off), entries,
                          (batch_flags & FD_BATCH_GRAPH) != 0, (hipStream_t)stream);
    });
}

extern "C" int fd_gradient_batch(int nshots, fd_shot *shots, void *workspace, size_t ws_bytes,
                                 uint32_t batch_flags, void *stream)
{
    return guarded([&]() -> int {
        if (nshots < 0 || (nshots > 0 && !shots)) return FD_EINVAL;
        if (nshots == 0) return FD_OK;
        const size_t need = fd_batch_workspace_size(nshots, shots, FD_OP_GRADIENT);
        if (!need) return FD_EINVAL;
        if (!workspace || ws_bytes < need || ((uintptr_t)workspace & 255)) return FD_EWORKSPACE;
        std::vector<GradJob> jobs(nshots);
        std::vector<std::vector<Op>> ops(nshots);
        size_t off = 0, entries = 0;
        for (int i = 0; i < nshots; ++i) {
            fd_shot &sh = shots[i];
            const size_t b = shot_ws(sh, FD_OP_GRADIENT);
            const int rc = grad_setup(jobs[i], &sh.grid, &sh.time, sh.v, &sh.src, &sh.rec, nullptr,
                                      sh.grad_v, nullptr, (char *)workspace + off, b, &sh.opts,
                                      stream, FD_OP_GRADIENT);
            if (rc) return rc;
            batch_chunk(jobs[i].c, sh.opts);
            jobs[i].c.ex.rec = &ops[i];
            grad_issue(jobs[i]);
            off += b;
            entries += entry_bound(sh, FD_OP_GRADIENT);
        }
        std::vector<int> shot_m(nshots);
        for (int i = 0; i < nshots; ++i) shot_m[i] = jobs[i].c.d.M;
        const int rc = run_merged(ops, shot_m, (GroupEntry *)((char *)workspace + off), entries,
                                  (batch_flags & FD_BATCH_GRAPH) != 0, (hipStream_t)stream);
        if (rc) return rc;
        for (int i = 0; i < nshots; ++i) shots[i].misfit = grad_misfit(jobs[i]);
        return FD_OK;
    });
}

// ====================================================================== batch autotuner
namespace fdw {
namespace {

// Kernel shapes a class of batched shots can share: compiled as grouped
// kernels for the Laplacian form of every shot in the class.
std::vector<KernelKey> batch_candidates(int M, const std::vector<bool> &forms)
{
    static const int shapes[][2] = {{4, 8}, {4, 4}, {8, 4}, {2, 16}, {2, 8}, {8, 2}, {16, 2}};
    std::vector<KernelKey> out;
    for (int T = 1; T <= 4; ++T)
        for (auto &sh : shapes) {
            const KernelKey k{M, T, sh[0], sh[1], kPlain};
            bool ok = true;
            for (bool iso : forms) ok = ok && stream_has_group(k, iso);
            if (ok) out.push_back(k);
        }
    return out;
}

}  // namespace
}  // namespace fdw

extern "C" int fd_batch_autotune(int nshots, fd_shot *shots, void *workspace, size_t ws_bytes, void *stream)
{
    return guarded([&]() -> int {
        if (nshots < 0 || (nshots > 0 && !shots)) return FD_EINVAL;
        if (!workspace || ((uintptr_t)workspace & 255)) return FD_EWORKSPACE;
        hipStream_t s = (hipStream_t)stream;
        // classes: shots of one stencil radius whose options are automatic
        std::map<int, std::vector<int>> cls;
        for (int i = 0; i < nshots; ++i) {
            Dims d;
            if (make_dims(&shots[i].grid, d)) return FD_EINVAL;
            if (shots[i].opts.variant == FD_VARIANT_AUTO) cls[d.M].push_back(i);
        }
        // seconds per step of a class under options o: two forward runs of n1
        // and n2 = 3 n1 steps (sources only: no receiver buffer is written),
        // differenced, which removes each call's set-up
        constexpr int n1 = 12, n2 = 36;  // multiples of every depth 1..4
        auto run = [&](const std::vector<int> &idx, const fd_options &o, int nt) -> double {
            std::vector<fd_shot> sub;
            for (int i : idx) {
                fd_shot x = shots[i];
                x.time.nt = std::min<int64_t>(x.time.nt, nt);
                x.rec = fd_points{};
                x.rec_out = nullptr;
                x.grad_v = nullptr;
                const uint32_t keep = x.opts.flags;
                x.opts = o;
                x.opts.flags = keep;
                sub.push_back(x);
            }
            const size_t need = fd_batch_workspace_size((int)sub.size(), sub.data(), FD_OP_FORWARD);
            if (!need || need > ws_bytes) throw Status{FD_EWORKSPACE};
            const auto t0 = std::chrono::steady_clock::now();
            const int rc = fd_forward_batch((int)sub.size(), sub.data(), workspace, ws_bytes, 0, stream);
            if (rc) throw Status{rc};
            FDW_HIP(hipStreamSynchronize(s));
            return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        };
        for (auto &kv : cls) {
            const std::vector<int> &idx = kv.second;
            std::vector<bool> forms;
            for (int i : idx) {
                Dims d;
                make_dims(&shots[i].grid, d);
                forms.push_back(grid_iso(d));
            }
            double best = 1e300;
            fd_options best_o{};
            bool found = false;
            for (const KernelKey &k : batch_candidates(kv.first, forms)) {
                for (int lx : {0, 128}) {  // automatic chunk (at least 64 planes), or 128
                    fd_options o{};
                    o.variant = k.T == 1 ? FD_VARIANT_STREAM : FD_VARIANT_TBLOCK;
                    o.tile[0] = lx;
                    o.tile[1] = k.PY * k.NW;
                    o.tile[2] = k.PY;
                    o.tblock = k.T;
                    (void)run(idx, o, n1);  // warm-up
                    const double t = run(idx, o, n2) - run(idx, o, n1);
                    if (t < best) {
                        best = t;
                        best_o = o;
                        found = true;
                    }
                }
            }
            if (!found) continue;  // no grouped kernel for this class: automatic plans stay
            for (int i : idx) {
                const uint32_t keep = shots[i].opts.flags;
                const int32_t ck = shots[i].opts.ckpt_every;
                shots[i].opts = best_o;
                shots[i].opts.flags = keep;
                shots[i].opts.ckpt_every = ck;
            }
        }
        return FD_OK;
    });
}
