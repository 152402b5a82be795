// fake_hip.hip -- a host-memory stand-in for the HIP runtime calls the library
// makes, for checking the library's host code under AddressSanitizer and
// UndefinedBehaviorSanitizer on a machine without a GPU.
//
// Test infrastructure only.  It runs no kernel.  "Device memory" is host
// memory the test driver allocates through hc_dev_alloc().  Copies are
// performed for real, so a copy that overruns a host buffer is an ASan
// report.  Every launch of a sweep kernel (single-pass or grouped) has its
// arguments checked against those allocations: fields, point tables and the
// rows a pass records or injects must lie inside the buffers the caller
// passed, and the tile counts must cover the grid.  Streams and events are
// tracked (use after destroy, a stream destroyed with work not yet known to be
// complete), and graph capture follows the fork/join rules: an event recorded
// during a capture pulls a waiting stream into it, and every such stream must
// be joined back before the capture ends.  Captured work runs (its checks
// included) when the graph is launched.
#include <hip/hip_runtime.h>

#include <cxxabi.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <set>
#include <string>
#include <vector>

#include "../../paper_1707_02347_amd/csrc/fd_internal.h"

namespace {

int g_errors = 0;
bool g_force_wave_timeout = false;  // wave passes end as if a wait ran out
int g_warnings = 0;
long g_launches = 0, g_checked = 0, g_grouped = 0, g_graph_launches = 0;

void fail(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::fprintf(stderr, "hostcheck error: ");
    std::vfprintf(stderr, fmt, ap);
    std::fprintf(stderr, "\n");
    va_end(ap);
    ++g_errors;
}

void warn(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::fprintf(stderr, "hostcheck warning: ");
    std::vfprintf(stderr, fmt, ap);
    std::fprintf(stderr, "\n");
    va_end(ap);
    ++g_warnings;
}

// ------------------------------------------------------------- allocations
std::map<uintptr_t, size_t> g_alloc;  // base -> bytes

bool in_dev(const void *p, size_t bytes)
{
    if (!p) return false;
    const uintptr_t a = (uintptr_t)p;
    auto it = g_alloc.upper_bound(a);
    if (it == g_alloc.begin()) return false;
    --it;
    return a >= it->first && a + bytes <= it->first + it->second;
}

// ------------------------------------------------------------- streams, events, capture
struct Capture;
struct Stream {
    long enq = 0, done = 0;    // ops enqueued / known complete
    Capture *cap = nullptr;    // capture this stream takes part in
    bool origin = false;       // the stream the capture began on
    long cap_ops = 0;          // ops recorded while in the capture
};
struct Event {
    Stream *s = nullptr;       // stream of the last record (nullptr: never recorded)
    long pos = 0;
    Capture *cap = nullptr;    // recorded inside this capture
};
struct Capture {
    Stream *origin = nullptr;
    std::vector<std::function<void()>> ops;
    std::set<Stream *> members;
    std::map<Stream *, long> joined;  // member -> its op count at the last join into origin
    bool ended = false;               // kept after the end: events may still name it
};
struct Graph {
    std::vector<std::function<void()>> ops;
};

std::vector<std::unique_ptr<Capture>> g_captures;  // kept to the end: events may name them
std::set<Stream *> g_streams;
std::set<Event *> g_events;
std::set<Graph *> g_graphs;
Stream g_null;  // the default stream: never destroyed

Stream *S(hipStream_t s, const char *where)
{
    if (!s) return &g_null;
    Stream *p = reinterpret_cast<Stream *>(s);
    if (!g_streams.count(p)) {
        fail("%s on a stream that is not live (%p)", where, (void *)s);
        return &g_null;
    }
    return p;
}

Event *E(hipEvent_t e, const char *where)
{
    Event *p = reinterpret_cast<Event *>(e);
    if (!p || !g_events.count(p)) {
        fail("%s on an event that is not live (%p)", where, (void *)e);
        return nullptr;
    }
    return p;
}

// Enqueue work: run now, or record it into the capture its stream is in.
void enqueue(Stream *s, std::function<void()> f)
{
    if (s->cap) {
        s->cap->ops.push_back(std::move(f));
        ++s->cap_ops;
        return;
    }
    ++s->enq;
    f();
}

// What completes when stream s is synchronised: its own ops and, through the
// events it waited on, the ops of other streams up to those events.
std::map<Stream *, std::vector<std::pair<Stream *, long>>> g_waits;  // s -> (other, pos) it waited on

void complete(Stream *s, long upto, int depth = 0)
{
    if (depth > 64 || s->done >= upto) return;
    s->done = upto;
    for (auto &w : g_waits[s]) complete(w.first, w.second, depth + 1);
}

// ------------------------------------------------------------- kernel registry
struct KInfo {
    std::string name;  // demangled
    int tmpl[8] = {};
    int ntmpl = 0;
    enum { kOther, kStream, kGrouped, kWave, kZero } kind = kOther;
};
// registered from the objects' module constructors, which may run before this
// file's globals are constructed: built on first use
std::map<const void *, KInfo> &kernels()
{
    static std::map<const void *, KInfo> *m = new std::map<const void *, KInfo>();
    return *m;
}

void parse_template(KInfo &k)
{
    const size_t lt = k.name.find('<');
    const size_t gt = k.name.find('>');
    if (lt == std::string::npos || gt == std::string::npos) return;
    std::string args = k.name.substr(lt + 1, gt - lt - 1);
    size_t p = 0;
    while (p < args.size() && k.ntmpl < 8) {
        size_t q = args.find(',', p);
        if (q == std::string::npos) q = args.size();
        std::string t = args.substr(p, q - p);
        while (!t.empty() && t[0] == ' ') t.erase(0, 1);
        k.tmpl[k.ntmpl++] = t == "true" ? 1 : t == "false" ? 0 : std::atoi(t.c_str());
        p = q + 1;
    }
}

// ------------------------------------------------------------- argument checks
using fdw::GroupEntry;
using fdw::PointTable;
using fdw::SweepArgs;

struct Ctx {
    const char *kname;
    int entry;
};

#define CHECK(cond, ...)                                                                   \
    do {                                                                                   \
        if (!(cond)) {                                                                     \
            char buf_[512];                                                                \
            std::snprintf(buf_, sizeof buf_, __VA_ARGS__);                                 \
            fail("%s (entry %d): %s", c.kname, c.entry, buf_);                             \
            return;                                                                        \
        }                                                                                  \
    } while (0)

void check_table(const Ctx &c, const PointTable &t, int nx, int64_t sxy, bool inj)
{
    if (t.cnt == 0) return;
    CHECK(t.cnt > 0 && t.stride > 0, "table cnt %d stride %d", t.cnt, t.stride);
    CHECK(in_dev(t.xptr, (size_t)(nx + 1) * 4), "%s xptr outside the workspace", inj ? "inj" : "rec");
    CHECK(in_dev(t.xe, (size_t)t.cnt * 4) && in_dev(t.yz, (size_t)t.cnt * 4) &&
              in_dev(t.id, (size_t)t.cnt * 4) && in_dev(t.wt, (size_t)t.cnt * 4),
          "%s entry arrays outside the workspace", inj ? "inj" : "rec");
    CHECK(in_dev(t.box, (size_t)nx * 16), "box outside the workspace");
    if (t.scale) CHECK(in_dev(t.scale, (size_t)t.cnt * 4), "scale outside the workspace");
    // the table's contents were copied in for real: check them
    CHECK(t.xptr[0] == 0 && t.xptr[nx] == t.cnt, "xptr spans [%d, %d], cnt %d", t.xptr[0], t.xptr[nx],
          t.cnt);
    for (int x = 0; x < nx; ++x) {
        CHECK(t.xptr[x] <= t.xptr[x + 1], "xptr not monotone at %d", x);
        for (int j = t.xptr[x]; j < t.xptr[x + 1]; ++j) {
            CHECK(t.xe[j] == x, "entry %d has x %d in plane %d", j, t.xe[j], x);
            CHECK(t.yz[j] >= 0 && t.yz[j] < sxy, "entry %d yz %d outside the plane (%lld)", j, t.yz[j],
                  (long long)sxy);
            CHECK(t.id[j] >= 0 && t.id[j] < t.stride, "entry %d id %d of %d points", j, t.id[j], t.stride);
        }
    }
}

// One pass of kernel (M, T, PY, NW, MODE) over the tiles of `a`.
void check_sweep(const Ctx &c, const KInfo &k, const SweepArgs &a, int ps_kernel)
{
    const int M = k.tmpl[0], T = k.tmpl[1], PY = k.tmpl[2], NW = k.tmpl[3], MODE = k.tmpl[4];
    CHECK(a.nx > 0 && a.ny > 0 && a.nz > 0, "extents %d %d %d", a.nx, a.ny, a.nz);
    CHECK(a.nzp >= a.nz && a.nzp % 32 == 0, "row pitch %d for nz %d", a.nzp, a.nz);
    CHECK(a.sxy == (int64_t)a.ny * a.nzp, "plane stride %lld", (long long)a.sxy);
    const size_t F = (size_t)a.nx * a.sxy * 4;
    CHECK(in_dev(a.u0, F), "u0 outside the buffers");
    CHECK(in_dev(a.um, F), "um outside the buffers");
    CHECK(in_dev(a.q, F), "q outside the buffers");
    CHECK(in_dev(a.o1, F), "o1 outside the buffers");
    CHECK(in_dev(a.px, (size_t)a.nx * 4) && in_dev(a.py, (size_t)a.ny * 4) && in_dev(a.pz, (size_t)a.nz * 4),
          "sponge profiles outside the buffers");
    if (T >= 2 || MODE == fdw::kBornFused) {
        CHECK(in_dev(a.o2, F), "o2 outside the buffers");
        CHECK(a.o2 != a.o1, "o1 == o2");
    }
    if (T >= 2) {
        CHECK(a.o1 != a.u0 && a.o1 != a.um && a.o2 != a.u0 && a.o2 != a.um,
              "a time-blocked pass writes over its inputs");
    }
    if (MODE == fdw::kBornFused) {
        CHECK(in_dev(a.u0b, F) && in_dev(a.umb, F) && in_dev(a.bs, F), "Born fields outside the buffers");
    }
    if (MODE == fdw::kBorn) CHECK(in_dev(a.bs, F), "Born coefficient outside the buffers");
    // tiles
    const int rows = NW * PY, cr = rows - 2 * M * (T - 1), cc = 64 - 2 * M * (T - 1);
    CHECK(cr > 0 && cc > 0, "no core for M %d T %d rows %d", M, T, rows);
    CHECK(a.lx >= 1 && a.lx <= fdw::kMaxLx, "chunk %d", a.lx);
    if (a.xstride > 0) {
        // chunks placed at xoff + bx xstride (the inverted trapezoids of a split pass)
        CHECK(a.split == 0 && T == 1 && a.xoff >= 0 && a.ntx >= 1 && a.xoff + (a.ntx - 1) * a.xstride < a.nx,
              "placed chunks: xoff %d stride %d ntx %d nx %d", a.xoff, a.xstride, a.ntx, a.nx);
        CHECK(a.xstride == a.xoff + M && a.lx == 2 * M, "gap chunks: lx %d xoff %d stride %d", a.lx, a.xoff,
              a.xstride);
    } else {
        CHECK(a.xoff == 0, "chunk offset %d without a stride", a.xoff);
        CHECK(a.ntx == (a.nx + a.lx - 1) / a.lx, "ntx %d for nx %d lx %d", a.ntx, a.nx, a.lx);
    }
    if (a.split) {
        CHECK(T == 2 && MODE == fdw::kPlain && a.rec.cnt <= fdw::kStageMin && (a.rec.cnt == 0 || a.ps == 0) &&
                  a.ntx >= 2 && a.lx >= 2 * M + 1,
              "split pass: T %d mode %d receivers %d staged %d ntx %d lx %d", T, MODE, a.rec.cnt, a.ps, a.ntx, a.lx);
    }
    CHECK(a.nty == (a.ny + cr - 1) / cr, "nty %d for ny %d core rows %d", a.nty, a.ny, cr);
    CHECK(a.ntz == (a.nz + cc - 1) / cc, "ntz %d for nz %d core cols %d", a.ntz, a.nz, cc);
    if (a.remap) {
        CHECK(a.gx >= 1 && a.gy >= 1 && a.ntx % a.gx == 0 && a.nty % a.gy == 0 &&
                  ((a.ntx / a.gx) * (a.nty / a.gy)) % 8 == 0,
              "super-tile %d x %d of %d x %d tiles", a.gx, a.gy, a.ntx, a.nty);
    }
    // point tables and the rows each level touches
    check_table(c, a.inj, a.nx, a.sxy, true);
    check_table(c, a.rec, a.nx, a.sxy, false);
    for (int t = 1; t <= T; ++t) {
        const int64_t s = (int64_t)a.step0 + t - 1;
        if (a.inj.cnt > 0) {
            const int64_t row = a.abase + (int64_t)a.adir * s;
            CHECK(row >= 0 && in_dev(a.amp + row * a.inj.stride, (size_t)a.inj.stride * 4),
                  "level %d injects amplitude row %lld outside the buffer", t, (long long)row);
        }
        if (a.rec.cnt > 0) {
            const int64_t row = a.rbase + (int64_t)a.rdir * s;
            if (a.rec.etr)
                CHECK(row >= 0 && in_dev(a.rec.etr + row * a.rec.cnt, (size_t)a.rec.cnt * 4),
                      "level %d records entry row %lld outside the buffer", t, (long long)row);
            else
                CHECK(row >= 0 && in_dev(a.rec_out + row * a.rec.stride, (size_t)a.rec.stride * 4),
                      "level %d records trace row %lld outside the buffer", t, (long long)row);
        }
        if (MODE == fdw::kSaveD2 || MODE == fdw::kImaging || MODE == fdw::kBorn) {
            const int64_t slot = a.dslot0 + (int64_t)a.ddir * (t - 1);
            CHECK(slot >= 0 && in_dev(a.d2 + slot * (int64_t)a.nx * a.sxy, F),
                  "level %d second-difference slot %lld outside the buffer", t, (long long)slot);
        }
    }
    if (MODE == fdw::kImaging) CHECK(in_dev(a.g, F), "imaging partial sums outside the buffers");
    // staged point walks: every chunk's entries (with the time block's overlap
    // planes) within the LDS capacity of the staged kernel form
    if (ps_kernel) {
        CHECK(fdw::points_stageable(M, T, PY, NW), "staged form of a configuration that cannot stage");
        const int cap = fdw::kPtsCap / T, H = (T - 1) * M;
        for (const PointTable *tb : {&a.inj, &a.rec}) {
            if (tb->cnt == 0) continue;
            for (int x0 = 0; x0 < a.nx; x0 += a.lx) {
                const int x1 = std::min(x0 + a.lx, a.nx);
                const int c0 = std::max(x0 - H, 0), c1 = std::min(x1 + H, a.nx);
                CHECK(tb->xptr[c1] - tb->xptr[c0] <= cap, "chunk at %d stages %d entries (cap %d)", x0,
                      tb->xptr[c1] - tb->xptr[c0], cap);
            }
        }
    }
}

// A two-level pass without redundant halos, kernel (M, PY, NW, ISO): one
// workgroup per (y, z) tile over the whole x axis, every workgroup resident at
// once (the stand-in's occupancy times 256 CUs), counters for every tile, and
// an epoch that starts at 1 after the counters were cleared and then grows by
// one per pass.
std::map<const void *, uint32_t> &epochs()
{
    static std::map<const void *, uint32_t> *m = new std::map<const void *, uint32_t>();
    return *m;
}

void check_wave(const Ctx &c, const KInfo &k, dim3 grid, dim3 block, const SweepArgs &a)
{
    const int M = k.tmpl[0], PY = k.tmpl[1], NW = k.tmpl[2];
    CHECK(block.x == (unsigned)(64 * NW) && block.y == 1 && block.z == 1, "block %u", block.x);
    CHECK(a.nx > 0 && a.ny > 0 && a.nz > 0 && a.nzp >= a.nz && a.nzp % 32 == 0 && a.sxy == (int64_t)a.ny * a.nzp,
          "extents %d %d %d pitch %d", a.nx, a.ny, a.nz, a.nzp);
    CHECK(a.ntz == (a.nz + 63) / 64 && a.nty == (a.ny + PY * NW - 1) / (PY * NW) && a.ntx == 1 && a.lx == a.nx,
          "tiles %d x %d x %d (lx %d) for %d x %d x %d", a.ntz, a.nty, a.ntx, a.lx, a.nx, a.ny, a.nz);
    CHECK(grid.x == (unsigned)(a.ntz * a.nty) && grid.y == 1 && grid.z == 1, "grid %u for %d tiles", grid.x,
          a.ntz * a.nty);
    CHECK(grid.x <= 2u * 256u, "grid %u beyond the resident workgroups", grid.x);
    const size_t F = (size_t)a.nx * a.sxy * 4;
    CHECK(in_dev(a.u0, F) && in_dev(a.um, F) && in_dev(a.q, F) && in_dev(a.o1, F) && in_dev(a.o2, F),
          "a field outside the buffers");
    CHECK(a.o1 != a.o2 && a.o1 != a.u0 && a.o1 != a.um && a.o2 != a.u0 && a.o2 != a.um,
          "the pass writes over its inputs or one output twice");
    CHECK(in_dev(a.px, (size_t)a.nx * 4) && in_dev(a.py, (size_t)a.ny * 4) && in_dev(a.pz, (size_t)a.nz * 4),
          "sponge profiles outside the buffers");
    CHECK(in_dev(a.prog, (size_t)a.ntz * a.nty * fdw::kWaveProgStride * 8) && in_dev(a.err, 4),
          "counters outside the workspace");
    CHECK(in_dev(a.ptab, (size_t)a.nx * fdw::kPlaneTab * 4), "per-plane table outside the workspace");
    // the table must describe the pass's point tables
    for (int x = 0; x < a.nx; ++x) {
        const int32_t *e = a.ptab + (size_t)x * fdw::kPlaneTab;
        const int ib = a.inj.cnt ? a.inj.xptr[x] : 0, ie = a.inj.cnt ? a.inj.xptr[x + 1] : 0;
        const int rb = a.rec.cnt ? a.rec.xptr[x] : 0, re = a.rec.cnt ? a.rec.xptr[x + 1] : 0;
        float px;
        std::memcpy(&px, &e[0], 4);
        CHECK(px == a.px[x] && e[1] == ib && e[2] == ie && e[3] == rb && e[4] == re &&
                  e[5] == ((ie > ib ? 1 : 0) | (re > rb ? 2 : 0)),
              "per-plane table entry %d does not match the pass's tables", x);
        if (re > rb)
            CHECK(e[6] == a.rec.yz[rb] && e[7] == (a.rec.etr ? rb : a.rec.id[rb]),
                  "per-plane table entry %d: first receiver entry (%d, %d) is not (%d, %d)", x, e[6], e[7],
                  a.rec.yz[rb], a.rec.etr ? rb : a.rec.id[rb]);
    }
    CHECK(a.epoch >= 1, "epoch 0");
    uint32_t &last = epochs()[a.prog];
    CHECK(a.epoch == 1 || a.epoch == last + 1, "epoch %u after %u", a.epoch, last);
    last = a.epoch;
    CHECK(a.split == 0 && a.ps == 0 && a.xstride == 0 && a.xoff == 0, "split / staged / placed chunks");
    check_table(c, a.inj, a.nx, a.sxy, true);
    check_table(c, a.rec, a.nx, a.sxy, false);
    for (int t = 1; t <= 2; ++t) {
        const int64_t s = (int64_t)a.step0 + t - 1;
        if (a.inj.cnt > 0) {
            const int64_t row = a.abase + (int64_t)a.adir * s;
            CHECK(row >= 0 && in_dev(a.amp + row * a.inj.stride, (size_t)a.inj.stride * 4),
                  "level %d injects amplitude row %lld outside the buffer", t, (long long)row);
        }
        if (a.rec.cnt > 0) {
            const int64_t row = a.rbase + (int64_t)a.rdir * s;
            if (a.rec.etr)
                CHECK(row >= 0 && in_dev(a.rec.etr + row * a.rec.cnt, (size_t)a.rec.cnt * 4),
                      "level %d records entry row %lld outside the buffer", t, (long long)row);
            else
                CHECK(row >= 0 && in_dev(a.rec_out + row * a.rec.stride, (size_t)a.rec.stride * 4),
                      "level %d records trace row %lld outside the buffer", t, (long long)row);
        }
    }
    (void)M;
}

void check_launch(const KInfo &k, dim3 grid, dim3 block, void **args)
{
    Ctx c{k.name.c_str(), -1};
    if (k.kind == KInfo::kStream) {
        ++g_checked;
        const SweepArgs &a = *reinterpret_cast<const SweepArgs *>(args[0]);
        const int NW = k.tmpl[3];
        CHECK(block.x == (unsigned)(64 * NW) && block.y == 1 && block.z == 1, "block %u", block.x);
        CHECK(grid.x == (unsigned)(a.ntx * a.nty * a.ntz) && grid.y == 1 && grid.z == 1,
              "grid %u for %d tiles", grid.x, a.ntx * a.nty * a.ntz);
        CHECK(a.ps == k.tmpl[7], "staged flag %d in kernel form %d", a.ps, k.tmpl[7]);
        check_sweep(c, k, a, k.tmpl[7]);
    } else if (k.kind == KInfo::kWave) {
        ++g_checked;
        check_wave(c, k, grid, block, *reinterpret_cast<const SweepArgs *>(args[0]));
    } else if (k.kind == KInfo::kGrouped) {
        ++g_grouped;
        const GroupEntry *list = *reinterpret_cast<const GroupEntry *const *>(args[0]);
        const int n = *reinterpret_cast<const int *>(args[1]);
        const int total = *reinterpret_cast<const int *>(args[2]);
        const int NW = k.tmpl[3];
        CHECK(block.x == (unsigned)(64 * NW), "block %u", block.x);
        CHECK(n >= 1 && in_dev(list, (size_t)n * sizeof(GroupEntry)), "table of %d entries outside the workspace", n);
        CHECK(grid.x >= 1 && (int)grid.x <= (total + 7) / 8 * 8, "grid %u for %d tiles", grid.x, total);
        int next = 0;
        for (int e = 0; e < n; ++e) {
            c.entry = e;
            const GroupEntry &g = list[e];
            CHECK(g.tile0 == next, "tile0 %d, expected %d", g.tile0, next);
            CHECK(g.a.remap == 0, "remapped entry in a grouped launch");
            next += g.a.ntx * g.a.nty * g.a.ntz;
            check_sweep(c, k, g.a, k.tmpl[7]);
        }
        c.entry = -1;
        CHECK(next == total, "entries cover %d tiles, launch says %d", next, total);
    }
}

// ------------------------------------------------------------- launch configuration stack
struct Cfg {
    dim3 grid, block;
    size_t shm;
    hipStream_t s;
};
std::vector<Cfg> g_cfg;

}  // namespace

// =============================================================== the runtime calls
extern "C" {

void **__hipRegisterFatBinary(const void *) { static void *m = nullptr; return &m; }
void __hipUnregisterFatBinary(void **) {}
void __hipRegisterFunction(void **, const void *host, char *, const char *dev_name, unsigned int,
                           void *, void *, void *, void *, int *)
{
    KInfo k;
    int st = 0;
    char *dm = abi::__cxa_demangle(dev_name, nullptr, nullptr, &st);
    k.name = (st == 0 && dm) ? dm : dev_name;
    std::free(dm);
    if (k.name.rfind("void fdw::k_stream_grouped<", 0) == 0) k.kind = KInfo::kGrouped;
    else if (k.name.rfind("void fdw::k_stream<", 0) == 0) k.kind = KInfo::kStream;
    else if (k.name.rfind("void fdw::k_wave<", 0) == 0) k.kind = KInfo::kWave;
    else if (k.name.rfind("fdw::k_zero(", 0) == 0) k.kind = KInfo::kZero;
    parse_template(k);
    kernels()[host] = k;
}
// device variables: their host shadows stand in for the device copies
std::map<const void *, size_t> &vars()
{
    static std::map<const void *, size_t> *m = new std::map<const void *, size_t>();
    return *m;
}
void __hipRegisterVar(void **, void *var, char *, const char *, int, size_t size, int, int)
{
    vars()[var] = size;
}
hipError_t hipGetSymbolAddress(void **p, const void *symbol)
{
    auto it = vars().find(symbol);
    if (it == vars().end()) {
        fail("address of an unregistered device symbol");
        return hipErrorInvalidSymbol;
    }
    g_alloc[(uintptr_t)symbol] = it->second;
    *p = const_cast<void *>(symbol);
    return hipSuccess;
}

hipError_t __hipPushCallConfiguration(dim3 grid, dim3 block, size_t shm, hipStream_t s)
{
    g_cfg.push_back(Cfg{grid, block, shm, s});
    return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3 *grid, dim3 *block, size_t *shm, hipStream_t *s)
{
    if (g_cfg.empty()) {
        fail("launch configuration popped without a push");
        return hipErrorInvalidValue;
    }
    *grid = g_cfg.back().grid;
    *block = g_cfg.back().block;
    *shm = g_cfg.back().shm;
    *s = g_cfg.back().s;
    g_cfg.pop_back();
    return hipSuccess;
}

hipError_t hipLaunchKernel(const void *fn, dim3 grid, dim3 block, void **args, size_t, hipStream_t s)
{
    ++g_launches;
    auto it = kernels().find(fn);
    if (it == kernels().end()) {
        fail("launch of an unregistered kernel %p", fn);
        return hipErrorInvalidDeviceFunction;
    }
    if (grid.x == 0 || block.x == 0 || block.x > 1024) fail("%s: grid %u block %u", it->second.name.c_str(), grid.x, block.x);
    const KInfo &k = it->second;
    // the arguments are only valid during the call: copy what the checks read
    if (k.kind == KInfo::kStream || k.kind == KInfo::kWave) {
        SweepArgs a = *reinterpret_cast<const SweepArgs *>(args[0]);
        const bool timeout = k.kind == KInfo::kWave && g_force_wave_timeout;
        enqueue(S(s, "hipLaunchKernel"), [k, grid, block, a, timeout]() {
            void *ar[1] = {(void *)&a};
            check_launch(k, grid, block, ar);
            if (timeout && in_dev(a.err, 4)) *a.err = 1;  // what a wait that runs out leaves
        });
    } else if (k.kind == KInfo::kZero) {
        // the fill kernel runs for real: the library clears counters and error
        // words with it
        uint32_t *p = *reinterpret_cast<uint32_t *const *>(args[0]);
        const int64_t n = *reinterpret_cast<const int64_t *>(args[1]);
        enqueue(S(s, "hipLaunchKernel"), [p, n]() {
            if (n < 0 || !in_dev(p, (size_t)n * 4)) {
                fail("k_zero over %lld words at %p outside the device buffers", (long long)n, (void *)p);
                return;
            }
            std::memset(p, 0, (size_t)n * 4);
        });
    } else if (k.kind == KInfo::kGrouped) {
        const GroupEntry *list = *reinterpret_cast<const GroupEntry *const *>(args[0]);
        const int n = *reinterpret_cast<const int *>(args[1]);
        const int total = *reinterpret_cast<const int *>(args[2]);
        enqueue(S(s, "hipLaunchKernel"), [k, grid, block, list, n, total]() {
            const GroupEntry *l = list;
            int nn = n, tt = total;
            void *ar[3] = {(void *)&l, (void *)&nn, (void *)&tt};
            check_launch(k, grid, block, ar);
        });
    } else {
        enqueue(S(s, "hipLaunchKernel"), []() {});
    }
    return hipSuccess;
}

hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipGetDevice(int *d)
{
    *d = 0;
    return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t attr, int)
{
    *v = attr == hipDeviceAttributeMultiprocessorCount ? 256 : 1;
    return hipSuccess;
}
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *n, const void *fn, int block, size_t)
{
    if (!kernels().count(fn)) fail("occupancy query of an unregistered kernel");
    *n = block >= 1024 ? 1 : 2;
    return hipSuccess;
}

hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    const bool ddst = in_dev(dst, bytes), dsrc = in_dev(src, bytes);
    switch (kind) {
    case hipMemcpyHostToDevice:
        if (!ddst) fail("host-to-device copy of %zu bytes to %p outside the device buffers", bytes, dst);
        break;
    case hipMemcpyDeviceToHost:
        if (!dsrc) fail("device-to-host copy of %zu bytes from %p outside the device buffers", bytes, src);
        break;
    case hipMemcpyDeviceToDevice:
        if (!ddst || !dsrc) fail("device-to-device copy of %zu bytes outside the device buffers", bytes);
        break;
    default: break;
    }
    Stream *st = S(s, "hipMemcpyAsync");
    if (kind == hipMemcpyHostToDevice || kind == hipMemcpyDeviceToHost) {
        // pageable copies: the runtime stages them before returning (HtoD), or
        // the host reads them after a synchronisation (DtoH); a copy between
        // host memory and the device cannot be captured in this library's use
        if (st->cap) fail("host copy recorded into a graph capture");
        ++st->enq;
        std::memcpy(dst, src, bytes);
        return hipSuccess;
    }
    enqueue(st, [dst, src, bytes]() { std::memmove(dst, src, bytes); });
    return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int)
{
    Stream *p = new Stream();
    g_streams.insert(p);
    *s = reinterpret_cast<hipStream_t>(p);
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s)
{
    Stream *p = S(s, "hipStreamDestroy");
    if (p == &g_null) return hipErrorInvalidHandle;
    if (p->cap) fail("stream destroyed while in a capture");
    if (p->done < p->enq) warn("stream destroyed with %ld ops not known to be complete", p->enq - p->done);
    g_streams.erase(p);
    g_waits.erase(p);
    for (auto &w : g_waits) {
        auto &v = w.second;
        v.erase(std::remove_if(v.begin(), v.end(), [p](const std::pair<Stream *, long> &x) { return x.first == p; }),
                v.end());
    }
    delete p;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s)
{
    Stream *p = S(s, "hipStreamSynchronize");
    if (p->cap) {
        fail("stream synchronised during a capture");
        return hipErrorStreamCaptureUnsupported;
    }
    complete(p, p->enq);
    return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned int)
{
    Event *p = new Event();
    g_events.insert(p);
    *e = reinterpret_cast<hipEvent_t>(p);
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) { return hipEventCreateWithFlags(e, 0); }
hipError_t hipEventDestroy(hipEvent_t e)
{
    Event *p = E(e, "hipEventDestroy");
    if (!p) return hipErrorInvalidHandle;
    g_events.erase(p);
    delete p;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    Event *p = E(e, "hipEventRecord");
    Stream *st = S(s, "hipEventRecord");
    if (!p) return hipErrorInvalidHandle;
    p->s = st;
    p->pos = st->cap ? st->cap_ops : st->enq;
    p->cap = st->cap;
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int)
{
    Event *p = E(e, "hipStreamWaitEvent");
    Stream *st = S(s, "hipStreamWaitEvent");
    if (!p) return hipErrorInvalidHandle;
    if (!p->s) return hipSuccess;  // never recorded: no dependency
    if (p->cap) {
        Capture *c = p->cap;
        if (c->ended) {
            fail("stream waits on an event recorded in a capture that has ended");
            return hipErrorStreamCaptureIsolation;
        }
        if (st->cap && st->cap != c) {
            fail("stream waits on an event of another capture");
            return hipErrorStreamCaptureIsolation;
        }
        if (!st->cap) {  // fork: st joins the capture
            st->cap = c;
            st->cap_ops = 0;
            c->members.insert(st);
        }
        if (st == c->origin && p->s != c->origin) c->joined[p->s] = p->pos;  // join
        return hipSuccess;
    }
    if (st->cap) {
        // a dependency on work outside the capture: legal, nothing to record
        return hipSuccess;
    }
    g_waits[st].push_back({p->s, p->pos});
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e)
{
    Event *p = E(e, "hipEventSynchronize");
    if (p && p->s) complete(p->s, p->pos);
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b)
{
    if (!E(a, "hipEventElapsedTime") || !E(b, "hipEventElapsedTime")) return hipErrorInvalidHandle;
    *ms = 1.0f;
    return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode)
{
    Stream *st = S(s, "hipStreamBeginCapture");
    if (st == &g_null) return hipErrorStreamCaptureUnsupported;
    if (st->cap) return hipErrorIllegalState;
    g_captures.emplace_back(new Capture());
    Capture *c = g_captures.back().get();
    c->origin = st;
    st->cap = c;
    st->origin = true;
    st->cap_ops = 0;
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g)
{
    Stream *st = S(s, "hipStreamEndCapture");
    Capture *c = st->cap;
    if (!c || c->origin != st) {
        fail("capture ended on a stream that did not begin it");
        return hipErrorIllegalState;
    }
    hipError_t rc = hipSuccess;
    for (Stream *m : c->members) {
        auto it = c->joined.find(m);
        if (it == c->joined.end() || it->second < m->cap_ops) {
            fail("a stream forked into the capture was not joined back before its end");
            rc = hipErrorStreamCaptureUnjoined;
        }
        m->cap = nullptr;
    }
    st->cap = nullptr;
    st->origin = false;
    Graph *gr = new Graph();
    gr->ops = std::move(c->ops);
    c->ended = true;  // not freed: events recorded in it still point here
    g_graphs.insert(gr);
    *g = reinterpret_cast<hipGraph_t>(gr);
    return rc;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *ge, hipGraph_t g, hipGraphNode_t *, char *, size_t)
{
    Graph *gr = reinterpret_cast<Graph *>(g);
    if (!g_graphs.count(gr)) {
        fail("instantiate of a graph that is not live");
        return hipErrorInvalidValue;
    }
    Graph *ex = new Graph(*gr);
    g_graphs.insert(ex);
    *ge = reinterpret_cast<hipGraphExec_t>(ex);
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t ge, hipStream_t s)
{
    Graph *ex = reinterpret_cast<Graph *>(ge);
    if (!g_graphs.count(ex)) {
        fail("launch of a graph that is not live");
        return hipErrorInvalidValue;
    }
    ++g_graph_launches;
    Stream *st = S(s, "hipGraphLaunch");
    for (auto &f : ex->ops) f();
    ++st->enq;
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t ge)
{
    Graph *ex = reinterpret_cast<Graph *>(ge);
    if (!g_graphs.erase(ex)) return hipErrorInvalidValue;
    delete ex;
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g)
{
    Graph *gr = reinterpret_cast<Graph *>(g);
    if (!g_graphs.erase(gr)) return hipErrorInvalidValue;
    delete gr;
    return hipSuccess;
}

// ------------------------------------------------------------- test driver hooks
void *hc_dev_alloc(size_t bytes)
{
    void *p = std::calloc(1, bytes ? bytes : 1);
    g_alloc[(uintptr_t)p] = bytes;
    return p;
}
void hc_dev_free(void *p)
{
    if (!p) return;
    if (!g_alloc.erase((uintptr_t)p)) fail("free of an unknown device buffer");
    std::free(p);
}
int hc_errors(void) { return g_errors; }
void hc_force_wave_timeout(int on) { g_force_wave_timeout = on != 0; }
int hc_warnings(void) { return g_warnings; }
void hc_stats(long *launches, long *checked, long *grouped, long *graphs)
{
    *launches = g_launches;
    *checked = g_checked;
    *grouped = g_grouped;
    *graphs = g_graph_launches;
}
// events and graphs still alive (each batch must release its own); streams
// may live on by design (the library's lane pools)
int hc_live_handles(void) { return (int)(g_events.size() + g_graphs.size()); }
int hc_live_streams(void) { return (int)g_streams.size(); }

}  // extern "C"
