// driver.cpp -- calls every entry point of libfdwave's C ABI against the
// host-memory runtime stand-in (fake_hip.hip), so that the library's host code
// (validation, planning, point tables, workspace carving, recorded batches,
// graph capture) runs under AddressSanitizer and UndefinedBehaviorSanitizer.
// No kernel runs: the checks are the sanitizers' and the stand-in's argument
// checks.  Exit status: 0 when every call returned its expected status and
// the stand-in reported no error.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fdwave.h"

extern "C" {
void *hc_dev_alloc(size_t bytes);
void hc_dev_free(void *p);
int hc_errors(void);
void hc_force_wave_timeout(int on);
int hc_warnings(void);
void hc_stats(long *launches, long *checked, long *grouped, long *graphs);
int hc_live_handles(void);
int hc_live_streams(void);
}

namespace {

int g_bad = 0;

void expect(int rc, int want, const std::string &what)
{
    if (rc != want) {
        std::fprintf(stderr, "driver: %s returned %d (%s), expected %d\n", what.c_str(), rc, fd_strerror(rc),
                     want);
        ++g_bad;
    } else {
        std::printf("ok   %s\n", what.c_str());
    }
    std::fflush(stdout);
}

struct Buf {
    void *p = nullptr;
    size_t n = 0;
    explicit Buf(size_t bytes) : p(hc_dev_alloc(bytes)), n(bytes) {}
    ~Buf() { hc_dev_free(p); }
    Buf(const Buf &) = delete;
    Buf &operator=(const Buf &) = delete;
    float *f() { return (float *)p; }
};

fd_grid grid(std::vector<int> n, int so, int sponge = 4)
{
    fd_grid g;
    std::memset(&g, 0, sizeof g);
    g.ndim = (int)n.size();
    g.space_order = so;
    for (size_t a = 0; a < n.size(); ++a) {
        g.n[a] = n[a];
        g.h[a] = 10.0;
    }
    g.sponge = sponge;
    g.sponge_vref = 4500.0;
    return g;
}

int64_t points(const fd_grid &g)
{
    int64_t N = 1;
    for (int a = 0; a < g.ndim; ++a) N *= g.n[a];
    return N;
}

fd_options opts(int variant = 0, int t0 = 0, int t1 = 0, int t2 = 0, int tb = 0, uint32_t flags = 0,
                int ck = 0)
{
    fd_options o;
    std::memset(&o, 0, sizeof o);
    o.variant = variant;
    o.tile[0] = t0;
    o.tile[1] = t1;
    o.tile[2] = t2;
    o.tblock = tb;
    o.flags = flags;
    o.ckpt_every = ck;
    return o;
}

// Point sets with host arrays kept alive.
struct Pts {
    std::vector<int32_t> idx;
    std::vector<double> pos;
    fd_points p;
    Pts() { std::memset(&p, 0, sizeof p); }
    Pts(const Pts &o) : idx(o.idx), pos(o.pos), p(o.p) { fix(); }
    Pts &operator=(const Pts &o)
    {
        idx = o.idx;
        pos = o.pos;
        p = o.p;
        fix();
        return *this;
    }
    void fix()
    {
        p.idx = idx.empty() ? nullptr : idx.data();
        p.pos = pos.empty() ? nullptr : pos.data();
    }
};

Pts centre_src(const fd_grid &g, int depth)
{
    Pts s;
    for (int a = 0; a < g.ndim; ++a) s.idx.push_back(a == g.ndim - 1 ? depth : (int)(g.n[a] / 2));
    s.p.n = 1;
    s.fix();
    return s;
}

Pts rec_line(const fd_grid &g, int step, int depth)
{
    Pts r;
    for (int x = 0; x < g.n[0]; x += step) {
        r.idx.push_back(x);
        if (g.ndim == 3) r.idx.push_back((int)(g.n[1] / 2));
        if (g.ndim >= 2) r.idx.push_back(depth);
        ++r.p.n;
    }
    r.fix();
    return r;
}

// n points at seeded positions between nodes (interp 0: multilinear, r: sinc)
Pts scattered(const fd_grid &g, int n, int interp, unsigned seed)
{
    Pts r;
    unsigned s = seed;
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < g.ndim; ++a) {
            s = s * 1103515245u + 12345u;
            const double u = ((s >> 8) & 0xffff) / 65536.0;
            r.pos.push_back(u * (double)(g.n[a] - 1));
        }
    r.p.n = n;
    r.p.interp = interp;
    r.fix();
    return r;
}

double stable_dt(const fd_grid &g) { return 0.3 * 10.0 / 2000.0; }

// ---------------------------------------------------------------- single-shot calls
void forward_case(const std::string &name, const fd_grid &g, int64_t nt, Pts src, Pts rec, fd_options o,
                  bool with_state, int want = FD_OK)
{
    const fd_time t{nt, stable_dt(g)};
    const int64_t N = points(g);
    Buf v(N * 4), amp((size_t)std::max<int64_t>(nt, 1) * std::max(src.p.n, 1) * 4);
    Buf out((size_t)std::max<int64_t>(nt, 1) * std::max(rec.p.n, 1) * 4), st(2 * N * 4);
    for (int64_t i = 0; i < N; ++i) v.f()[i] = 2000.0f;
    src.p.amp = amp.f();
    const size_t ws = fd_workspace_size(&g, &t, &src.p, &rec.p, &o, FD_OP_FORWARD);
    Buf w(ws);
    expect(fd_forward(&g, &t, v.f(), &src.p, &rec.p, rec.p.n ? out.f() : nullptr, with_state ? st.f() : nullptr,
                      w.p, ws, &o, nullptr),
           want, "forward " + name);
}

void adjoint_case(const std::string &name, const fd_grid &g, int64_t nt, Pts src, Pts rec, fd_options o)
{
    const fd_time t{nt, stable_dt(g)};
    const int64_t N = points(g);
    Buf v(N * 4), res((size_t)nt * std::max(rec.p.n, 1) * 4), so((size_t)nt * std::max(src.p.n, 1) * 4),
        lam(2 * N * 4);
    for (int64_t i = 0; i < N; ++i) v.f()[i] = 2000.0f;
    rec.p.amp = res.f();
    const size_t ws = fd_workspace_size(&g, &t, &src.p, &rec.p, &o, FD_OP_ADJOINT);
    Buf w(ws);
    expect(fd_adjoint(&g, &t, v.f(), &src.p, &rec.p, so.f(), lam.f(), w.p, ws, &o, nullptr), FD_OK,
           "adjoint " + name);
}

void gradient_case(const std::string &name, const fd_grid &g, int64_t nt, Pts src, Pts rec, fd_options o,
                   bool vjp)
{
    const fd_time t{nt, stable_dt(g)};
    const int64_t N = points(g);
    Buf v(N * 4), amp((size_t)nt * std::max(src.p.n, 1) * 4), dob((size_t)nt * std::max(rec.p.n, 1) * 4),
        gv(N * 4), resid((size_t)nt * std::max(rec.p.n, 1) * 4);
    for (int64_t i = 0; i < N; ++i) v.f()[i] = 2000.0f;
    src.p.amp = amp.f();
    rec.p.amp = dob.f();
    const int op = vjp ? FD_OP_VJP : FD_OP_GRADIENT;
    const size_t ws = fd_workspace_size(&g, &t, &src.p, &rec.p, &o, op);
    Buf w(ws);
    double J = -1.0;
    if (vjp)
        expect(fd_vjp(&g, &t, v.f(), &src.p, &rec.p, gv.f(), w.p, ws, &o, nullptr), FD_OK, "vjp " + name);
    else
        expect(fd_gradient(&g, &t, v.f(), &src.p, &rec.p, gv.f(), &J, resid.f(), w.p, ws, &o, nullptr), FD_OK,
               "gradient " + name);
}

void born_case(const std::string &name, const fd_grid &g, int64_t nt, Pts src, Pts rec, fd_options o)
{
    const fd_time t{nt, stable_dt(g)};
    const int64_t N = points(g);
    Buf v(N * 4), dv(N * 4), amp((size_t)nt * std::max(src.p.n, 1) * 4),
        out((size_t)nt * std::max(rec.p.n, 1) * 4);
    for (int64_t i = 0; i < N; ++i) v.f()[i] = 2000.0f;
    src.p.amp = amp.f();
    const size_t ws = fd_workspace_size(&g, &t, &src.p, &rec.p, &o, FD_OP_BORN);
    Buf w(ws);
    expect(fd_born(&g, &t, v.f(), dv.f(), &src.p, &rec.p, out.f(), w.p, ws, &o, nullptr), FD_OK, "born " + name);
}

void noalloc_case(const std::string &name, const fd_grid &g, int64_t nt, Pts src, Pts rec, fd_options o, int want)
{
    const fd_time t{nt, stable_dt(g)};
    const int64_t N = points(g);
    Buf v(N * 4), amp((size_t)std::max<int64_t>(nt, 1) * std::max(src.p.n, 1) * 4);
    Buf out((size_t)std::max<int64_t>(nt, 1) * std::max(rec.p.n, 1) * 4), st(2 * N * 4);
    for (int64_t i = 0; i < N; ++i) v.f()[i] = 2000.0f;
    src.p.amp = amp.f();
    expect(fd_forward_noalloc(&g, &t, v.f(), &src.p, &rec.p, rec.p.n ? out.f() : nullptr, st.f(), &o, nullptr), want,
           "forward without allocation " + name);
}

// ---------------------------------------------------------------- batches
struct ShotSpec {
    std::vector<int> n;
    int so;
    int64_t nt;
    fd_options o;
};

void batch_case(const std::string &name, const std::vector<ShotSpec> &specs, bool gradient, uint32_t bflags,
                uint32_t flags)
{
    std::vector<fd_shot> shots(specs.size());
    std::vector<Pts> srcs, recs;
    std::vector<Buf *> bufs;
    srcs.reserve(specs.size());
    recs.reserve(specs.size());
    for (size_t i = 0; i < specs.size(); ++i) {
        const ShotSpec &sp = specs[i];
        fd_shot &sh = shots[i];
        std::memset(&sh, 0, sizeof sh);
        sh.grid = grid(sp.n, sp.so);
        sh.time = fd_time{sp.nt, stable_dt(sh.grid)};
        const int64_t N = points(sh.grid);
        Buf *v = new Buf(N * 4);
        for (int64_t k = 0; k < N; ++k) v->f()[k] = 2000.0f;
        bufs.push_back(v);
        sh.v = v->f();
        srcs.push_back(centre_src(sh.grid, sp.n.back() / 3));
        recs.push_back(rec_line(sh.grid, 7, sp.n.back() / 3));
        Buf *amp = new Buf((size_t)sp.nt * 4);
        bufs.push_back(amp);
        srcs.back().p.amp = amp->f();
        Buf *tr = new Buf((size_t)sp.nt * recs.back().p.n * 4);
        bufs.push_back(tr);
        sh.src = srcs.back().p;
        sh.rec = recs.back().p;
        if (gradient) {
            sh.rec.amp = tr->f();
            Buf *gv = new Buf(N * 4);
            bufs.push_back(gv);
            sh.grad_v = gv->f();
        } else {
            sh.rec_out = tr->f();
        }
        sh.opts = sp.o;
        sh.opts.flags |= flags;
    }
    const int op = gradient ? FD_OP_GRADIENT : FD_OP_FORWARD;
    const size_t ws = fd_batch_workspace_size((int)shots.size(), shots.data(), op);
    Buf w(ws);
    const int rc = gradient ? fd_gradient_batch((int)shots.size(), shots.data(), w.p, ws, bflags, nullptr)
                            : fd_forward_batch((int)shots.size(), shots.data(), w.p, ws, bflags, nullptr);
    expect(rc, FD_OK, std::string(gradient ? "gradient batch " : "forward batch ") + name);
    for (Buf *b : bufs) delete b;
}

}  // namespace

int main()
{
    // a cached exchange choice for a grid of 576 tiles, more than the stand-in's
    // 512 resident workgroups: written before the library first reads its cache
    const fd_grid gbig = grid({3, 136, 4096}, 8, 0);
    if (const char *cache = std::getenv("FD_AUTOTUNE_CACHE")) {
        if (FILE *f = std::fopen(cache, "a")) {
            std::fprintf(f, "3 3 136 4096 8 gfx950 iso %d 3 16 2 2\n", FD_VARIANT_WAVE);
            std::fclose(f);
        }
    }
    const fd_grid g3 = grid({40, 38, 44}, 8), g3p = grid({36, 40, 64}, 8);
    // forward: every variant, state in and out (converted and in place), cache policies
    forward_case("so8 naive", g3, 24, centre_src(g3, 12), rec_line(g3, 7, 12), opts(FD_VARIANT_NAIVE), true);
    forward_case("so8 stream", g3, 24, centre_src(g3, 12), rec_line(g3, 7, 12), opts(FD_VARIANT_STREAM), true);
    forward_case("so8 stream in place", g3p, 24, centre_src(g3p, 12), rec_line(g3p, 7, 12), opts(FD_VARIANT_STREAM),
                 true);
    forward_case("so8 T2", g3, 25, centre_src(g3, 12), rec_line(g3, 7, 12), opts(FD_VARIANT_TBLOCK, 0, 0, 0, 2), true);
    forward_case("so8 auto", g3, 24, centre_src(g3, 12), rec_line(g3, 7, 12), opts(), false);
    for (uint32_t f : {FD_FLAG_LOADS_STREAM, FD_FLAG_LOADS_KEEP})
        forward_case("so8 stream flags " + std::to_string(f), g3, 24, centre_src(g3, 12), rec_line(g3, 7, 12),
                     opts(FD_VARIANT_STREAM, 0, 0, 0, 0, f), false);
    const fd_grid g4 = grid({42, 37, 45}, 4), g2o = grid({46, 41, 70}, 2);
    forward_case("so4 T2", g4, 33, centre_src(g4, 15), rec_line(g4, 7, 15), opts(FD_VARIANT_TBLOCK, 0, 0, 0, 2), true);
    forward_case("so4 T3 tile", g4, 33, centre_src(g4, 15), rec_line(g4, 7, 15),
                 opts(FD_VARIANT_TBLOCK, 0, 32, 4, 3), true);
    forward_case("so2 T4", g2o, 31, centre_src(g2o, 9), rec_line(g2o, 5, 9), opts(FD_VARIANT_TBLOCK, 0, 0, 0, 4),
                 true);
    forward_case("so4 split", g4, 33, centre_src(g4, 15), Pts(), opts(FD_VARIANT_SPLIT, 9), true);
    forward_case("so2 split receivers", g2o, 31, centre_src(g2o, 9), rec_line(g2o, 5, 9), opts(FD_VARIANT_SPLIT, 8),
                 true);
    forward_case("so8 split offgrid sources", g3, 24, scattered(g3, 40, 0, 21), Pts(), opts(FD_VARIANT_SPLIT, 17),
                 true);
    const fd_grid g16 = grid({48, 40, 46}, 16);
    forward_case("so16 stream", g16, 20, centre_src(g16, 12), rec_line(g16, 9, 12), opts(FD_VARIANT_STREAM), true);
    // two levels without redundant halos: counters, epochs, tails and routes
    forward_case("so8 wave", g3, 25, centre_src(g3, 12), rec_line(g3, 7, 12), opts(FD_VARIANT_WAVE), true);
    forward_case("so4 wave tile offgrid", g4, 33, scattered(g4, 3, 0, 22), scattered(g4, 20, 0, 23),
                 opts(FD_VARIANT_WAVE, 0, 16, 2), true);
    forward_case("so16 wave", g16, 20, centre_src(g16, 12), rec_line(g16, 9, 12), opts(FD_VARIANT_WAVE), true);
    forward_case("so8 wave sinc receivers", g3, 20, centre_src(g3, 12), scattered(g3, 30, 4, 24),
                 opts(FD_VARIANT_WAVE), false);
    const fd_grid g2 = grid({60, 70}, 4), g1 = grid({100}, 2, 0);
    forward_case("2-D so4", g2, 40, centre_src(g2, 20), rec_line(g2, 7, 5), opts(), true);
    forward_case("1-D so2", g1, 40, centre_src(g1, 30), Pts(), opts(), true);
    // anisotropic spacing
    fd_grid ga = grid({40, 38, 44}, 8);
    ga.h[1] = 12.5;
    forward_case("so8 anisotropic", ga, 20, centre_src(ga, 12), rec_line(ga, 7, 12), opts(FD_VARIANT_STREAM), true);
    // points between nodes: multilinear and windowed sinc, staged, routed and heavy tables
    forward_case("offgrid receivers", g3, 24, centre_src(g3, 12), scattered(g3, 40, 0, 1), opts(FD_VARIANT_STREAM),
                 false);
    forward_case("offgrid T2", g4, 24, scattered(g4, 3, 0, 2), scattered(g4, 90, 0, 3),
                 opts(FD_VARIANT_TBLOCK, 0, 0, 0, 2), false);
    forward_case("300 sources T2", g4, 24, scattered(g4, 300, 0, 4), rec_line(g4, 7, 15),
                 opts(FD_VARIANT_TBLOCK, 0, 0, 0, 2), false);
    forward_case("sinc source and receivers", g3, 20, scattered(g3, 1, 4, 5), scattered(g3, 30, 4, 6),
                 opts(FD_VARIANT_STREAM), false);
    forward_case("sinc 2-D", g2, 20, scattered(g2, 2, 3, 7), scattered(g2, 20, 8, 8), opts(), false);
    // the entry point without a workspace: twice, then a grid beyond its scratch
    noalloc_case("so8", g3, 24, centre_src(g3, 12), rec_line(g3, 7, 12), opts(FD_VARIANT_STREAM), FD_OK);
    noalloc_case("so4 smaller", g4, 20, centre_src(g4, 15), rec_line(g4, 7, 15), opts(), FD_OK);
    {
        const fd_grid big = grid({160, 160, 160}, 8);
        noalloc_case("too large", big, 4, centre_src(big, 12), Pts(), opts(), FD_ESCRATCH);
    }
    // seeded random draws over the planner's options (rank, ragged extents,
    // order, variant, tile, chunk, points on and between nodes, steps); a
    // draw whose kernel is not compiled returns FD_EUNSUPPORTED
    {
        uint32_t r = 12345u;
        auto rnd = [&r](int n) {
            r = r * 1664525u + 1013904223u;
            return (int)((r >> 8) % (uint32_t)n);
        };
        static const int shapes[][2] = {{4, 8}, {2, 16}, {4, 4}, {8, 4}, {16, 2}, {8, 2}, {2, 8}};
        static const int variants[] = {FD_VARIANT_STREAM, FD_VARIANT_TBLOCK, FD_VARIANT_SPLIT, FD_VARIANT_WAVE, 0};
        int ok = 0, unsupported = 0;
        for (int it = 0; it < 120; ++it) {
            const int nd = 1 + (rnd(6) < 4 ? 2 : rnd(2));
            const int so = 2 * (1 + rnd(8)), M = so / 2;
            std::vector<int> n;
            for (int a = 0; a < nd; ++a) n.push_back(2 * M + 1 + rnd(nd == 1 ? 250 : 60));
            fd_grid g = grid(n, so, rnd(3) == 0 ? 0 : 1 + rnd(std::max(1, n[0] / 4)));
            for (int a = 0; a < nd; ++a)
                if (2 * g.sponge > n[a]) g.sponge = 0;
            if (rnd(5) == 0) g.h[nd - 1] = 12.5;
            fd_options o = opts(variants[rnd(5)]);
            if (o.variant == FD_VARIANT_TBLOCK) o.tblock = 2 + rnd(3);
            if (o.variant && rnd(10) < 7) {
                static const int lxs[] = {0, 0, 7, 13, 32, 64};
                const int k = rnd(7);
                o.tile[0] = lxs[rnd(6)];
                o.tile[1] = shapes[k][0] * shapes[k][1];
                o.tile[2] = shapes[k][0];
            }
            const int64_t nt = 1 + rnd(40);
            const bool between = rnd(5) < 2;
            Pts src = between ? scattered(g, rnd(4), 0, 100 + it) : Pts();
            if (!between && rnd(2)) src = centre_src(g, n.back() / 2);
            Pts rec = (rnd(5) < 2) ? scattered(g, rnd(12), rnd(4) == 0 ? 2 : 0, 200 + it) : rec_line(g, 1 + rnd(9), 0);
            const fd_time t{nt, stable_dt(g)};
            const int64_t N = points(g);
            Buf v(N * 4), amp((size_t)nt * std::max(src.p.n, 1) * 4), out((size_t)nt * std::max(rec.p.n, 1) * 4),
                st(2 * N * 4);
            for (int64_t i = 0; i < N; ++i) v.f()[i] = 2000.0f;
            src.p.amp = amp.f();
            const size_t ws = fd_workspace_size(&g, &t, &src.p, &rec.p, &o, FD_OP_FORWARD);
            Buf w(ws);
            const int rc = fd_forward(&g, &t, v.f(), &src.p, &rec.p, rec.p.n ? out.f() : nullptr, st.f(), w.p, ws, &o,
                                      nullptr);
            if (rc == FD_OK) ++ok;
            else if (rc == FD_EUNSUPPORTED) ++unsupported;
            else expect(rc, FD_OK, "random draw " + std::to_string(it));
        }
        std::printf("random draws: %d ran, %d not compiled\n", ok, unsupported);
        expect(ok >= 60 ? FD_OK : -100, FD_OK, "random draws mostly compiled");
    }
    // an automatic plan whose cached exchange choice cannot be resident on this
    // device falls back to the default plan
    if (std::getenv("FD_AUTOTUNE_CACHE")) {
        const fd_time t{4, stable_dt(gbig)};
        const fd_options o = opts();
        const size_t ws = fd_workspace_size(&gbig, &t, nullptr, nullptr, &o, FD_OP_FORWARD);
        Buf w(ws), v(points(gbig) * 4), st(2 * points(gbig) * 4);
        for (int64_t i = 0; i < points(gbig); ++i) v.f()[i] = 2000.0f;
        expect(fd_forward(&gbig, &t, v.f(), nullptr, nullptr, nullptr, st.f(), w.p, ws, &o, nullptr), FD_OK,
               "automatic plan with an exchange choice that cannot be resident");
        fd_options last{};
        fd_last_config(&last);
        expect(last.variant == FD_VARIANT_STREAM ? FD_OK : -100, FD_OK, "it ran the space-tiled default");
        fd_options wv = opts(FD_VARIANT_WAVE);
        expect(fd_forward(&gbig, &t, v.f(), nullptr, nullptr, nullptr, st.f(), w.p, ws, &wv, nullptr),
               FD_EUNSUPPORTED, "an explicit exchange plan that cannot be resident");
    }
    // a pass without redundant halos whose wait ran out (forced by the
    // stand-in): the call reports FD_ESYNC; the next call on the same
    // workspace clears the error word before its first such pass
    {
        const fd_time t{21, stable_dt(g3)};
        const fd_options o = opts(FD_VARIANT_WAVE);
        const size_t ws = fd_workspace_size(&g3, &t, nullptr, nullptr, &o, FD_OP_FORWARD);
        Buf w(ws), v(points(g3) * 4), st(2 * points(g3) * 4);
        for (int64_t i = 0; i < points(g3); ++i) v.f()[i] = 2000.0f;
        hc_force_wave_timeout(1);
        expect(fd_forward(&g3, &t, v.f(), nullptr, nullptr, nullptr, st.f(), w.p, ws, &o, nullptr), FD_ESYNC,
               "wave pass whose wait ran out");
        hc_force_wave_timeout(0);
        expect(fd_forward(&g3, &t, v.f(), nullptr, nullptr, nullptr, st.f(), w.p, ws, &o, nullptr), FD_OK,
               "the next call clears the error word");
    }
    // adjoint, gradients (checkpointed and whole time axis), vjp, Born
    adjoint_case("so8", g3, 24, centre_src(g3, 12), rec_line(g3, 7, 12), opts(FD_VARIANT_STREAM));
    adjoint_case("so8 wave", g3, 25, centre_src(g3, 12), rec_line(g3, 7, 12), opts(FD_VARIANT_WAVE));
    adjoint_case("so4 T2 offgrid", g4, 24, scattered(g4, 2, 0, 9), scattered(g4, 30, 0, 10),
                 opts(FD_VARIANT_TBLOCK, 0, 0, 0, 2));
    gradient_case("so8 ckpt 7", g3, 30, centre_src(g3, 12), rec_line(g3, 7, 12), opts(FD_VARIANT_STREAM, 0, 0, 0, 0, 0, 7),
                  false);
    gradient_case("so8 wave ckpt 7", g3, 30, centre_src(g3, 12), rec_line(g3, 7, 12),
                  opts(FD_VARIANT_WAVE, 0, 0, 0, 0, 0, 7), false);
    gradient_case("so8 full", g3, 30, centre_src(g3, 12), rec_line(g3, 7, 12),
                  opts(FD_VARIANT_STREAM, 0, 0, 0, 0, 0, 30), false);
    gradient_case("so4 T2 ckpt 11", g4, 33, centre_src(g4, 15), rec_line(g4, 7, 15),
                  opts(FD_VARIANT_TBLOCK, 0, 0, 0, 2, 0, 11), false);
    gradient_case("sinc", g3, 20, scattered(g3, 1, 4, 11), scattered(g3, 30, 4, 12), opts(FD_VARIANT_STREAM, 0, 0, 0, 0, 0, 6),
                  false);
    gradient_case("naive", g3, 20, centre_src(g3, 12), rec_line(g3, 7, 12), opts(FD_VARIANT_NAIVE, 0, 0, 0, 0, 0, 6),
                  false);
    gradient_case("vjp so8", g3, 20, centre_src(g3, 12), rec_line(g3, 7, 12), opts(FD_VARIANT_STREAM, 0, 0, 0, 0, 0, 8),
                  true);
    born_case("so8 fused", g3, 20, centre_src(g3, 12), rec_line(g3, 7, 12), opts(FD_VARIANT_STREAM));
    born_case("so16 two passes", g16, 16, centre_src(g16, 12), rec_line(g16, 9, 12), opts(FD_VARIANT_STREAM));
    born_case("so8 offgrid", g3, 20, scattered(g3, 1, 0, 13), scattered(g3, 20, 0, 14), opts(FD_VARIANT_STREAM));
    // autotuner
    {
        const fd_grid ag = grid({40, 38, 44}, 8);
        fd_time t{8, stable_dt(ag)};
        fd_options o = opts();
        const size_t ws = fd_workspace_size(&ag, &t, nullptr, nullptr, nullptr, FD_OP_FORWARD);
        Buf w(ws);
        expect(fd_autotune(&ag, &t, &o, w.p, ws, nullptr), FD_OK, "autotune so8");
    }
    // batches: uneven grids, mixed orders, time blocks; graph and direct issue
    const std::vector<ShotSpec> mix = {
        {{40, 38, 44}, 4, 30, opts()},
        {{36, 44, 52}, 8, 25, opts()},
        {{48, 40, 46}, 16, 20, opts()},
        {{60, 70}, 4, 40, opts()},
        {{44, 40, 50}, 8, 27, opts(FD_VARIANT_TBLOCK, 0, 0, 0, 2)},
        {{42, 37, 45}, 4, 33, opts(FD_VARIANT_TBLOCK, 0, 32, 4, 3)},
        {{44, 40, 50}, 8, 21, opts(FD_VARIANT_WAVE)},
    };
    for (uint32_t bf : {0u, (uint32_t)FD_BATCH_GRAPH}) {
        batch_case(bf ? "graph" : "direct", mix, false, bf, 0);
        std::vector<ShotSpec> gmix = mix;
        for (auto &s : gmix) s.o.ckpt_every = 11;
        batch_case(bf ? "graph" : "direct", gmix, true, bf, 0);
    }
    // the batch tuner on the mixed batch (automatic shots tuned per class)
    {
        std::vector<fd_shot> shots(mix.size());
        std::vector<Pts> srcs;
        std::vector<Buf *> bufs;
        srcs.reserve(mix.size());
        for (size_t i = 0; i < mix.size(); ++i) {
            fd_shot &sh = shots[i];
            std::memset(&sh, 0, sizeof sh);
            sh.grid = grid(mix[i].n, mix[i].so);
            sh.time = fd_time{mix[i].nt, stable_dt(sh.grid)};
            Buf *v = new Buf(points(sh.grid) * 4);
            for (int64_t k = 0; k < points(sh.grid); ++k) v->f()[k] = 2000.0f;
            Buf *amp = new Buf((size_t)mix[i].nt * 4);
            bufs.push_back(v);
            bufs.push_back(amp);
            sh.v = v->f();
            srcs.push_back(centre_src(sh.grid, mix[i].n.back() / 3));
            srcs.back().p.amp = amp->f();
            sh.src = srcs.back().p;
            sh.opts = mix[i].o;
        }
        const size_t ws = fd_batch_workspace_size((int)shots.size(), shots.data(), FD_OP_FORWARD);
        Buf w(ws);
        expect(fd_batch_autotune((int)shots.size(), shots.data(), w.p, ws, nullptr), FD_OK, "batch autotune");
        for (size_t i = 0; i < shots.size(); ++i)
            if (mix[i].o.variant == 0 && (shots[i].opts.variant < FD_VARIANT_STREAM || shots[i].opts.tile[2] <= 0))
                expect(-100, FD_OK, "batch autotune sets the options of automatic shots");
        for (Buf *b : bufs) delete b;
    }
    const std::vector<ShotSpec> three = {
        {{40, 38, 44}, 4, 24, opts()}, {{36, 44, 52}, 8, 21, opts()}, {{48, 40, 46}, 16, 18, opts()}};
    for (uint32_t f : {0u, (uint32_t)FD_FLAG_LOADS_STREAM, (uint32_t)FD_FLAG_LOADS_KEEP})
        batch_case("three orders flags " + std::to_string(f), three, false, FD_BATCH_GRAPH, f);
    // the GPU suite's order: graph batches under both load policies, then the
    // mixed batch issued directly and with a graph, three times over (the
    // lane pool and its streams carry over from call to call)
    for (int rep = 0; rep < 3; ++rep) {
        for (uint32_t f : {(uint32_t)FD_FLAG_LOADS_STREAM, (uint32_t)FD_FLAG_LOADS_KEEP})
            batch_case("sequence flags " + std::to_string(f), three, false, FD_BATCH_GRAPH, f);
        batch_case("sequence direct", mix, false, 0, 0);
        batch_case("sequence graph", mix, false, FD_BATCH_GRAPH, 0);
    }
    // error paths
    {
        const fd_time t{10, stable_dt(g3)};
        Buf v(points(g3) * 4);
        fd_options o = opts();
        const size_t ws = fd_workspace_size(&g3, &t, nullptr, nullptr, &o, FD_OP_FORWARD);
        Buf w(ws);
        expect(fd_forward(&g3, &t, v.f(), nullptr, nullptr, nullptr, nullptr, w.p, ws - 256, &o, nullptr),
               FD_EWORKSPACE, "forward small workspace");
        expect(fd_forward(nullptr, &t, v.f(), nullptr, nullptr, nullptr, nullptr, w.p, ws, &o, nullptr), FD_EINVAL,
               "forward null grid");
        fd_options bad = opts(FD_VARIANT_TBLOCK, 0, 0, 0, 9);
        expect(fd_forward(&g3, &t, v.f(), nullptr, nullptr, nullptr, nullptr, w.p, ws, &bad, nullptr), FD_EINVAL,
               "forward tblock 9");
        Pts out = centre_src(g3, 60);
        Buf amp(10 * 4);
        out.p.amp = amp.f();
        expect(fd_forward(&g3, &t, v.f(), &out.p, nullptr, nullptr, nullptr, w.p, ws, &o, nullptr), FD_EDOM,
               "forward source outside");
    }
    long launches, checked, grouped, graphs;
    hc_stats(&launches, &checked, &grouped, &graphs);
    std::printf("launches %ld, sweep launches checked %ld, grouped %ld, graph launches %ld\n", launches, checked,
                grouped, graphs);
    std::printf("live events and graphs %d, live streams %d\n", hc_live_handles(), hc_live_streams());
    std::printf("hostcheck errors %d warnings %d, unexpected status %d\n", hc_errors(), hc_warnings(), g_bad);
    return (hc_errors() || g_bad || hc_live_handles()) ? 1 : 0;
}
