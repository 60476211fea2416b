// Solver drivers of libwdirac.
//
//  * eo_solve  : single-mass BiCGstab on the even-odd preconditioned system (Sec. 6.2.3, eq.
//                eo2-eo4) for one or many systems at once. With mixed precision the Krylov vectors
//                are stored in FP32 or FP16 and the operator uses FP16/BF16/FP32 12-real links;
//                FP64 reliable updates (x_hi += x_lo, r = b_prec - M_prec x_hi in FP64) keep the
//                true residual in step.
//  * ms_solve  : BiCGstab-M (Sec. 6.1), FP64, full lattice; with one mass it is plain BiCGstab.
//  * multimass : heaviest mass first, polynomial start guess (Sec. 6.2.1, Sec. 7).
//
// All kernels of an iteration are queued without host round trips: the BiCGstab scalars live on
// the device and each kernel skips systems that are no longer RUNNING. The host reads the
// per-system status every `poll` iterations and performs reliable updates, restarts and
// convergence checks.
#include <algorithm>
#include <type_traits>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <sys/stat.h>

#include "wd_host.hpp"

namespace wd {

static double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------- HIP graphs
// A chunk of `poll` solver iterations is captured once per solve on a private stream and replayed
// with hipGraphLaunch on the caller's stream. The captured kernels read only device-resident job
// tables and scalars, so every replay continues from the current device state. Per-kernel timing
// needs one event pair per launch, so graphs are not used while it is on.
static bool g_graphs = false;

struct ChunkGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    template <class F>
    void capture(F&& body)
    {
        WD_CHECK_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        WD_CHECK_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        body(cap);
        WD_CHECK_HIP(hipStreamEndCapture(cap, &graph));
        WD_CHECK_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    }
    void launch(hipStream_t st) { WD_CHECK_HIP(hipGraphLaunch(exec, st)); }
    ~ChunkGraph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

// A captured chunk is replayed by later solves whose launches are identical: the same kernels
// with the same arguments (table and state buffers are kept by the handle, so their addresses
// repeat) and grid sizes. The key lists all of them; the tables' contents (masses, fields) are
// read by the kernels at run time.
template <class... T>
static std::string launch_key(const char* kind, int a, int b, int c, SysState* sys, const T&... tabs)
{
    std::string k = std::string(kind) + "|" + std::to_string(a) + "|" + std::to_string(b) + "|" + std::to_string(c) + "|" +
                    std::to_string((uintptr_t)sys);
    auto add = [&](const auto& t) {
        int tg = 0;
        if constexpr (std::is_same_v<std::decay_t<decltype(t)>, JobTable<HopJob>>)
            for (auto& j : t.host) tg |= j.tg;
        k += "|" + std::to_string((uintptr_t)t.d()) + ":" + std::to_string(t.nblocks) + ":" + std::to_string(t.n()) +
             ":" + std::to_string(tg);
    };
    (add(tabs), ...);
    return k;
}

template <class F>
static std::shared_ptr<ChunkGraph> cached_graph(wd_gauge* g, const std::string& key, F&& body)
{
    auto& slot = g->graphs[key];
    if (!slot) {
        if (g->graphs.size() > 32) {  // bound the cache; keep the entry being made
            g->graphs.clear();
            return cached_graph(g, key, body);
        }
        auto gp = std::make_shared<ChunkGraph>();
        gp->capture(body);
        slot = gp;
    }
    return std::static_pointer_cast<ChunkGraph>(slot);
}

void set_graphs(bool on) { g_graphs = on; }
bool graphs_on() { return g_graphs && !timer().on; }

static double spinor_site_bytes(int sf) { return sf == SF64 ? 192.0 : sf == SF32 ? 96.0 : 52.0; }
static double link_site_bytes(int lf) { return 8.0 * link_chunks(lf) * link_chunk_bytes(lf); }

// ---------------------------------------------------------------- device system records
struct SysArray {
    std::shared_ptr<DevMem> dev;
    std::vector<SysState> h;
    // cache: a buffer kept by a gauge handle across solves (grown when too small)
    void alloc(int n, std::shared_ptr<DevMem>& cache)
    {
        h.assign(n, SysState{});
        if (!cache || cache->bytes < sizeof(SysState) * n) cache = std::make_shared<DevMem>(sizeof(SysState) * n);
        dev = cache;
    }
    SysState* d() const { return (SysState*)dev->p; }
    void upload(hipStream_t s)
    {
        size_t n = sizeof(SysState) * h.size();
        char* st = stage_alloc(n);
        std::memcpy(st, h.data(), n);
        WD_CHECK_HIP(hipMemcpyAsync(dev->p, st, n, hipMemcpyHostToDevice, s));
    }
    void download(hipStream_t s)
    {
        size_t n = sizeof(SysState) * h.size();
        void* st = pinned(n);
        WD_CHECK_HIP(hipMemcpyAsync(st, dev->p, n, hipMemcpyDeviceToHost, s));
        WD_CHECK_HIP(hipStreamSynchronize(s));
        std::memcpy(h.data(), st, n);
    }
};

static inline int nblk(long n) { return (int)((n + BLOCK - 1) / BLOCK); }

// ---------------------------------------------------------------- hop autotuner
// For the hops of one handle in a launch in which nshared systems read its links, the tuner picks
// the block order (site order, tz = 0, or t fastest within groups of tz z-planes) and the way the
// systems share the link loads (rhs = 0: one system per thread, systems sharing links in
// interleaved block pairs; rhs = k >= 2: the multi-RHS hop, k systems per thread). Every candidate
// is timed on the handle's lattice with min(nshared, 4) systems in the solver's storage formats,
// each candidate's best of three interleaved passes counts. The choice is kept per (device
// architecture, lattice extents, formats, temporal gauge, systems) for the process and in a text
// file ($WD_TUNE_CACHE, else $HOME/.cache/wdirac/hop_tune.txt) that later processes read first.
struct HopChoice {
    int tz = 0;
    int rhs = 0;
};

static std::string arch_name()
{
    static const std::string a = [] {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return std::string("unknown");
        const std::string s(p.gcnArchName);
        return s.substr(0, s.find(':'));
    }();
    return a;
}

static std::string tune_path()
{
    if (const char* e = std::getenv("WD_TUNE_CACHE")) return e;
    const char* h = std::getenv("HOME");
    return h ? std::string(h) + "/.cache/wdirac/hop_tune.txt" : std::string();
}

static std::map<std::string, HopChoice>& tune_cache()
{
    static std::map<std::string, HopChoice> c;
    static bool loaded = false;
    if (!loaded) {
        loaded = true;
        const std::string path = tune_path();
        if (FILE* f = path.empty() ? nullptr : std::fopen(path.c_str(), "r")) {
            char key[256];
            int tz, rhs;
            while (std::fscanf(f, "%255s %d %d", key, &tz, &rhs) == 3) c[key] = HopChoice{tz, rhs};
            std::fclose(f);
        }
    }
    return c;
}

static void tune_store(const std::string& key, HopChoice ch)
{
    tune_cache()[key] = ch;
    const std::string path = tune_path();
    if (path.empty()) return;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) {
        // create the directory and its parent if missing (errors are ignored: the file is a cache)
        const std::string dir = path.substr(0, slash);
        const size_t up = dir.rfind('/');
        if (up != std::string::npos && up > 0) (void)mkdir(dir.substr(0, up).c_str(), 0755);
        (void)mkdir(dir.c_str(), 0755);
    }
    if (FILE* f = std::fopen(path.c_str(), "a")) {
        std::fprintf(f, "%s %d %d\n", key.c_str(), ch.tz, ch.rhs);
        std::fclose(f);
    }
}

static bool tile_valid(const Geo& g, int tz)
{
    if (tz == 0) return true;
    return tz > 0 && (g.Xh * g.Y) % BLOCK == 0 && g.Z % tz == 0 && g.Vh % BLOCK == 0;
}

static void set_tile(HopJob& j, int tz)
{
    if (!tile_valid(j.g, tz)) tz = 0;
    j.tz = tz;
    j.bpp = tz > 0 ? j.g.Xh * j.g.Y / BLOCK : 0;
}

static HopJob hop_job(const Geo& g, int parity, int sys, const SpinorRef& in, const SpinorRef& out,
                      const void* links, long lcs, double c2);
template <class J> static void layout(JobTable<J>& t);

// The link-load policy a launch of this handle's hops takes (run_hop): non-temporal unless systems
// of the launch share the links through L2 (interleaved) or the links are small enough to stay
// in the Infinity Cache. The block order is tuned for that policy.
static int link_policy(wd_gauge* g, int lf, bool shared)
{
    const double bytes = (double)g->geo.Vh * 8 * link_chunks(lf) * link_chunk_bytes(lf);
    return !shared && bytes > 64.0 * (1 << 20);
}

HopChoice tune_hop(wd_gauge* g, int sf, int lf, hipStream_t st, int nshared)
{
    const Geo& G = g->geo;
    const int nc = std::max(1, std::min(nshared, 4));
    std::vector<HopChoice> cands;
    for (int rhs : {0, 2, 4}) {
        if (rhs > 0 && (sf == SF64 || nc < 2 || (rhs == 4 && nc < 3))) continue;
        for (int tz : {0, 2, 4, 8, 16})
            if (tile_valid(G, tz)) cands.push_back(HopChoice{tz, rhs});
    }
    if (cands.size() == 1) return cands[0];
    char key[160];
    std::snprintf(key, sizeof(key), "%s|%dx%dx%dx%d|sf%d|lf%d|tg%d|n%d", arch_name().c_str(), G.X, G.Y, G.Z, G.T, sf, lf,
                  (int)g->tg, nc);
    // a cached choice counts only if it is one of this configuration's candidates (the file may be
    // stale or edited by hand)
    auto it = tune_cache().find(key);
    if (it != tune_cache().end())
        for (const HopChoice& c : cands)
            if (c.tz == it->second.tz && c.rhs == it->second.rhs) return c;
    g->ensure_slinks(lf, st);
    std::vector<Field> in(nc), out(nc);
    for (int k = 0; k < nc; k++) {
        in[k] = g->field("tune.in" + std::to_string(k), sf, 1);
        out[k] = g->field("tune.out" + std::to_string(k), sf, 1);
    }
    SysState* dummy = (SysState*)g->rawbuf("tune.sys", sizeof(SysState) * nc);
    const int ntl = link_policy(g, lf, nc > 1);
    std::vector<JobTable<HopJob>> tabs(cands.size());
    for (size_t c = 0; c < cands.size(); c++) {
        for (int k = 0; k < nc; k++) {
            HopJob j = hop_job(G, 1, k, in[k].all(), out[k].all(), g->slk(lf, 1), g->lcs(), 1.0);
            j.tg = g->tg;
            j.nc = g->nc;
            j.rhs = cands[c].rhs;
            set_tile(j, cands[c].tz);
            tabs[c].host.push_back(j);
        }
        layout(tabs[c]);
        tabs[c].upload(st);
    }
    auto launch = [&](const JobTable<HopJob>& t) {
        if (t.host[0].rhs >= 2) {
            int kmax = 1;
            for (auto& j : t.host) kmax = std::max(kmax, j.ilv);
            WD_CHECK_HIP(launch_hop_mrhs(sf, lf, false, RED_NONE, mrhs_kt(kmax), t.d(), t.n(), t.nblocks, dummy, 0, st));
        } else {
            WD_CHECK_HIP(launch_hop(sf, lf, false, RED_NONE, FIN_STORE, t.d(), t.n(), t.nblocks, dummy, 0, st, nullptr, -1,
                                    t.host[0].tg, ntl));
        }
    };
    hipEvent_t e0, e1;  // timing only: no system-scope fence (L2 writeback and invalidate)
    WD_CHECK_HIP(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
    WD_CHECK_HIP(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
    // three interleaved passes over the candidates, each candidate's best pass counts (a single
    // pass let the clock and cache state of the moment decide within a few %)
    std::vector<float> cand_ms(cands.size(), 1e30f);
    for (int pass = 0; pass < 3; pass++)
        for (size_t c = 0; c < cands.size(); c++) {
            launch(tabs[c]);
            WD_CHECK_HIP(hipEventRecord(e0, st));
            for (int w = 0; w < 4; w++) launch(tabs[c]);
            WD_CHECK_HIP(hipEventRecord(e1, st));
            WD_CHECK_HIP(hipEventSynchronize(e1));
            float ms = 0;
            WD_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
            cand_ms[c] = std::min(cand_ms[c], ms / (4.0f * nc));
        }
    size_t best = 0;
    for (size_t c = 1; c < cands.size(); c++)
        if (cand_ms[c] < cand_ms[best]) best = c;
    WD_CHECK_HIP(hipEventDestroy(e0));
    WD_CHECK_HIP(hipEventDestroy(e1));
    if (std::getenv("WD_VERBOSE")) {
        for (size_t c = 0; c < cands.size(); c++)
            std::fprintf(stderr, "wdirac: tune %s: tz=%d rhs=%d %.1f us per system-hop\n", key, cands[c].tz, cands[c].rhs,
                         cand_ms[c] * 1e3);
        std::fprintf(stderr, "wdirac: tune %s: chose tz=%d rhs=%d\n", key, cands[best].tz, cands[best].rhs);
    }
    for (int k = 0; k < nc; k++) {
        g->ws.erase("tune.in" + std::to_string(k));
        g->ws.erase("tune.out" + std::to_string(k));
    }
    tune_store(key, cands[best]);
    return cands[best];
}

// block order alone, for launches in which the handle's links are not shared (or interleaved pairs)
int tune_tile(wd_gauge* g, int sf, int lf, hipStream_t st, bool shared = false)
{
    return tune_hop(g, sf, lf, st, shared ? 2 : 1).tz;
}

static HopJob hop_job(const Geo& g, int parity, int sys, const SpinorRef& in, const SpinorRef& out,
                      const void* links, long lcs, double c2)
{
    HopJob j;
    std::memset(&j, 0, sizeof(j));
    j.g = g;
    j.parity = parity;
    j.sys = sys;
    j.in = in;
    j.out = out;
    j.links = links;
    j.lcs = lcs;
    j.c2 = c2;
    j.nblk = nblk(g.Vh);
    return j;
}

// Hop jobs that share their links (same gauge field and parity) run in interleaved block groups of
// at most kIlvMax systems: pairs share the link loads while the neighbour spinors of both still fit
// the L2 reuse window. Measured at 32^3x64 with 8 systems (FP16 links, FP32 spinors): pairs at
// their best block order (tz = 16) 585 us per hop and 57.3 ms per 8-mass solve, groups of 4 at
// theirs (tz = 8) 573 us and 56.6 ms, groups of 3 (3 + 3 + 2) at tz = 8 622 us and 59.3 ms. The
// 1% that groups of 4 gain needs a block order of their own, so pairs stay.
constexpr int kIlvMax = 2;
static bool interleave_on() { return true; }
static int interleave_max() { return kIlvMax; }

static bool same_links(const HopJob& a, const HopJob& b)
{
    return a.links == b.links && a.parity == b.parity && a.g.Vh == b.g.Vh && a.g.X == b.g.X && a.g.Y == b.g.Y &&
           a.g.Z == b.g.Z && a.g.T == b.g.T && a.nblk == b.nblk && a.tz == b.tz && a.bpp == b.bpp && a.rhs == b.rhs &&
           a.tg == b.tg && a.lcs == b.lcs;
}
static bool same_links(const SweepJob&, const SweepJob&) { return false; }
// largest group of jobs sharing links: rhs systems per thread for the multi-RHS hop, else kIlvMax
static int group_max(const HopJob& j) { return j.rhs >= 2 ? j.rhs : interleave_max(); }
static int group_max(const SweepJob&) { return 1; }
static int group_blocks(const HopJob& j, int K) { return j.rhs >= 2 ? j.nblk : K * j.nblk; }
static int group_blocks(const SweepJob& j, int K) { return K * j.nblk; }
static void set_group(HopJob& j, int k, int pos)
{
    j.ilv = k;
    j.ilv_pos = pos;
}
static void set_group(SweepJob&, int, int) {}

// Assign block ranges; jobs with the same sys form one reduction group. Consecutive hop jobs
// that read the same links form an interleaved group (at most interleave_max() jobs).
template <class J>
static void layout(JobTable<J>& t)
{
    int b = 0;
    std::map<int, int> group;
    const size_t n = t.host.size();
    for (size_t i = 0; i < n;) {
        size_t k = i + 1;
        if (interleave_on())
            while (k < n && (int)(k - i) < group_max(t.host[i]) && same_links(t.host[i], t.host[k])) k++;
        const int K = (int)(k - i);
        for (size_t m = i; m < k; m++) {
            J& j = t.host[m];
            j.blk0 = b;
            set_group(j, K, (int)(m - i));
            j.rblk0 = group[j.sys];
            group[j.sys] += j.nblk;
        }
        b += group_blocks(t.host[i], K);
        i = k;
    }
    for (auto& j : t.host) j.rnblk = group[j.sys];
    t.nblocks = b;
}

static SweepJob sweep_job(int sys, long n)
{
    SweepJob j;
    std::memset(&j, 0, sizeof(j));
    j.sys = sys;
    j.n = (int)n;
    j.nblk = nblk(n);
    return j;
}

// Compulsory bytes of a hop launch: every job's spinors; the links once per interleaved group,
// in temporal gauge without the unit time links (loaded on the sites of time slices 0 and T - 1)
static double hop_bytes(const JobTable<HopJob>& t, int sf, int lf, int extra_fields)
{
    double n = 0, nl = 0;
    for (auto& j : t.host) {
        n += (double)j.g.Vh;
        const double frac = j.tg ? 0.75 + 0.25 * (j.g.T > 2 ? 2.0 / j.g.T : 1.0) : 1.0;
        if (j.ilv <= 1 || j.ilv_pos == 0) nl += (double)j.g.Vh * frac;
    }
    return n * (2 + extra_fields) * spinor_site_bytes(sf) + nl * link_site_bytes(lf);
}
// Compulsory bytes of an OP_INIT launch, per job from its flags: r_hi read (FP64), r_lo written,
// rhat written (flags 1) or read (when it is a field of its own: CG passes r_lo), s written
// (flags 2), p read and written (flags 8), x_lo cleared (flags 4; FP32 storage for the 16-bit
// formats)
static double init_bytes(const JobTable<SweepJob>& t, int sfl)
{
    const double bl = spinor_site_bytes(sfl), bx = spinor_site_bytes(sfl == SF64 ? SF64 : SF32);
    double n = 0;
    for (auto& j : t.host) {
        double b = spinor_site_bytes(SF64) + bl;
        if ((j.flags & 1) || j.f[R_F2].p != j.f[R_F0].p) b += bl;
        if (j.flags & 2) b += bl;
        if (j.flags & 8) b += 2 * bl;
        if (j.flags & 4) b += bx;
        n += (double)j.n * b;
    }
    return n;
}
static double sweep_bytes(const JobTable<SweepJob>& t, double per_site)
{
    double n = 0;
    for (auto& j : t.host) n += (double)j.n;
    return n * per_site;
}

// Jobs that read the same links made consecutive (stable in the systems' order), so that layout()
// can group them; one job per system and table, so reduction groups are unaffected.
static void group_by_links(JobTable<HopJob>& t)
{
    std::stable_sort(t.host.begin(), t.host.end(), [](const HopJob& a, const HopJob& b) {
        return a.links != b.links ? (uintptr_t)a.links < (uintptr_t)b.links : a.parity < b.parity;
    });
}

// Tuned hop choices for a batch of systems: per system the block orders of its handle (low
// precision, FP64) for the number of systems in the batch that share the handle's links, and one
// multi-RHS mode for the low-precision launches (a launch runs a single kernel): the mode tuned for
// the handle that carries the most work.
template <class Sys>
static int tune_shared_hops(const std::vector<Sys>& S, int SFL, int LFL, int L64, hipStream_t st, std::vector<int>& tile_lo,
                            std::vector<int>& tile_64)
{
    const int n = (int)S.size();
    std::map<wd_gauge*, int> count;
    for (auto& e : S) count[e.g]++;
    int rhs = 0;
    double most = -1;
    for (int i = 0; i < n; i++) {
        const int c = interleave_on() ? count[S[i].g] : 1;
        const HopChoice lo = tune_hop(S[i].g, SFL, LFL, st, c);
        tile_lo[i] = lo.tz;
        tile_64[i] = tune_hop(S[i].g, SF64, L64, st, c).tz;
        const double work = (double)S[i].g->geo.Vh * c;
        if (work > most) {
            most = work;
            rhs = lo.rhs;
        }
    }
    return rhs;
}

// ================================================================ even-odd BiCGstab (batched)

// A packed source: b in the internal layout, h = 1/2 D_eo b_o (independent of the mass, so a
// multi-mass solve computes it once) and |b|^2.
struct EoSource {
    Field B64, HB;
    double bb = -1;
};

struct EoSys {
    wd_gauge* g;
    double kappa, a;
    const double* b;
    double* x;
    int slot;
    EoSource src;      // prepared by the caller, or built here
    Field X64;         // FP64 solution (even half iterated, odd half rebuilt); caller-provided or own
    bool x_ready = false;  // X64 already holds the start vector (use_x0 handled by the caller)
    bool r_ready = false;  // RH already holds b_prec - M_prec x0 for that start vector (one system only)
    bool keep_odd = false; // store the rebuilt odd half into X64 as well (a later guess reads it)
    bool bp_ready = false; // BP (caller-provided) already holds b_prec (one system only)
    Field RH;              // FP64 residual b_prec - M_prec x_e; caller-provided or own
    Field BP, T64;
    Field r, rh, s, w, As, Aw, tmp, xl;
    bool done = false;
    int restarts = 0, reliable = 0;
    int final_status = WD_OK;
    int iters = 0;
    double rr_true = -1;   // |r_prec|^2 of the last FP64 residual
    double true_rel = 0;
    double t0 = 0, t1 = 0;
};

static void prepare_source(wd_gauge* g, const std::string& key, const double* b, int dagger, EoSource& src,
                           hipStream_t st)
{
    src.B64 = g->field(key + "B64", SF64, 2);
    src.HB = g->field(key + "HB", SF64, 1);
    WD_CHECK_HIP(launch_pack_spinor(SF64, b, g->geo, src.B64.half(0), src.B64.half(1), dagger, 1.0, st, g->gm(), g->nc));
    src.bb = -1;
}

// Iterations queued between host checks of the systems' status in the even-odd solver (measured
// best of 2/3/4/6/8 at 16^3x32 and 32^3x64: fewer means more round trips, more means more gated
// launches after a system has stopped).
constexpr int kPoll = 3;

static void eo_solve(std::vector<EoSys>& S, const wd_solver_params& P, hipStream_t st, int poll)
{
    const int n = (int)S.size();
    const int SFL = P.mixed ? spinor_fmt_of(P.spinor_store) : SF64;
    const int SFX = SFL == SF64 ? SF64 : SF32;
    // the FP64 operator (b_prec, reliable updates, eq. eo3) uses 12-real links when every handle's
    // links are SU(3) to rounding; the iteration uses the low-precision format
    int L64 = L64_12;
    for (auto& e : S)
        if (e.g->f64_links() != L64_12) L64 = L64_18;
    const int LFL = P.mixed ? link_fmt_of(P.link_store, P.recon) : L64;
    if (P.mixed && link_recon12(LFL))
        for (auto& e : S)
            if (e.g->recon_err > 1e-6)
                throw Error{WD_ERR_UNSUPPORTED, "links are not SU(3): the 12-real low-precision formats would change "
                                                "the operator; solve with mixed = 0"};
    const double t_start = now_s();

    // systems on the same gauge field share link loads (multi-RHS hop or interleaved block pairs)
    std::vector<int> tile_lo(n), tile_64(n);
    const int rhs_lo = tune_shared_hops(S, SFL, LFL, L64, st, tile_lo, tile_64);
    for (auto& e : S) {
        e.g->ensure_slinks(LFL, st);
        e.g->ensure_slinks(L64, st);
        const std::string k = "eo" + std::to_string(e.slot) + ".";
        if (!e.src.B64.mem) prepare_source(e.g, k, e.b, P.dagger, e.src, st);
        if (!e.X64.mem) e.X64 = e.g->field(k + "X64", SF64, 2);
        if (!e.BP.mem) e.BP = e.g->field(k + "BP", SF64, 1);
        if (!e.RH.mem) e.RH = e.g->field(k + "RH", SF64, 1);
        e.T64 = e.g->field(k + "T64", SF64, 1);
        e.r = e.g->field(k + "r", SFL, 1);
        e.rh = e.g->field(k + "rh", SFL, 1);
        e.s = e.g->field(k + "s", SFL, 1);
        e.w = e.g->field(k + "w", SFL, 1);
        e.As = e.g->field(k + "As", SFL, 1);
        e.Aw = e.g->field(k + "Aw", SFL, 1);
        e.tmp = e.g->field(k + "tmp", SFL, 1);
        e.xl = e.g->field(k + "xl", SFX, 1);
        e.a = 1.0 / (2.0 * e.kappa);
    }

    SysArray sys;
    sys.alloc(n, S[0].g->raw["eo.sys"]);
    for (int i = 0; i < n; i++) {
        EoSys& e = S[i];
        SysState& q = sys.h[i];
        std::memset(&q, 0, sizeof(q));
        q.partials = (double*)e.g->rawbuf("eo" + std::to_string(e.slot) + ".partials",
                                          sizeof(double) * NRED * (2 * e.g->geo.stride / BLOCK + 1));
        q.maxit = P.max_iter;
        q.mixed = P.mixed;
        q.delta_rel2 = P.delta_reliable * P.delta_reliable;
        q.dc = P.mixed && P.mixed_mode == WD_MIXED_DEFECT;
        q.target2 = -1.0;
        q.status = ST_RUNNING;
    }
    sys.upload(st);

    // ---- static job tables
    JobTable<HopJob> Hhb, Hx1, Hx2, Hrec;
    JobTable<SweepJob> Nb, Bp, InitFirst, InitRel, InitRestart, Acc;
    JobTable<HopJob> H1, H2, H3, H4;
    JobTable<SweepJob> SW, SXR, SS;
    std::vector<int> need_src;
    for (int i = 0; i < n; i++) {
        EoSys& e = S[i];
        const Geo& g = e.g->geo;
        const void* d0 = e.g->slk(L64, 0);
        const void* d1 = e.g->slk(L64, 1);
        const long lcs = e.g->lcs();
        bool shared = false;  // another system of this solve already prepares the same source
        for (int k = 0; k < i; k++) shared = shared || S[k].src.B64.base() == e.src.B64.base();
        if (e.src.bb < 0 && !shared) {
            need_src.push_back(i);
            // h = 1/2 D_eo b_o ; |b|^2
            Hhb.host.push_back(hop_job(g, 0, i, e.src.B64.half(1), e.src.HB.all(), d0, lcs, 0.5));
            SweepJob nj = sweep_job(i, e.src.B64.nsites());
            nj.f[R_F0] = e.src.B64.all();
            Nb.host.push_back(nj);
        }
        // b_prec = a b_e + 1/2 D_eo b_o  (eq. eo4)
        SweepJob bj = sweep_job(i, e.BP.nsites());
        bj.f[R_F0] = e.BP.all();
        bj.f[R_F1] = e.src.B64.half(0);
        bj.f[R_F2] = e.src.HB.all();
        bj.c[0] = e.a;
        bj.c[1] = 1.0;
        Bp.host.push_back(bj);
        // FP64 residual r_hi = b_prec - M_prec x_e: T64 = D_oe x_e ; RH = b_prec - a^2 x_e + 1/4 D_eo T64
        Hx1.host.push_back(hop_job(g, 1, i, e.X64.half(0), e.T64.all(), d1, lcs, 1.0));
        HopJob j = hop_job(g, 0, i, e.T64.all(), e.RH.all(), d0, lcs, 0.25);
        j.x0 = e.BP.all();
        j.c0 = 1.0;
        j.x1 = e.X64.half(0);
        j.c1 = -e.a * e.a;
        Hx2.host.push_back(j);
        // odd half: x_o = (b_o + 1/2 D_oe x_e) / a  (eq. eo3)
        j = hop_job(g, 1, i, e.X64.half(0), e.X64.half(1), d1, lcs, 0.5 / e.a);
        j.x0 = e.src.B64.half(1);
        j.c0 = 1.0 / e.a;
        Hrec.host.push_back(j);
        SweepJob sj = sweep_job(i, e.r.nsites());
        sj.f[R_F0] = e.r.all();
        sj.f[R_F1] = e.RH.all();
        sj.f[R_F2] = e.rh.all();
        sj.f[R_F3] = e.s.all();
        sj.f[R_F4] = e.xl.all();
        sj.flags = 1 | 2 | 4;
        InitFirst.host.push_back(sj);
        sj.flags = 0;
        InitRel.host.push_back(sj);
        sj.flags = 1 | 2;
        InitRestart.host.push_back(sj);
        sj = sweep_job(i, e.xl.nsites());
        sj.f[R_F0] = e.X64.half(0);
        sj.f[R_F1] = e.xl.all();
        sj.flags = 1;
        Acc.host.push_back(sj);
        // iteration: As = a^2 s - 1/4 D_eo D_oe s, <rhat, As>; w; Aw = M_prec w, <Aw, w>, |Aw|^2; x, r; s
        const void* l0 = e.g->slk(LFL, 0);
        const void* l1 = e.g->slk(LFL, 1);
        H1.host.push_back(hop_job(g, 1, i, e.s.all(), e.tmp.all(), l1, lcs, 1.0));
        j = hop_job(g, 0, i, e.tmp.all(), e.As.all(), l0, lcs, -0.25);
        j.x0 = e.s.all();
        j.c0 = e.a * e.a;
        j.z = e.rh.all();
        H2.host.push_back(j);
        H3.host.push_back(hop_job(g, 1, i, e.w.all(), e.tmp.all(), l1, lcs, 1.0));
        j = hop_job(g, 0, i, e.tmp.all(), e.Aw.all(), l0, lcs, -0.25);
        j.x0 = e.w.all();
        j.c0 = e.a * e.a;
        H4.host.push_back(j);
        sj = sweep_job(i, e.r.nsites());
        sj.f[R_F0] = e.w.all();
        sj.f[R_F1] = e.r.all();
        sj.f[R_F2] = e.As.all();
        sj.f[R_F3] = e.r.all();
        SW.host.push_back(sj);
        sj = sweep_job(i, e.r.nsites());
        sj.f[R_F0] = e.xl.all();
        sj.f[R_F1] = e.r.all();
        sj.f[R_F2] = e.s.all();
        sj.f[R_F3] = e.w.all();
        sj.f[R_F4] = e.Aw.all();
        sj.f[R_F5] = e.rh.all();
        sj.f[R_F6] = e.r.all();
        SXR.host.push_back(sj);
        sj = sweep_job(i, e.r.nsites());
        sj.f[R_F0] = e.s.all();
        sj.f[R_F1] = e.r.all();
        sj.f[R_F2] = e.As.all();
        sj.f[R_F3] = e.r.all();
        SS.host.push_back(sj);
    }
    for (auto* t : {&Hhb, &Hx1, &Hx2, &Hrec})
        for (auto& j : t->host) set_tile(j, tile_64[j.sys]);
    for (auto* t : {&H1, &H2, &H3, &H4})
        for (auto& j : t->host) {
            set_tile(j, tile_lo[j.sys]);
            j.rhs = rhs_lo;
        }
    for (auto* t : {&Hhb, &Hx1, &Hx2, &Hrec, &H1, &H2, &H3, &H4}) {
        for (auto& j : t->host) {
            j.tg = S[j.sys].g->tg;  // solver links of a temporal-gauge handle
            j.nc = S[j.sys].g->nc;  // and the handle's spin basis
        }
        group_by_links(*t);
        layout(*t);
    }
    for (auto* t : {&Nb, &Bp, &InitFirst, &InitRel, &InitRestart, &Acc, &SW, &SXR, &SS}) layout(*t);
    // one copy for all tables, into a buffer kept by the first handle across solves
    upload_tables(st, S[0].g->raw["eo.tables"],
                  {&Hhb, &Hx1, &Hx2, &Hrec, &H1, &H2, &H3, &H4, &Nb, &Bp, &InitFirst, &InitRel, &InitRestart, &Acc,
                   &SW, &SXR, &SS});

    // ---- setup
    if (!need_src.empty()) {
        run_hop(SF64, L64, false, RED_NONE, FIN_STORE, Hhb, sys.d(), 0, st, hop_bytes(Hhb, SF64, L64, 0));
        run_sweep(OP_NORM, SF64, Nb, sys.d(), 0, st, sweep_bytes(Nb, 192));
        sys.download(st);
        for (int i : need_src) S[i].src.bb = sys.h[i].red[2];
        for (int i = 0; i < n; i++)
            for (int k : need_src)
                if (S[i].src.bb < 0 && S[i].src.B64.base() == S[k].src.B64.base()) S[i].src.bb = S[k].src.bb;
    }
    bool any_x0 = false;
    for (auto& e : S) {
        any_x0 = any_x0 || e.x_ready || P.use_x0;
        if (e.x_ready) continue;
        if (P.use_x0)
            WD_CHECK_HIP(launch_pack_spinor(SF64, e.x, e.g->geo, e.X64.half(0), e.X64.half(1), P.dagger, 1.0, st,
                                            e.g->gm(), e.g->nc));
        else
            WD_CHECK_HIP(hipMemsetAsync(e.X64.base(), 0, e.X64.mem->bytes, st));
    }
    WD_REQUIRE(n == 1 || !(S[0].r_ready || S[0].bp_ready), "a prepared start is for single-system solves");
    if (!S[0].bp_ready) run_sweep(OP_AXPY, SF64, Bp, sys.d(), 0, st, sweep_bytes(Bp, 3 * 192));
    if (any_x0 && !S[0].r_ready) {
        // start vector: r_hi = b_prec - M_prec x0 (systems without one have x0 = 0 and get b_prec)
        run_hop(SF64, L64, false, RED_NONE, FIN_STORE, Hx1, sys.d(), 0, st, hop_bytes(Hx1, SF64, L64, 0));
        run_hop(SF64, L64, false, RED_NONE, FIN_STORE, Hx2, sys.d(), 0, st, hop_bytes(Hx2, SF64, L64, 2));
    }
    // no host round trip here: the targets need |b|^2 only (known), and the start residual's norm
    // comes with the first iteration's restart finisher
    for (int i = 0; i < n; i++) {
        EoSys& e = S[i];
        // |b_prec - M_prec x_e| < tol (1/(2 kappa)) |b| is |b - M x| < tol |b| (the odd residual vanishes)
        sys.h[i].target2 = P.tol * P.tol * e.a * e.a * e.src.bb;
        sys.h[i].status = ST_RUNNING;
        if (e.src.bb == 0.0) {  // zero source: x = 0 (also when a start vector was given)
            e.done = true;
            e.rr_true = 0;
            sys.h[i].status = ST_DONE;
            WD_CHECK_HIP(hipMemsetAsync(e.X64.base(), 0, e.X64.mem->bytes, st));
            WD_CHECK_HIP(hipMemsetAsync(e.T64.base(), 0, e.T64.mem->bytes, st));
        }
    }
    sys.upload(st);
    if (!any_x0) {
        for (auto& j : InitFirst.host) j.f[R_F1] = S[j.sys].BP.all();
        InitFirst.upload(st);
    }
    run_sweep(OP_INIT, SFL, InitFirst, sys.d(), GATE_RUN, st, init_bytes(InitFirst, SFL));
    for (int i = 0; i < n; i++) S[i].t0 = t_start;

    const double bl = spinor_site_bytes(SFL), bx = spinor_site_bytes(SFX);
    const double bH1 = hop_bytes(H1, SFL, LFL, 0), bH2 = hop_bytes(H2, SFL, LFL, 2), bH4 = hop_bytes(H4, SFL, LFL, 1);
    const double bSW = sweep_bytes(SW, 3 * bl), bSXR = sweep_bytes(SXR, 2 * bx + 5 * bl), bSS = sweep_bytes(SS, 4 * bl);

    auto iterate = [&](hipStream_t q) {
        run_hop(SFL, LFL, false, RED_NONE, FIN_STORE, H1, sys.d(), GATE_RUN, q, bH1);
        run_hop(SFL, LFL, false, RED_ZDOT, FIN_BETA, H2, sys.d(), GATE_RUN, q, bH2);
        run_sweep(OP_W, SFL, SW, sys.d(), GATE_RUN, q, bSW);
        run_hop(SFL, LFL, false, RED_NONE, FIN_STORE, H3, sys.d(), GATE_RUN, q, bH1);
        run_hop(SFL, LFL, false, RED_OUTX, FIN_CHI, H4, sys.d(), GATE_RUN, q, bH4);
        run_sweep(OP_XR, SFL, SXR, sys.d(), GATE_RUN, q, bSXR);
        run_sweep(OP_S, SFL, SS, sys.d(), GATE_RUN, q, bSS);
    };
    std::shared_ptr<ChunkGraph> graph;
    if (graphs_on())
        graph = cached_graph(S[0].g, launch_key("eo", poll, SFL, LFL, sys.d(), H1, H2, SW, H3, H4, SXR, SS),
                             [&](hipStream_t q) {
                                 for (int k = 0; k < poll; k++) iterate(q);
                             });
    // Reliable update of the systems that stopped (gate GATE_STOPPED; finished systems are marked
    // ST_DONE first): x_hi += x_lo, r_hi = b_prec - M_prec x_hi, |r_hi|^2. Every step runs on the
    // full job tables, so no per-subset tables or host synchronisation are needed.
    auto reliable_update = [&]() {
        // the s update of the iteration in which the system stopped was gated off: apply it
        // (the scalars of that iteration are still in place), since a continuing reliable update
        // keeps s; defect correction restarts with s = r instead
        if (!(P.mixed && P.mixed_mode == WD_MIXED_DEFECT)) run_sweep(OP_S, SFL, SS, sys.d(), GATE_STOPPED, st, bSS);
        run_sweep(OP_ACC, SFL, Acc, sys.d(), GATE_STOPPED, st, sweep_bytes(Acc, 2 * 192 + 2 * bx));
        run_hop(SF64, L64, false, RED_NONE, FIN_STORE, Hx1, sys.d(), GATE_STOPPED, st, hop_bytes(Hx1, SF64, L64, 0));
        run_hop(SF64, L64, false, RED_NORM, FIN_STORE, Hx2, sys.d(), GATE_STOPPED, st, hop_bytes(Hx2, SF64, L64, 2));
    };

    int active = 0;
    for (auto& e : S) active += !e.done;
    long host_iters = 0;
    const long host_cap = (long)P.max_iter + 16L * poll + 64;
    while (active > 0) {
        if (graph) graph->launch(st);
        else
            for (int k = 0; k < poll; k++) iterate(st);
        host_iters += poll;
        sys.download(st);
        if (host_iters > host_cap) {
            // the device never reported an exit state: stop instead of iterating forever
            for (auto& e : S)
                if (!e.done) {
                    e.done = true;
                    e.final_status = WD_ERR_NOCONV;
                    e.t1 = now_s();
                }
            break;
        }
        bool any = false;
        for (int i = 0; i < n; i++) {
            const int stt = sys.h[i].status;
            if (S[i].done || stt == ST_RUNNING) continue;
            if (stt == ST_NAN) {  // gated off for good: no status change needed on the device
                S[i].done = true;
                S[i].final_status = WD_ERR_NAN;
                S[i].t1 = now_s();
                active--;
                continue;
            }
            any = true;
        }
        if (!any) continue;
        reliable_update();
        sys.download(st);
        bool any_next = false, any_fresh = false;
        for (int i = 0; i < n; i++) {
            EoSys& e = S[i];
            SysState& q = sys.h[i];
            const int stt = q.status;
            if (e.done || stt == ST_RUNNING || stt == ST_NAN) continue;
            e.reliable++;
            const double rr = q.red[2];
            e.rr_true = rr;
            int next = ST_SEL1;  // continue: keep rhat and s
            if (!std::isfinite(rr)) {
                e.done = true;
                e.final_status = WD_ERR_NAN;
            } else if (rr <= q.target2) {
                e.done = true;
                e.final_status = WD_OK;
            } else if (stt == ST_MAXIT || q.iter >= q.maxit) {
                e.done = true;
                e.final_status = WD_ERR_NOCONV;
            } else if (stt == ST_BREAKDOWN) {
                if (++e.restarts > 2) {
                    e.done = true;
                    e.final_status = WD_ERR_BREAKDOWN;
                } else {
                    next = ST_SEL2;  // restart fresh
                }
            }
            // new residual: keep rhat and s (reliable update) or restart with rhat = s = r
            // (breakdown, and every outer step of defect correction: a fresh inner solve)
            if (!e.done && P.mixed && P.mixed_mode == WD_MIXED_DEFECT) next = ST_SEL2;
            if (e.done) {
                e.t1 = now_s();
                active--;
                q.status = ST_DONE;
            } else {
                q.status = next;
                any_next = any_next || next == ST_SEL1;
                any_fresh = any_fresh || next == ST_SEL2;
            }
        }
        sys.upload(st);
        // the restart finishers set the continuing systems RUNNING again
        if (any_next) run_sweep(OP_INIT, SFL, InitRel, sys.d(), 1 << ST_SEL1, st, init_bytes(InitRel, SFL));
        if (any_fresh) run_sweep(OP_INIT, SFL, InitRestart, sys.d(), 1 << ST_SEL2, st, init_bytes(InitRestart, SFL));
    }

    // ---- finish: odd half from eq. eo3, unpack. With x_o from eq. eo3 the full residual is
    // b - M x = (b_prec - M_prec x_e) / a on the even sites and exactly zero on the odd ones, so
    // the last FP64 residual gives the true relative residual without another operator pass.
    // Systems whose last step was an FP64 residual update reuse its D_oe x_e (T64; zero for a zero
    // source); any other system applies the hop once more.
    {
        int nsweep = 0;
        for (int i = 0; i < n; i++) {
            const bool by_sweep = S[i].reliable > 0 || S[i].src.bb == 0.0;
            sys.h[i].status = by_sweep ? ST_SEL1 : ST_SEL2;
            nsweep += by_sweep;
        }
        if (nsweep < n) {
            sys.upload(st);
            run_hop(SF64, L64, false, RED_NONE, FIN_STORE, Hrec, sys.d(), 1 << ST_SEL2, st, hop_bytes(Hrec, SF64, L64, 1));
        }
        for (int i = 0; i < n; i++) {
            EoSys& e = S[i];
            if (sys.h[i].status == ST_SEL1)  // x_o = (b_o + 1/2 T64) / a, rebuilt while unpacking
                WD_CHECK_HIP(launch_unpack_eo(e.x, e.g->geo, e.X64.half(0), e.keep_odd ? e.X64.half(1) : SpinorRef{},
                                              e.src.B64.half(1), e.T64.all(), 1.0 / e.a, 0.5 / e.a, P.dagger, 1.0,
                                              st, e.g->gm(), e.g->nc));
            else
                WD_CHECK_HIP(launch_unpack_spinor(SF64, e.x, e.g->geo, e.X64.half(0), e.X64.half(1), P.dagger, 1.0,
                                                  st, e.g->gm(), e.g->nc));
        }
    }
    sys.download(st);
    for (int i = 0; i < n; i++) {
        EoSys& e = S[i];
        if (e.t1 == 0) e.t1 = now_s();
        e.iters = sys.h[i].iter;
        if (!std::isfinite(e.src.bb) || e.final_status == WD_ERR_NAN) e.true_rel = std::nan("");
        else e.true_rel = (e.src.bb > 0 && e.rr_true >= 0) ? std::sqrt(e.rr_true) / (e.a * std::sqrt(e.src.bb)) : 0.0;
    }
}

// ================================================================ BiCGstab-M (FP64, full lattice)

static wd_status ms_solve(wd_gauge* g, int nk, const double* kappas, double* const* x, const double* b,
                          const wd_solver_params& P, wd_solver_stats* stats, hipStream_t st, int poll)
{
    WD_REQUIRE(nk >= 1 && nk <= 32, "number of masses must be in 1..32");
    const double t0 = now_s();
    int base = 0;
    for (int i = 1; i < nk; i++)
        if (kappas[i] > kappas[base]) base = i;
    const double a = 1.0 / (2.0 * kappas[base]);
    const int ns = nk - 1;
    std::vector<int> shift_of(nk, -1), mass_of_shift;
    for (int i = 0; i < nk; i++)
        if (i != base) {
            shift_of[i] = (int)mass_of_shift.size();
            mass_of_shift.push_back(i);
        }

    Field B = g->field("ms.B", SF64, 2), X = g->field("ms.X", SF64, 2), R0 = g->field("ms.R0", SF64, 2);
    Field R1 = ns > 0 ? g->field("ms.R1", SF64, 2) : R0;
    Field Sv = g->field("ms.S", SF64, 2), AS = g->field("ms.AS", SF64, 2), W = g->field("ms.W", SF64, 2);
    Field AW = g->field("ms.AW", SF64, 2), RES = g->field("ms.RES", SF64, 2);
    std::vector<Field> XS(ns), SS(ns);
    for (int k = 0; k < ns; k++) {
        XS[k] = g->field("ms.XS" + std::to_string(k), SF64, 2);
        SS[k] = g->field("ms.SS" + std::to_string(k), SF64, 2);
    }
    const Geo& geo = g->geo;
    const int L64 = g->f64_links();

    SysArray sys;
    sys.alloc(1, g->raw["ms.sys"]);
    SysState& q = sys.h[0];
    std::memset(&q, 0, sizeof(q));
    q.partials = (double*)g->rawbuf("ms.partials", sizeof(double) * NRED * (2 * geo.stride / BLOCK + 1));
    q.maxit = P.max_iter;
    q.mixed = 0;
    q.nshift = ns;
    q.target2 = -1;
    q.beta_prev = make_double2(1.0, 0.0);
    q.alpha = make_double2(0.0, 0.0);
    std::vector<ShiftScal> sh(std::max(ns, 1));
    std::vector<SpinorRef> shv(2 * std::max(ns, 1));
    for (int k = 0; k < ns; k++) {
        ShiftScal& z = sh[k];
        std::memset(&z, 0, sizeof(z));
        z.sigma = 1.0 / (2.0 * kappas[mass_of_shift[k]]) - a;
        z.zeta_prev = z.zeta = z.rho = make_double2(1.0, 0.0);
        z.active = 1;
        shv[2 * k] = XS[k].all();
        shv[2 * k + 1] = SS[k].all();
    }
    ShiftScal* d_sh = (ShiftScal*)g->rawbuf("ms.sh", sizeof(ShiftScal) * sh.size());
    SpinorRef* d_shv = (SpinorRef*)g->rawbuf("ms.shv", sizeof(SpinorRef) * shv.size());
    {
        size_t n1 = sizeof(ShiftScal) * sh.size(), n2 = sizeof(SpinorRef) * shv.size();
        char* stg = (char*)pinned(n1 + n2);
        std::memcpy(stg, sh.data(), n1);
        std::memcpy(stg + n1, shv.data(), n2);
        WD_CHECK_HIP(hipMemcpyAsync(d_sh, stg, n1, hipMemcpyHostToDevice, st));
        WD_CHECK_HIP(hipMemcpyAsync(d_shv, stg + n1, n2, hipMemcpyHostToDevice, st));
        WD_CHECK_HIP(hipStreamSynchronize(st));
    }
    q.sh = d_sh;
    q.shv = d_shv;
    sys.upload(st);

    WD_CHECK_HIP(launch_pack_spinor(SF64, b, geo, B.half(0), B.half(1), P.dagger, 1.0, st, g->gm(), g->nc));
    const long nsites = B.nsites();
    JobTable<SweepJob> Init, SW, SXR, SEND;
    SweepJob j = sweep_job(0, nsites);
    j.f[R_F0] = R0.all();
    j.f[R_F1] = B.all();
    j.f[R_F2] = Sv.all();
    j.f[R_F3] = Sv.all();
    j.f[R_F4] = X.all();
    Init.host.push_back(j);
    j = sweep_job(0, nsites);
    j.f[R_F0] = W.all();
    j.f[R_F1] = R0.all();
    j.f[R_F2] = AS.all();
    j.f[R_F3] = R1.all();
    SW.host.push_back(j);
    j = sweep_job(0, nsites);
    j.f[R_F0] = X.all();
    j.f[R_F1] = R0.all();
    j.f[R_F2] = Sv.all();
    j.f[R_F3] = W.all();
    j.f[R_F4] = AW.all();
    j.f[R_F5] = B.all();
    j.f[R_F6] = R1.all();
    SXR.host.push_back(j);
    j = sweep_job(0, nsites);
    j.f[R_F0] = Sv.all();
    j.f[R_F1] = R0.all();
    j.f[R_F2] = AS.all();
    j.f[R_F3] = R1.all();
    j.f[R_F4] = W.all();
    SEND.host.push_back(j);
    JobTable<HopJob> HAs, HAw;
    for (int p = 0; p < 2; p++) {
        HopJob h = hop_job(geo, p, 0, Sv.half(1 - p), AS.half(p), g->slk(L64, p), g->lcs(), -0.5);
        h.tg = g->tg;
        h.nc = g->nc;
        h.x0 = Sv.half(p);
        h.c0 = a;
        h.z = B.half(p);
        HAs.host.push_back(h);
        h = hop_job(geo, p, 0, W.half(1 - p), AW.half(p), g->slk(L64, p), g->lcs(), -0.5);
        h.tg = g->tg;
        h.nc = g->nc;
        h.x0 = W.half(p);
        h.c0 = a;
        HAw.host.push_back(h);
    }
    const int tz64 = tune_tile(g, SF64, L64, st);
    for (auto* t : {&HAs, &HAw})
        for (auto& h : t->host) set_tile(h, tz64);
    for (auto* t : {&Init, &SW, &SXR, &SEND}) layout(*t);
    for (auto* t : {&HAs, &HAw}) layout(*t);
    upload_tables(st, g->raw["ms.tables"], {&Init, &SW, &SXR, &SEND, &HAs, &HAw});
    run_sweep(OP_MSINIT, SF64, Init, sys.d(), 0, st, sweep_bytes(Init, (4 + 2 * ns) * 192.0));
    sys.download(st);
    const double bb = sys.h[0].red[2];
    sys.h[0].target2 = P.tol * P.tol * bb;
    sys.h[0].shift_target2 = P.tol * P.tol * bb;
    sys.h[0].beta_prev = make_double2(1.0, 0.0);
    sys.h[0].alpha = make_double2(0.0, 0.0);
    if (bb == 0.0) sys.h[0].status = ST_CONVERGED;
    sys.upload(st);

    const int endop = ns > 0 ? OP_SHIFT : OP_S;
    const double bH = hop_bytes(HAs, SF64, L64, 2), bHw = hop_bytes(HAw, SF64, L64, 1);
    auto iterate = [&](int active_shifts, hipStream_t q) {
        run_hop(SF64, L64, false, RED_ZDOT, FIN_BETA, HAs, sys.d(), GATE_RUN, q, bH);
        run_sweep(OP_W, SF64, SW, sys.d(), GATE_RUN, q, sweep_bytes(SW, 3 * 192));
        run_hop(SF64, L64, false, RED_OUTX, FIN_CHI, HAw, sys.d(), GATE_RUN, q, bHw);
        run_sweep(OP_XR, SF64, SXR, sys.d(), GATE_RUN, q, sweep_bytes(SXR, 7 * 192));
        run_sweep(endop, SF64, SEND, sys.d(), GATE_RUN, q, sweep_bytes(SEND, (ns > 0 ? 6 : 4) * 192 + 4 * 192 * active_shifts));
    };
    std::shared_ptr<ChunkGraph> graph;
    if (graphs_on())
        graph = cached_graph(g, launch_key("ms", poll, ns, endop, sys.d(), HAs, SW, HAw, SXR, SEND), [&](hipStream_t q) {
            for (int k = 0; k < poll; k++) iterate(ns, q);
        });
    int status = WD_OK;
    int active_shifts = ns;
    long host_iters = 0;
    const long host_cap = (long)P.max_iter + 16L * poll + 64;
    while (true) {
        if (sys.h[0].status != ST_RUNNING) break;
        if (host_iters > host_cap) break;  // no exit state reported by the device
        if (graph) graph->launch(st);
        else
            for (int k = 0; k < poll; k++) iterate(active_shifts, st);
        host_iters += poll;
        sys.download(st);
        if (ns > 0) {
            size_t n1 = sizeof(ShiftScal) * ns;
            void* stg = pinned(n1);
            WD_CHECK_HIP(hipMemcpyAsync(stg, d_sh, n1, hipMemcpyDeviceToHost, st));
            WD_CHECK_HIP(hipStreamSynchronize(st));
            std::memcpy(sh.data(), stg, n1);
            active_shifts = 0;
            for (int k = 0; k < ns; k++) active_shifts += sh[k].active;
        }
    }
    switch (sys.h[0].status) {
    case ST_CONVERGED: status = WD_OK; break;
    case ST_MAXIT: status = WD_ERR_NOCONV; break;
    case ST_BREAKDOWN: status = WD_ERR_BREAKDOWN; break;
    case ST_NAN: status = WD_ERR_NAN; break;
    default: status = WD_ERR_NOCONV;
    }
    if (ns > 0) {
        size_t n1 = sizeof(ShiftScal) * ns;
        void* stg = pinned(n1);
        WD_CHECK_HIP(hipMemcpyAsync(stg, d_sh, n1, hipMemcpyDeviceToHost, st));
        WD_CHECK_HIP(hipStreamSynchronize(st));
        std::memcpy(sh.data(), stg, n1);
    }
    const int iters = sys.h[0].iter;
    const double t1 = now_s();

    // true residual of every mass in one launch (one reduction group per mass; the residual
    // fields are not kept, only their norms), then unpack
    {
        const size_t pstride = (size_t)NRED * (2 * geo.stride / BLOCK + 1);
        SysArray rs;
        rs.alloc(nk, g->raw["ms.rsys"]);
        double* rpart = (double*)g->rawbuf("ms.rpartials", sizeof(double) * pstride * nk);
        for (int i = 0; i < nk; i++) {
            std::memset(&rs.h[i], 0, sizeof(SysState));
            rs.h[i].partials = rpart + pstride * i;
        }
        JobTable<HopJob> R;
        for (int i = 0; i < nk; i++) {
            const Field& Xi = i == base ? X : XS[shift_of[i]];
            const double ai = 1.0 / (2.0 * kappas[i]);
            for (int p = 0; p < 2; p++) {
                HopJob h = hop_job(geo, p, i, Xi.half(1 - p), RES.half(p), g->slk(L64, p), g->lcs(), 0.5);
                h.tg = g->tg;
                h.nc = g->nc;
                h.x0 = B.half(p);
                h.c0 = 1.0;
                h.x1 = Xi.half(p);
                h.c1 = -ai;
                set_tile(h, tz64);
                R.host.push_back(h);
            }
        }
        layout(R);
        upload_tables(st, g->raw["ms.rtables"], {&R});
        rs.upload(st);
        run_hop(SF64, L64, false, RED_NORM, FIN_STORE, R, rs.d(), 0, st, hop_bytes(R, SF64, L64, 2));
        for (int i = 0; i < nk; i++) {
            const Field& Xi = i == base ? X : XS[shift_of[i]];
            WD_CHECK_HIP(launch_unpack_spinor(SF64, x[i], geo, Xi.half(0), Xi.half(1), P.dagger, 1.0, st, g->gm(), g->nc));
        }
        rs.download(st);
        if (stats)
            for (int i = 0; i < nk; i++) {
                stats[i].iters = i == base ? iters : (sh[shift_of[i]].active ? iters : sh[shift_of[i]].conv_iter);
                stats[i].reliable_updates = 0;
                stats[i].true_rel_res = !std::isfinite(bb) ? std::nan("") : bb > 0 ? std::sqrt(rs.h[i].red[2] / bb) : 0.0;
                stats[i].status = status;
                stats[i].seconds = t1 - t0;
            }
    }
    return (wd_status)status;
}

// ================================================================ entry points used by the C ABI

wd_status solve_single(wd_gauge* g, double kappa, double* x, const double* b, const wd_solver_params& P,
                       wd_solver_stats* stats, hipStream_t st)
{
    WD_REQUIRE(kappa > 0, "kappa must be positive");
    if (!P.eo) {
        WD_REQUIRE(!P.mixed, "mixed precision requires even-odd preconditioning");
        WD_REQUIRE(!P.use_x0, "a start vector requires even-odd preconditioning");
        double* xs[1] = {x};
        return ms_solve(g, 1, &kappa, xs, b, P, stats, st, 4);
    }
    std::vector<EoSys> S(1);
    S[0].g = g;
    S[0].kappa = kappa;
    S[0].b = b;
    S[0].x = x;
    S[0].slot = 0;
    eo_solve(S, P, st, kPoll);
    if (stats) {
        stats->iters = S[0].iters;
        stats->reliable_updates = S[0].reliable;
        stats->status = S[0].final_status;
        stats->true_rel_res = S[0].true_rel;
        stats->seconds = S[0].t1 - S[0].t0;
    }
    return (wd_status)S[0].final_status;
}

wd_status solve_multishift(wd_gauge* g, int n, const double* kappas, double* const* x, const double* b,
                           const wd_solver_params& P, wd_solver_stats* stats, hipStream_t st)
{
    for (int i = 0; i < n; i++) WD_REQUIRE(kappas[i] > 0, "kappa must be positive");
    return ms_solve(g, n, kappas, x, b, P, stats, st, 4);
}

wd_status solve_batch(int nsys, const wd_system* sys, const wd_solver_params& P, wd_solver_stats* stats,
                      hipStream_t st)
{
    WD_REQUIRE(nsys >= 1 && nsys <= 1024, "nsys must be in 1..1024");
    WD_REQUIRE(P.eo, "batched solves use even-odd preconditioning");
    std::vector<EoSys> S(nsys);
    std::map<wd_gauge*, int> slots;
    for (int i = 0; i < nsys; i++) {
        WD_REQUIRE(sys[i].gauge && sys[i].b && sys[i].x, "null system entry");
        WD_REQUIRE(sys[i].kappa > 0, "kappa must be positive");
        S[i].g = sys[i].gauge;
        S[i].kappa = sys[i].kappa;
        S[i].b = sys[i].b;
        S[i].x = sys[i].x;
        S[i].slot = slots[sys[i].gauge]++;
    }
    eo_solve(S, P, st, kPoll);
    wd_status worst = WD_OK;
    for (int i = 0; i < nsys; i++) {
        if (stats) {
            stats[i].iters = S[i].iters;
            stats[i].reliable_updates = S[i].reliable;
            stats[i].status = S[i].final_status;
            stats[i].true_rel_res = S[i].true_rel;
            stats[i].seconds = S[i].t1 - S[i].t0;
        }
        if (S[i].final_status != WD_OK && worst == WD_OK) worst = (wd_status)S[i].final_status;
    }
    return worst;
}

// The even-odd operator in the solvers' storage formats, hop variants chosen by the caller: out_o =
// D_oe in_e (first hop, stored), out_e = a^2 in_e - 1/4 D_eo out_o (second hop with the epilogue of
// v.red); the adjoint hops with v.dagger. Each of v.copies systems has its own fields and its own
// reduction group; systems on one gauge field share link loads (interleaved groups) as in the
// batched solvers.
wd_status apply_prec(wd_gauge* g, double kappa, double* out, const double* in, const wd_solver_params& P,
                     const wd_op_variant& v, double* dots, hipStream_t st)
{
    WD_REQUIRE(kappa > 0, "kappa must be positive");
    WD_REQUIRE(v.red >= WD_RED_NONE && v.red <= WD_RED_NORM, "unknown reduction");
    WD_REQUIRE(v.copies >= 1 && v.copies <= 64, "copies must be in 1..64");
    WD_REQUIRE(v.stage >= -1 && v.stage <= 1 && v.nontemporal >= -1 && v.nontemporal <= 1, "bad stage / nontemporal");
    WD_REQUIRE(v.tile >= -1, "bad tile");
    WD_REQUIRE(v.rhs_per_thread >= -1 && v.rhs_per_thread <= 4, "rhs_per_thread must be in -1..4");
    const int SFL = P.mixed ? spinor_fmt_of(P.spinor_store) : SF64;
    const int LFL = P.mixed ? link_fmt_of(P.link_store, P.recon) : g->f64_links();
    if (v.dagger && !(v.red == WD_RED_NONE || v.red == WD_RED_ZDOT || (SFL == SF64 && v.red == WD_RED_NORM)))
        throw Error{WD_ERR_UNSUPPORTED, "the adjoint hops fuse no <out, in> reduction (and |out|^2 in FP64 only)"};
    if (SFL == SF64 && LFL != L64_12 && LFL != L64_18)
        throw Error{WD_ERR_UNSUPPORTED, "FP64 spinors take FP64 links"};
    if (SFL != SF64 && (LFL == L64_12 || LFL == L64_18))
        throw Error{WD_ERR_UNSUPPORTED, "FP64 links take FP64 spinors"};
    if (link_recon12(LFL) && g->recon_err > 1e-6)
        throw Error{WD_ERR_UNSUPPORTED, "links are not SU(3): the 12-real formats would change the operator"};
    g->ensure_slinks(LFL, st);
    const Geo& G = g->geo;
    const int K = v.copies;
    const double a = 1.0 / (2.0 * kappa);
    const long V = g->V;
    std::vector<Field> F(K), Tm(K), O(K);
    for (int k = 0; k < K; k++) {
        F[k] = g->field("ap.in" + std::to_string(k), SFL, 2);
        Tm[k] = g->field("ap.t" + std::to_string(k), SFL, 1);
        O[k] = g->field("ap.out" + std::to_string(k), SFL, 1);
    }
    SysArray sys;
    sys.alloc(K, g->raw["ap.sys"]);
    const size_t pstride = (size_t)NRED * (2 * G.stride / BLOCK + 1);
    double* part = (double*)g->rawbuf("ap.partials", sizeof(double) * pstride * K);
    for (int k = 0; k < K; k++) {
        std::memset(&sys.h[k], 0, sizeof(SysState));
        sys.h[k].partials = part + pstride * k;
    }
    sys.upload(st);
    HopChoice ch;
    if (v.tile < 0 || v.rhs_per_thread < 0) ch = tune_hop(g, SFL, LFL, st, K);
    const int tz = v.tile < 0 ? ch.tz : (tile_valid(G, v.tile) ? v.tile : 0);
    const int rhs = v.rhs_per_thread < 0 ? ch.rhs : (v.rhs_per_thread <= 1 ? 0 : v.rhs_per_thread);
    if (rhs >= 2 && (SFL == SF64 || v.red == WD_RED_NORM))
        throw Error{WD_ERR_UNSUPPORTED, "the multi-RHS hop takes FP32 / FP16 spinors and no |out|^2-only reduction"};
    const bool tg = g->tg && !v.dagger;  // the adjoint hops read every stored link
    JobTable<HopJob> H1, H2;
    for (int k = 0; k < K; k++) {
        HopJob j = hop_job(G, 1, k, F[k].half(0), Tm[k].all(), g->slk(LFL, 1), g->lcs(), 1.0);
        j.tg = tg;
        j.nc = g->nc;
        j.rhs = rhs;
        set_tile(j, tz);
        H1.host.push_back(j);
        j = hop_job(G, 0, k, Tm[k].all(), O[k].all(), g->slk(LFL, 0), g->lcs(), -0.25);
        j.tg = tg;
        j.nc = g->nc;
        j.rhs = rhs;
        j.x0 = F[k].half(0);
        j.c0 = a * a;
        j.z = F[k].half(0);
        set_tile(j, tz);
        H2.host.push_back(j);
    }
    layout(H1);
    layout(H2);
    upload_tables(st, g->raw["ap.tables"], {&H1, &H2});
    for (int k = 0; k < K; k++)
        WD_CHECK_HIP(launch_pack_spinor(SFL, in + (size_t)k * V * 24, G, F[k].half(0), F[k].half(1), 0, 1.0, st, g->gm(), g->nc));
    const int ext[4] = {1, 2, 1, 1};  // epilogue fields read by the second hop (x0, and z for ZDOT)
    run_hop(SFL, LFL, v.dagger != 0, RED_NONE, FIN_STORE, H1, sys.d(), 0, st, hop_bytes(H1, SFL, LFL, 0), v.stage,
            v.nontemporal);
    // the hop kernel depends on the reduction kind only; its finisher here just stores the sums
    run_hop(SFL, LFL, v.dagger != 0, v.red, FIN_STORE, H2, sys.d(), 0, st, hop_bytes(H2, SFL, LFL, ext[v.red]),
            v.stage, v.nontemporal);
    for (int k = 0; k < K; k++)
        WD_CHECK_HIP(
            launch_unpack_spinor(SFL, out + (size_t)k * V * 24, G, O[k].all(), Tm[k].all(), 0, 1.0, st, g->gm(), g->nc));
    sys.download(st);
    if (dots)
        for (int k = 0; k < K; k++)
            for (int i = 0; i < 3; i++) dots[3 * k + i] = sys.h[k].red[i];
    return WD_OK;
}

// <a, v_j> for every view v_j (full FP64 fields of handle g), through the device multi-dot
static std::vector<double2> field_dots(wd_gauge* g, const SpinorRef& a, const std::vector<SpinorRef>& vs,
                                       hipStream_t st)
{
    std::vector<double2> out;
    const Geo& G = g->geo;
    double* partials = (double*)g->rawbuf("dots.partials", sizeof(double) * 2 * DOTS_MAX * (2 * G.stride / BLOCK + 1));
    SpinorRef* refs = (SpinorRef*)g->rawbuf("dots.refs", sizeof(SpinorRef) * DOTS_MAX);
    double* res = (double*)g->rawbuf("dots.out", sizeof(double) * 2 * DOTS_MAX);
    for (size_t j0 = 0; j0 < vs.size(); j0 += DOTS_MAX) {
        const int m = (int)std::min<size_t>(DOTS_MAX, vs.size() - j0);
        char* stg = (char*)pinned(sizeof(SpinorRef) * DOTS_MAX + sizeof(double) * 2 * DOTS_MAX);
        std::memcpy(stg, vs.data() + j0, sizeof(SpinorRef) * m);
        WD_CHECK_HIP(hipMemcpyAsync(refs, stg, sizeof(SpinorRef) * m, hipMemcpyHostToDevice, st));
        WD_CHECK_HIP(launch_dots(a, refs, m, G, partials, res, st));
        double* back = (double*)(stg + sizeof(SpinorRef) * DOTS_MAX);
        WD_CHECK_HIP(hipMemcpyAsync(back, res, sizeof(double) * 2 * m, hipMemcpyDeviceToHost, st));
        WD_CHECK_HIP(hipStreamSynchronize(st));
        for (int j = 0; j < m; j++) out.push_back(make_double2(back[2 * j], back[2 * j + 1]));
    }
    return out;
}

// Solution-space minimisation (Sec. 6.2.2) for the mass kappa over the solutions done[j_first ..
// j_first + k): with d_j = M(kappa) psi_j = b + s_j psi_j, s_j = 1/(2 kappa) - 1/(2 kappa_j),
// minimise |b - sum_j c_j d_j|_2: sum_j <d_i, d_j> c_j = <d_i, b>, with
//   <d_i, d_j> = |b|^2 + s_j <b, psi_j> + s_i <psi_i, b> + s_i s_j <psi_i, psi_j>.
// Gaussian elimination with partial pivoting on the small Hermitian system, with a relative
// 1e-13 diagonal shift against exactly dependent solutions.
static std::vector<double2> minres_coefficients(const std::vector<std::vector<double2>>& Pg,
                                                const std::vector<double2>& qb, double bb, const double* kappas,
                                                const std::vector<int>& done, int j_first, int k, double kappa)
{
    auto cmul = [](double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); };
    auto cdiv = [](double2 a, double2 b) {
        const double d = b.x * b.x + b.y * b.y;
        return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
    };
    std::vector<double> sv(k);
    for (int j = 0; j < k; j++) sv[j] = 1.0 / (2.0 * kappa) - 1.0 / (2.0 * kappas[done[j_first + j]]);
    std::vector<std::vector<double2>> A(k, std::vector<double2>(k + 1));
    double dmax = 0;
    for (int i = 0; i < k; i++) {
        const int gi = j_first + i;
        const double2 qi = qb[gi], qic = make_double2(qi.x, -qi.y);  // <b, psi_i>, <psi_i, b>
        for (int j = 0; j < k; j++) {
            const int gj = j_first + j;
            const double2 qj = qb[gj];
            const double2 pij = Pg[gi][gj];
            A[i][j] = make_double2(bb + sv[j] * qj.x + sv[i] * qic.x + sv[i] * sv[j] * pij.x,
                                   sv[j] * qj.y + sv[i] * qic.y + sv[i] * sv[j] * pij.y);
        }
        A[i][k] = make_double2(bb + sv[i] * qic.x, sv[i] * qic.y);
        dmax = std::max(dmax, A[i][i].x);
    }
    for (int i = 0; i < k; i++) A[i][i].x += 1e-13 * dmax;
    for (int col = 0; col < k; col++) {
        int piv = col;
        for (int r = col + 1; r < k; r++)
            if (std::hypot(A[r][col].x, A[r][col].y) > std::hypot(A[piv][col].x, A[piv][col].y)) piv = r;
        std::swap(A[col], A[piv]);
        if (A[col][col].x == 0.0 && A[col][col].y == 0.0) continue;
        for (int r = col + 1; r < k; r++) {
            const double2 f = cdiv(A[r][col], A[col][col]);
            for (int c = col; c <= k; c++) {
                const double2 t = cmul(f, A[col][c]);
                A[r][c] = make_double2(A[r][c].x - t.x, A[r][c].y - t.y);
            }
        }
    }
    std::vector<double2> c(k, make_double2(0, 0));
    for (int i = k - 1; i >= 0; i--) {
        double2 t = A[i][k];
        for (int j = i + 1; j < k; j++) {
            const double2 u = cmul(A[i][j], c[j]);
            t = make_double2(t.x - u.x, t.y - u.y);
        }
        c[i] = (A[i][i].x == 0.0 && A[i][i].y == 0.0) ? make_double2(0, 0) : cdiv(t, A[i][i]);
    }
    return c;
}

wd_status solve_multimass(wd_gauge* g, int n, const double* kappas, double* const* x, const double* b, int method,
                          int guess, const wd_solver_params& P, wd_solver_stats* stats, hipStream_t st)
{
    WD_REQUIRE(n >= 1 && n <= 32, "number of masses must be in 1..32");
    for (int i = 0; i < n; i++) WD_REQUIRE(kappas[i] > 0, "kappa must be positive");
    if (method == WD_METHOD_MULTISHIFT) return solve_multishift(g, n, kappas, x, b, P, stats, st);
    if (method == WD_METHOD_BATCHED) {
        // every mass is its own single-mass system; all iterate together, one launch per solver
        // step, sharing one packed source (no start guesses: the masses are solved simultaneously)
        WD_REQUIRE(P.eo, "batched solves use even-odd preconditioning");
        WD_REQUIRE(guess == WD_GUESS_NONE || guess == WD_GUESS_POLY || guess == WD_GUESS_MINRES, "unknown guess");
        EoSource src;
        prepare_source(g, "mm.", b, P.dagger, src, st);
        std::vector<EoSys> S(n);
        for (int i = 0; i < n; i++) {
            S[i].g = g;
            S[i].kappa = kappas[i];
            S[i].b = b;
            S[i].x = x[i];
            S[i].slot = i;
            S[i].src = src;
        }
        wd_solver_params Q = P;
        Q.use_x0 = 0;
        eo_solve(S, Q, st, kPoll);
        wd_status worst = WD_OK;
        for (int i = 0; i < n; i++) {
            if (stats) {
                stats[i].iters = S[i].iters;
                stats[i].reliable_updates = S[i].reliable;
                stats[i].status = S[i].final_status;
                stats[i].true_rel_res = S[i].true_rel;
                stats[i].seconds = S[i].t1 - S[i].t0;
            }
            if (S[i].final_status != WD_OK && worst == WD_OK) worst = (wd_status)S[i].final_status;
        }
        return worst;
    }
    WD_REQUIRE(method == WD_METHOD_SEQUENTIAL, "unknown method");
    WD_REQUIRE(guess == WD_GUESS_NONE || guess == WD_GUESS_POLY || guess == WD_GUESS_MINRES, "unknown guess");
    WD_REQUIRE(P.guess_order >= 0, "guess_order must be >= 0");
    std::vector<int> order(n);
    for (int i = 0; i < n; i++) order[i] = i;
    // heaviest mass (smallest kappa) first (Sec. 7)
    std::stable_sort(order.begin(), order.end(), [&](int p, int q) { return kappas[p] < kappas[q]; });
    wd_status worst = WD_OK;
    if (!P.eo) {
        if (guess != WD_GUESS_NONE) throw Error{WD_ERR_UNSUPPORTED, "start guesses need even-odd preconditioning"};
        for (int idx : order) {
            wd_status s = solve_single(g, kappas[idx], x[idx], b, P, stats ? &stats[idx] : nullptr, st);
            if (s != WD_OK && worst == WD_OK) worst = s;
        }
        return worst;
    }
    // the source is packed once and 1/2 D_eo b_o is shared by all masses; every mass keeps its
    // FP64 solution so that the next start vector is a combination of them in the internal layout
    EoSource src;
    prepare_source(g, "mm.", b, P.dagger, src, st);
    // and its final FP64 residual b_prec - M_prec x_e (for the next start residual)
    std::vector<Field> X(n), R(n);
    for (int i = 0; i < n; i++) {
        X[i] = g->field("mm.X" + std::to_string(i), SF64, 2);
        R[i] = g->field("mm.R" + std::to_string(i), SF64, 1);
    }
    std::vector<char> res_ok(n, 0);  // R[i] holds the residual of X[i] (a converged FP64 check)
    Field BPm = g->field("mm.BP", SF64, 1);
    SysState* dummy = (SysState*)g->rawbuf("apply.sys", sizeof(SysState));
    std::vector<int> done;
    // solution-space minimisation: Gram entries <psi_i, psi_j> and <b, psi_i> of the solutions in
    // order of completion (indices into done)
    std::vector<std::vector<double2>> Pg;
    std::vector<double2> qb;
    for (int idx : order) {
        wd_solver_params Q = P;
        Q.use_x0 = 0;
        EoSys e;
        e.g = g;
        e.kappa = kappas[idx];
        e.b = b;
        e.x = x[idx];
        e.slot = 0;
        e.src = src;
        e.X64 = X[idx];
        e.RH = R[idx];
        e.BP = BPm;
        e.keep_odd = guess == WD_GUESS_MINRES;  // its inner products run over full solutions
        const int kall = (int)done.size();
        const int k = P.guess_order > 0 ? std::min(P.guess_order, kall) : kall;
        const int j_first = kall - k;  // the k most recently solved masses
        if (guess != WD_GUESS_NONE && k > 0) {
            std::vector<double2> c(k);
            if (guess == WD_GUESS_POLY) {
                // Lagrange weights in m a = 1/(2 kappa) - 4 (Sec. 6.2.1) over the distinct masses
                // among the previous ones (the latest solution of a repeated mass); a mass solved
                // before is its own guess
                const double m = 1.0 / (2.0 * kappas[idx]) - 4.0;
                std::vector<bool> use(k, true);
                int same = -1;
                for (int jj = 0; jj < k; jj++) {
                    const double kj = kappas[done[j_first + jj]];
                    for (int ii = jj + 1; ii < k; ii++)
                        if (kappas[done[j_first + ii]] == kj) use[jj] = false;
                    if (use[jj] && kj == kappas[idx]) same = jj;
                }
                for (int jj = 0; jj < k; jj++) {
                    double w = 0.0;
                    if (same >= 0) w = jj == same ? 1.0 : 0.0;
                    else if (use[jj]) {
                        const double mj = 1.0 / (2.0 * kappas[done[j_first + jj]]) - 4.0;
                        w = 1.0;
                        for (int ii = 0; ii < k; ii++) {
                            if (ii == jj || !use[ii]) continue;
                            const double mi = 1.0 / (2.0 * kappas[done[j_first + ii]]) - 4.0;
                            w *= (m - mi) / (mj - mi);
                        }
                    }
                    c[jj] = make_double2(w, 0.0);
                }
            } else {
                c = minres_coefficients(Pg, qb, src.bb, kappas, done, j_first, k, kappas[idx]);
            }
            const bool cplx = guess == WD_GUESS_MINRES;
            bool fused = !cplx;
            for (int jj = 0; jj < k; jj++)
                if (c[jj].x != 0.0 && !res_ok[done[j_first + jj]]) fused = false;
            // Lagrange guess: x0 and its start residual b_prec - M_prec x0 in one pass over the
            // stored solutions and their FP64 residuals (k_guess; no operator application)
            const double a = 1.0 / (2.0 * kappas[idx]);
            double sum_c = 0.0, sum_ca = 0.0;
            for (int jj = 0; jj < k && fused; jj++) {
                sum_c += c[jj].x;
                sum_ca += c[jj].x / (2.0 * kappas[done[j_first + jj]]);
            }
            for (int j0 = 0; j0 < k && fused; j0 += GUESS_MAX) {
                GuessArgs A;
                std::memset(&A, 0, sizeof(A));
                A.x0 = X[idx].half(0);
                A.r0 = R[idx].all();
                A.n = R[idx].nsites();
                A.acc = j0 > 0;
                if (j0 == 0) {
                    A.be = src.B64.half(0);
                    A.h = src.HB.all();
                    A.cb = a - sum_ca;
                    A.ch = 1.0 - sum_c;
                    A.bp = BPm.all();  // b_prec of this mass, for its FP64 residual updates
                    A.a = a;
                }
                A.k = std::min(GUESS_MAX, k - j0);
                for (int jj = 0; jj < A.k; jj++) {
                    const int j = done[j_first + j0 + jj];
                    const double aj = 1.0 / (2.0 * kappas[j]);
                    A.xs[jj] = X[j].half(0);
                    A.rs[jj] = R[j].all();
                    A.c[jj] = c[j0 + jj].x;
                    A.cx[jj] = c[j0 + jj].x * (aj * aj - a * a);
                }
                WD_CHECK_HIP(launch_guess(A, st));
            }
            if (fused) e.r_ready = e.bp_ready = true;
            // otherwise x0 = sum_j c_j x_j over the even half, in chunks (7 real or 4 complex inputs
            // per sweep), and the solver computes its residual with the FP64 operator
            const int per = cplx ? 4 : 7;
            for (int j0 = 0; j0 < k && !fused; j0 += per) {
                JobTable<SweepJob> L;
                SweepJob sj = sweep_job(0, X[idx].stride);
                sj.f[R_F0] = X[idx].half(0);
                const int mc = std::min(per, k - j0);
                for (int jj = 0; jj < mc; jj++) {
                    sj.f[1 + jj] = X[done[j_first + j0 + jj]].half(0);
                    if (cplx) {
                        sj.c[2 * jj] = c[j0 + jj].x;
                        sj.c[2 * jj + 1] = c[j0 + jj].y;
                    } else {
                        sj.c[jj] = c[j0 + jj].x;
                    }
                }
                sj.flags = (mc << 8) | (j0 > 0 ? 1 : 0) | (cplx ? 2 : 0);
                L.host.push_back(sj);
                layout(L);
                // stream order: the copy runs after the previous chunk's sweep has read the buffer
                upload_tables(st, g->raw["mm.tables"], {&L});
                run_sweep(OP_LINCOMB, SF64, L, dummy, 0, st, sweep_bytes(L, (mc + 1 + (j0 > 0)) * 192.0));
            }
            e.x_ready = true;
        }
        std::vector<EoSys> S{e};
        eo_solve(S, Q, st, kPoll);
        src = S[0].src;  // |b|^2 is known after the first mass
        if (stats) {
            stats[idx].iters = S[0].iters;
            stats[idx].reliable_updates = S[0].reliable;
            stats[idx].status = S[0].final_status;
            stats[idx].true_rel_res = S[0].true_rel;
            stats[idx].seconds = S[0].t1 - S[0].t0;
        }
        if (S[0].final_status != WD_OK && worst == WD_OK) worst = (wd_status)S[0].final_status;
        res_ok[idx] = S[0].final_status == WD_OK && S[0].reliable > 0;
        done.push_back(idx);
        if (guess == WD_GUESS_MINRES && (int)done.size() < n) {
            // inner products of the new solution with b and with every stored solution (itself
            // included), full lattice: <x_new, v> for v in (b, x_done...)
            std::vector<SpinorRef> vs{src.B64.all()};
            for (int j : done) vs.push_back(X[j].all());
            std::vector<double2> d = field_dots(g, X[idx].all(), vs, st);
            qb.push_back(make_double2(d[0].x, -d[0].y));  // <b, x_new>
            const int kn = (int)done.size();
            for (auto& row : Pg) row.push_back(make_double2(0, 0));
            Pg.emplace_back(kn);
            for (int j = 0; j < kn; j++) {
                Pg[kn - 1][j] = d[1 + j];                                   // <x_new, x_j>
                Pg[j][kn - 1] = make_double2(d[1 + j].x, -d[1 + j].y);      // <x_j, x_new>
            }
        }
    }
    return worst;
}


// ================================================================ CG / CG-M on the shifted normal equations

// The even-site systems (M_prec^dag M_prec + sigma) x = b_e, M_prec of eq. eo4 (Sec. 8 names CG and
// CG-M as the Krylov pair the findings carry over to; the shifted family shares one Krylov space,
// Sec. 6.1). A = M_prec^dag M_prec is applied as four hops: t = D_oe p, v = a^2 p - 1/4 D_eo t,
// t = (D_eo)^dag v, A p + sigma p = a^2 v - 1/4 (D_oe)^dag t + sigma p, the adjoint hops being the
// parity blocks of D^dag = gamma5 D gamma5 on the same links.
struct CgSys {
    wd_gauge* g;
    double kappa, a, sigma;
    const double* b;
    double* x;
    int slot;
    EoSource src;          // packed b (shared by systems with the same source)
    double be2 = -1;       // |b_e|^2 (computed here when negative)
    Field X64;             // FP64 solution: even half iterated, odd half zero
    bool x_ready = false;  // the even half of X64 holds the start vector, the odd half is zero
    bool r_ready = false;  // RH (caller-provided) holds b_e - (A + sigma) x0 (one system only)
    Field RH, T64, V64;    // FP64 residual (even) and operator temporaries (odd, even)
    Field r, p, t, v, w, xl;
    bool done = false;
    int restarts = 0, reliable = 0, final_status = WD_OK, iters = 0;
    double rr_true = -1, true_rel = 0, t0 = 0, t1 = 0;
};

// Single-shift CG for a batch of systems (one launch per solver step for all of them), in the
// precision scheme of the even-odd BiCGstab: low-precision iteration, FP64 reliable updates
// (x_hi += x_lo, r_hi = b_e - (A + sigma) x_hi in FP64) or defect correction, an FP64 check of
// every exit.
static void cg_solve(std::vector<CgSys>& S, const wd_solver_params& P, hipStream_t st, int poll)
{
    const int n = (int)S.size();
    const int SFL = P.mixed ? spinor_fmt_of(P.spinor_store) : SF64;
    const int SFX = SFL == SF64 ? SF64 : SF32;
    int L64 = L64_12;
    for (auto& e : S)
        if (e.g->f64_links() != L64_12) L64 = L64_18;
    const int LFL = P.mixed ? link_fmt_of(P.link_store, P.recon) : L64;
    if (P.mixed && link_recon12(LFL))
        for (auto& e : S)
            if (e.g->recon_err > 1e-6)
                throw Error{WD_ERR_UNSUPPORTED, "links are not SU(3): the 12-real low-precision formats would change "
                                                "the operator; solve with mixed = 0"};
    const double t_start = now_s();
    // systems on the same gauge field share link loads (multi-RHS hop or interleaved block pairs)
    std::vector<int> tile_lo(n), tile_64(n);
    const int rhs_lo = tune_shared_hops(S, SFL, LFL, L64, st, tile_lo, tile_64);
    for (auto& e : S) {
        e.g->ensure_slinks(LFL, st);
        e.g->ensure_slinks(L64, st);
        const std::string k = "cg" + std::to_string(e.slot) + ".";
        if (!e.src.B64.mem) prepare_source(e.g, k, e.b, 0, e.src, st);
        if (!e.X64.mem) e.X64 = e.g->field(k + "X64", SF64, 2);
        if (!e.RH.mem) e.RH = e.g->field(k + "RH", SF64, 1);
        e.T64 = e.g->field(k + "T64", SF64, 1);
        e.V64 = e.g->field(k + "V64", SF64, 1);
        e.r = e.g->field(k + "r", SFL, 1);
        e.p = e.g->field(k + "p", SFL, 1);
        e.t = e.g->field(k + "t", SFL, 1);
        e.v = e.g->field(k + "v", SFL, 1);
        e.w = e.g->field(k + "w", SFL, 1);
        e.xl = e.g->field(k + "xl", SFX, 1);
        e.a = 1.0 / (2.0 * e.kappa);
    }

    SysArray sys;
    sys.alloc(n, S[0].g->raw["cg.sys"]);
    for (int i = 0; i < n; i++) {
        CgSys& e = S[i];
        SysState& q = sys.h[i];
        std::memset(&q, 0, sizeof(q));
        q.partials = (double*)e.g->rawbuf("cg" + std::to_string(e.slot) + ".partials",
                                          sizeof(double) * NRED * (2 * e.g->geo.stride / BLOCK + 1));
        q.maxit = P.max_iter;
        q.mixed = P.mixed;
        q.delta_rel2 = P.delta_reliable * P.delta_reliable;
        q.dc = P.mixed && P.mixed_mode == WD_MIXED_DEFECT;
        q.target2 = -1.0;
        q.cga_prev = 1.0;
        q.status = ST_RUNNING;
    }
    sys.upload(st);

    JobTable<SweepJob> Nb, Bs, Acc, InitFirst, InitRel, InitRestart, SX, SP;
    JobTable<HopJob> Hx1, Hx2, Hx3, Hx4, H1, H2, H3, H4;
    std::vector<int> need_norm;
    for (int i = 0; i < n; i++) {
        CgSys& e = S[i];
        const Geo& g = e.g->geo;
        const void* d0 = e.g->slk(L64, 0);
        const void* d1 = e.g->slk(L64, 1);
        const void* l0 = e.g->slk(LFL, 0);
        const void* l1 = e.g->slk(LFL, 1);
        const long lcs = e.g->lcs();
        const double a2 = e.a * e.a;
        bool shared = false;
        for (int k = 0; k < i; k++) shared = shared || S[k].src.B64.base() == e.src.B64.base();
        if (e.be2 < 0 && !shared) {
            need_norm.push_back(i);
            SweepJob nj = sweep_job(i, e.RH.nsites());
            nj.f[R_F0] = e.src.B64.half(0);
            Nb.host.push_back(nj);
        }
        // RH = b_e - sigma x_e
        SweepJob sj = sweep_job(i, e.RH.nsites());
        sj.f[R_F0] = e.RH.all();
        sj.f[R_F1] = e.src.B64.half(0);
        sj.f[R_F2] = e.X64.half(0);
        sj.c[0] = 1.0;
        sj.c[1] = -e.sigma;
        Bs.host.push_back(sj);
        sj = sweep_job(i, e.xl.nsites());
        sj.f[R_F0] = e.X64.half(0);
        sj.f[R_F1] = e.xl.all();
        sj.flags = 1;
        Acc.host.push_back(sj);
        // FP64 residual: T64 = D_oe x ; V64 = M_prec x ; T64 = (D_eo)^dag V64 ;
        // RH <- RH - a^2 V64 + 1/4 (D_oe)^dag T64 = b_e - (A + sigma) x, |RH|^2
        Hx1.host.push_back(hop_job(g, 1, i, e.X64.half(0), e.T64.all(), d1, lcs, 1.0));
        HopJob j = hop_job(g, 0, i, e.T64.all(), e.V64.all(), d0, lcs, -0.25);
        j.x0 = e.X64.half(0);
        j.c0 = a2;
        Hx2.host.push_back(j);
        Hx3.host.push_back(hop_job(g, 1, i, e.V64.all(), e.T64.all(), d1, lcs, 1.0));
        j = hop_job(g, 0, i, e.T64.all(), e.RH.all(), d0, lcs, 0.25);
        j.x0 = e.RH.all();
        j.c0 = 1.0;
        j.x1 = e.V64.all();
        j.c1 = -a2;
        Hx4.host.push_back(j);
        // r_lo = r_hi (FP64 residual or, without a start vector, b_e); p = r; x_lo = 0; |r|^2
        sj = sweep_job(i, e.r.nsites());
        sj.f[R_F0] = e.r.all();
        sj.f[R_F1] = e.RH.all();
        sj.f[R_F2] = e.r.all();
        sj.f[R_F3] = e.p.all();
        sj.f[R_F4] = e.xl.all();
        sj.flags = 2 | 4;
        InitFirst.host.push_back(sj);
        sj.flags = 8;  // p = r + beta' p (beta' set by the host)
        InitRel.host.push_back(sj);
        sj.flags = 2;
        InitRestart.host.push_back(sj);
        // iteration: t = D_oe p ; v = M_prec p ; t = (D_eo)^dag v ; w = (A + sigma) p, <p, w> ;
        // x += alpha p, r -= alpha w, |r|^2 ; p = r + beta p
        H1.host.push_back(hop_job(g, 1, i, e.p.all(), e.t.all(), l1, lcs, 1.0));
        j = hop_job(g, 0, i, e.t.all(), e.v.all(), l0, lcs, -0.25);
        j.x0 = e.p.all();
        j.c0 = a2;
        H2.host.push_back(j);
        H3.host.push_back(hop_job(g, 1, i, e.v.all(), e.t.all(), l1, lcs, 1.0));
        j = hop_job(g, 0, i, e.t.all(), e.w.all(), l0, lcs, -0.25);
        j.x0 = e.v.all();
        j.c0 = a2;
        j.x1 = e.p.all();
        j.c1 = e.sigma;
        j.z = e.p.all();
        H4.host.push_back(j);
        sj = sweep_job(i, e.r.nsites());
        sj.f[R_F0] = e.xl.all();
        sj.f[R_F1] = e.p.all();
        sj.f[R_F2] = e.r.all();
        sj.f[R_F3] = e.w.all();
        SX.host.push_back(sj);
        sj = sweep_job(i, e.r.nsites());
        sj.f[R_F0] = e.p.all();
        sj.f[R_F1] = e.r.all();
        SP.host.push_back(sj);
    }
    for (auto* t : {&Hx1, &Hx2, &Hx3, &Hx4})
        for (auto& j : t->host) set_tile(j, tile_64[j.sys]);
    for (auto* t : {&H1, &H2, &H3, &H4})
        for (auto& j : t->host) {
            set_tile(j, tile_lo[j.sys]);
            j.rhs = rhs_lo;
        }
    // the forward hops skip the unit time links of a temporal-gauge handle; the adjoint hops read
    // every link (all of them are stored)
    for (auto* t : {&Hx1, &Hx2, &H1, &H2})
        for (auto& j : t->host) j.tg = S[j.sys].g->tg;
    for (auto* t : {&Hx1, &Hx2, &Hx3, &Hx4, &H1, &H2, &H3, &H4}) {
        for (auto& j : t->host) j.nc = S[j.sys].g->nc;  // every hop works in the handle's spin basis
        group_by_links(*t);
        layout(*t);
    }
    for (auto* t : {&Nb, &Bs, &Acc, &InitFirst, &InitRel, &InitRestart, &SX, &SP}) layout(*t);
    upload_tables(st, S[0].g->raw["cg.tables"],
                  {&Hx1, &Hx2, &Hx3, &Hx4, &H1, &H2, &H3, &H4, &Nb, &Bs, &Acc, &InitFirst, &InitRel, &InitRestart,
                   &SX, &SP});

    const double bl = spinor_site_bytes(SFL), bx = spinor_site_bytes(SFX);
    const double bHx1 = hop_bytes(Hx1, SF64, L64, 0), bHx2 = hop_bytes(Hx2, SF64, L64, 1),
                 bHx4 = hop_bytes(Hx4, SF64, L64, 2);
    auto residual = [&](int gate) {
        run_sweep(OP_AXPY, SF64, Bs, sys.d(), gate, st, sweep_bytes(Bs, 3 * 192));
        run_hop(SF64, L64, false, RED_NONE, FIN_STORE, Hx1, sys.d(), gate, st, bHx1);
        run_hop(SF64, L64, false, RED_NONE, FIN_STORE, Hx2, sys.d(), gate, st, bHx2);
        run_hop(SF64, L64, true, RED_NONE, FIN_STORE, Hx3, sys.d(), gate, st, bHx1);
        run_hop(SF64, L64, true, RED_NORM, FIN_STORE, Hx4, sys.d(), gate, st, bHx4);
    };

    // ---- setup: |b_e|^2 (one round trip, skipped when the caller knows it), start residual
    if (!need_norm.empty()) {
        run_sweep(OP_NORM, SF64, Nb, sys.d(), 0, st, sweep_bytes(Nb, 192));
        sys.download(st);
        for (int i : need_norm) S[i].be2 = sys.h[i].red[2];
        for (int i = 0; i < n; i++)
            for (int k : need_norm)
                if (S[i].be2 < 0 && S[i].src.B64.base() == S[k].src.B64.base()) S[i].be2 = S[k].be2;
    }
    bool any_x0 = false;
    for (auto& e : S) {
        // the odd half stays zero: the solution lives on the even sites
        if (!e.x_ready) WD_CHECK_HIP(hipMemsetAsync(e.X64.base(), 0, e.X64.mem->bytes, st));
        any_x0 = any_x0 || e.x_ready;
    }
    WD_REQUIRE(n == 1 || !S[0].r_ready, "a prepared start residual is for single-system solves");
    if (any_x0 && !S[0].r_ready) residual(0);
    for (int i = 0; i < n; i++) {
        CgSys& e = S[i];
        sys.h[i].target2 = P.tol * P.tol * e.be2;
        sys.h[i].status = ST_RUNNING;
        if (e.be2 == 0.0) {  // zero source: x = 0
            e.done = true;
            e.rr_true = 0;
            sys.h[i].status = ST_DONE;
            WD_CHECK_HIP(hipMemsetAsync(e.X64.base(), 0, e.X64.mem->bytes, st));
        }
    }
    sys.upload(st);
    if (!any_x0) {
        for (auto& j : InitFirst.host) j.f[R_F1] = S[j.sys].src.B64.half(0);
        InitFirst.upload(st);
    }
    run_sweep(OP_INIT, SFL, InitFirst, sys.d(), GATE_RUN, st, init_bytes(InitFirst, SFL));
    for (int i = 0; i < n; i++) S[i].t0 = t_start;

    const double bH = hop_bytes(H1, SFL, LFL, 0), bH2 = hop_bytes(H2, SFL, LFL, 1), bH4 = hop_bytes(H4, SFL, LFL, 2);
    const double bSX = sweep_bytes(SX, 2 * bx + 4 * bl), bSP = sweep_bytes(SP, 3 * bl);
    auto iterate = [&](hipStream_t q) {
        run_hop(SFL, LFL, false, RED_NONE, FIN_STORE, H1, sys.d(), GATE_RUN, q, bH);
        run_hop(SFL, LFL, false, RED_NONE, FIN_STORE, H2, sys.d(), GATE_RUN, q, bH2);
        run_hop(SFL, LFL, true, RED_NONE, FIN_STORE, H3, sys.d(), GATE_RUN, q, bH);
        run_hop(SFL, LFL, true, RED_ZDOT, FIN_CGA, H4, sys.d(), GATE_RUN, q, bH4);
        run_sweep(OP_CGX, SFL, SX, sys.d(), GATE_RUN, q, bSX);
        run_sweep(OP_CGP, SFL, SP, sys.d(), GATE_RUN, q, bSP);
    };
    std::shared_ptr<ChunkGraph> graph;
    if (graphs_on())
        graph = cached_graph(S[0].g, launch_key("cg", poll, SFL, LFL, sys.d(), H1, H2, H3, H4, SX, SP),
                             [&](hipStream_t q) {
                                 for (int k = 0; k < poll; k++) iterate(q);
                             });
    // Reliable update of the systems that stopped (gate GATE_STOPPED). The p update of the
    // iteration in which a system stopped was gated off, so p is still p_n; a continuing system
    // takes the new search direction from the true residual, p = r_true + (|r_true|^2 / |r_n|^2) p_n,
    // as if the iteration had produced r_true (keeping p_{n+1} = r_iter + beta p_n instead makes
    // alpha overshoot once the true residual exceeds the iterated one, and the iteration diverges)
    auto reliable_update = [&]() {
        run_sweep(OP_ACC, SFL, Acc, sys.d(), GATE_STOPPED, st, sweep_bytes(Acc, 2 * 192 + 2 * bx));
        residual(GATE_STOPPED);
    };

    int active = 0;
    for (auto& e : S) active += !e.done;
    long host_iters = 0;
    const long host_cap = (long)P.max_iter + 16L * poll + 64;
    while (active > 0) {
        if (graph) graph->launch(st);
        else
            for (int k = 0; k < poll; k++) iterate(st);
        host_iters += poll;
        sys.download(st);
        if (host_iters > host_cap) {
            for (auto& e : S)
                if (!e.done) {
                    e.done = true;
                    e.final_status = WD_ERR_NOCONV;
                    e.t1 = now_s();
                }
            break;
        }
        bool any = false;
        for (int i = 0; i < n; i++) {
            const int stt = sys.h[i].status;
            if (S[i].done || stt == ST_RUNNING) continue;
            if (stt == ST_NAN) {
                S[i].done = true;
                S[i].final_status = WD_ERR_NAN;
                S[i].t1 = now_s();
                active--;
                continue;
            }
            any = true;
        }
        if (!any) continue;
        reliable_update();
        sys.download(st);
        bool any_next = false, any_fresh = false;
        for (int i = 0; i < n; i++) {
            CgSys& e = S[i];
            SysState& q = sys.h[i];
            const int stt = q.status;
            if (e.done || stt == ST_RUNNING || stt == ST_NAN) continue;
            e.reliable++;
            const double rr = q.red[2];
            e.rr_true = rr;
            // continue (p from the true residual) while the true residual stays within a factor 2 in
            // |r|^2 of the iterated one (q.rr); otherwise, and after a failed exit check (the
            // iterated residual met the tolerance, the true one did not), restart with p = r
            int next = (stt == ST_RELIABLE && rr <= 2.0 * q.rr && q.rr > 0 && q.cgb > 0) ? ST_SEL1 : ST_SEL2;
            if (next == ST_SEL1) q.cgb = rr * q.cgb / q.rr;  // |r_true|^2 / |r_n|^2, |r_n|^2 = q.rr / q.cgb
            if (!std::isfinite(rr)) {
                e.done = true;
                e.final_status = WD_ERR_NAN;
            } else if (rr <= q.target2) {
                e.done = true;
                e.final_status = WD_OK;
            } else if (stt == ST_MAXIT || q.iter >= q.maxit) {
                e.done = true;
                e.final_status = WD_ERR_NOCONV;
            } else if (stt == ST_BREAKDOWN) {
                if (++e.restarts > 2) {
                    e.done = true;
                    e.final_status = WD_ERR_BREAKDOWN;
                } else {
                    next = ST_SEL2;  // restart with p = r
                }
            }
            if (!e.done && P.mixed && P.mixed_mode == WD_MIXED_DEFECT) next = ST_SEL2;
            if (e.done) {
                e.t1 = now_s();
                active--;
                q.status = ST_DONE;
            } else {
                q.status = next;
                any_next = any_next || next == ST_SEL1;
                any_fresh = any_fresh || next == ST_SEL2;
            }
        }
        sys.upload(st);
        if (any_next) run_sweep(OP_INIT, SFL, InitRel, sys.d(), 1 << ST_SEL1, st, init_bytes(InitRel, SFL));
        if (any_fresh) run_sweep(OP_INIT, SFL, InitRestart, sys.d(), 1 << ST_SEL2, st, init_bytes(InitRestart, SFL));
    }

    for (auto& e : S)
        WD_CHECK_HIP(launch_unpack_spinor(SF64, e.x, e.g->geo, e.X64.half(0), e.X64.half(1), 0, 1.0, st, e.g->gm(), e.g->nc));
    sys.download(st);
    for (int i = 0; i < n; i++) {
        CgSys& e = S[i];
        if (e.t1 == 0) e.t1 = now_s();
        e.iters = sys.h[i].iter;
        if (!std::isfinite(e.be2) || e.final_status == WD_ERR_NAN) e.true_rel = std::nan("");
        else e.true_rel = (e.be2 > 0 && e.rr_true >= 0) ? std::sqrt(e.rr_true / e.be2) : 0.0;
    }
}

// CG-M in FP64 for all shifts at once; the base is the smallest shift (the slowest to converge),
// the others are frozen once their residual |zeta| |r| meets the tolerance.
static wd_status cgm_solve(wd_gauge* g, double kappa, int n, const double* sigmas, double* const* x, const double* b,
                           const wd_solver_params& P, wd_solver_stats* stats, hipStream_t st, int poll)
{
    const double t0 = now_s();
    int base = 0;
    for (int i = 1; i < n; i++)
        if (sigmas[i] < sigmas[base]) base = i;
    const double a = 1.0 / (2.0 * kappa), a2 = a * a, s0 = sigmas[base];
    const int ns = n - 1;
    std::vector<int> shift_of(n, -1), sys_of_shift;
    for (int i = 0; i < n; i++)
        if (i != base) {
            shift_of[i] = (int)sys_of_shift.size();
            sys_of_shift.push_back(i);
        }
    const Geo& geo = g->geo;
    const int L64 = g->f64_links();
    g->ensure_slinks(L64, st);
    Field B = g->field("cgm.B", SF64, 2);
    std::vector<Field> X(n), PS(ns);
    for (int i = 0; i < n; i++) X[i] = g->field("cgm.X" + std::to_string(i), SF64, 2);
    for (int k = 0; k < ns; k++) PS[k] = g->field("cgm.P" + std::to_string(k), SF64, 1);
    Field R = g->field("cgm.r", SF64, 1), Pb = g->field("cgm.p", SF64, 1), Tm = g->field("cgm.t", SF64, 1);
    Field Vm = g->field("cgm.v", SF64, 1), Wm = g->field("cgm.w", SF64, 1);
    for (int i = 0; i < n; i++) WD_CHECK_HIP(hipMemsetAsync(X[i].base(), 0, X[i].mem->bytes, st));
    WD_CHECK_HIP(launch_pack_spinor(SF64, b, geo, B.half(0), B.half(1), 0, 1.0, st, g->gm(), g->nc));

    SysArray sys;
    sys.alloc(1, g->raw["cgm.sys"]);
    SysState& q = sys.h[0];
    std::memset(&q, 0, sizeof(q));
    q.partials = (double*)g->rawbuf("cgm.partials", sizeof(double) * NRED * (2 * geo.stride / BLOCK + 1));
    q.maxit = P.max_iter;
    q.nshift = ns;
    q.target2 = -1;
    q.cga_prev = 1.0;
    std::vector<ShiftScal> sh(std::max(ns, 1));
    std::vector<SpinorRef> shv(2 * std::max(ns, 1));
    for (int k = 0; k < ns; k++) {
        ShiftScal& z = sh[k];
        std::memset(&z, 0, sizeof(z));
        z.sigma = sigmas[sys_of_shift[k]] - s0;
        z.zeta_prev = z.zeta = make_double2(1.0, 0.0);
        z.active = 1;
        shv[2 * k] = X[sys_of_shift[k]].half(0);
        shv[2 * k + 1] = PS[k].all();
    }
    ShiftScal* d_sh = (ShiftScal*)g->rawbuf("cgm.sh", sizeof(ShiftScal) * sh.size());
    SpinorRef* d_shv = (SpinorRef*)g->rawbuf("cgm.shv", sizeof(SpinorRef) * shv.size());
    {
        const size_t n1 = sizeof(ShiftScal) * sh.size(), n2 = sizeof(SpinorRef) * shv.size();
        char* stg = stage_alloc(n1 + n2);
        std::memcpy(stg, sh.data(), n1);
        std::memcpy(stg + n1, shv.data(), n2);
        WD_CHECK_HIP(hipMemcpyAsync(d_sh, stg, n1, hipMemcpyHostToDevice, st));
        WD_CHECK_HIP(hipMemcpyAsync(d_shv, stg + n1, n2, hipMemcpyHostToDevice, st));
    }
    q.sh = d_sh;
    q.shv = d_shv;
    sys.upload(st);

    const long nh = R.nsites();
    JobTable<SweepJob> Init, SX, SP;
    SweepJob j = sweep_job(0, nh);
    // r = p = b_e, x = 0, x^s = 0, p^s = b_e, |b_e|^2
    j.f[R_F0] = R.all();
    j.f[R_F1] = B.half(0);
    j.f[R_F2] = Pb.all();
    j.f[R_F3] = Pb.all();
    j.f[R_F4] = X[base].half(0);
    Init.host.push_back(j);
    j = sweep_job(0, nh);
    j.f[R_F0] = X[base].half(0);
    j.f[R_F1] = Pb.all();
    j.f[R_F2] = R.all();
    j.f[R_F3] = Wm.all();
    SX.host.push_back(j);
    j = sweep_job(0, nh);
    j.f[R_F0] = Pb.all();
    j.f[R_F1] = R.all();
    SP.host.push_back(j);
    JobTable<HopJob> H1, H2, H3, H4;
    {
        const void* d0 = g->slk(L64, 0);
        const void* d1 = g->slk(L64, 1);
        const long lcs = g->lcs();
        HopJob h = hop_job(geo, 1, 0, Pb.all(), Tm.all(), d1, lcs, 1.0);
        h.tg = g->tg;
        h.nc = g->nc;
        H1.host.push_back(h);
        h = hop_job(geo, 0, 0, Tm.all(), Vm.all(), d0, lcs, -0.25);
        h.tg = g->tg;
        h.nc = g->nc;
        h.x0 = Pb.all();
        h.c0 = a2;
        H2.host.push_back(h);
        H3.host.push_back(hop_job(geo, 1, 0, Vm.all(), Tm.all(), d1, lcs, 1.0));
        h = hop_job(geo, 0, 0, Tm.all(), Wm.all(), d0, lcs, -0.25);
        h.x0 = Vm.all();
        h.c0 = a2;
        h.x1 = Pb.all();
        h.c1 = s0;
        h.z = Pb.all();
        H4.host.push_back(h);
    }
    const int tz64 = tune_tile(g, SF64, L64, st);
    for (auto* t : {&H1, &H2, &H3, &H4}) {
        for (auto& h : t->host) {
            set_tile(h, tz64);
            h.nc = g->nc;  // the adjoint hops too work in the handle's spin basis
        }
        layout(*t);
    }
    for (auto* t : {&Init, &SX, &SP}) layout(*t);
    upload_tables(st, g->raw["cgm.tables"], {&Init, &SX, &SP, &H1, &H2, &H3, &H4});
    run_sweep(OP_MSINIT, SF64, Init, sys.d(), 0, st, sweep_bytes(Init, (4 + 2 * ns) * 192.0));
    sys.download(st);
    const double bb = sys.h[0].red[2];
    sys.h[0].target2 = P.tol * P.tol * bb;
    sys.h[0].shift_target2 = P.tol * P.tol * bb;
    sys.h[0].cga_prev = 1.0;
    sys.h[0].cgb = 0.0;
    if (bb == 0.0) sys.h[0].status = ST_CONVERGED;
    sys.upload(st);

    const double bH = hop_bytes(H1, SF64, L64, 0);
    auto iterate = [&](int active_shifts, hipStream_t qs) {
        run_hop(SF64, L64, false, RED_NONE, FIN_STORE, H1, sys.d(), GATE_RUN, qs, bH);
        run_hop(SF64, L64, false, RED_NONE, FIN_STORE, H2, sys.d(), GATE_RUN, qs, bH + nh * 192.0);
        run_hop(SF64, L64, true, RED_NONE, FIN_STORE, H3, sys.d(), GATE_RUN, qs, bH);
        run_hop(SF64, L64, true, RED_ZDOT, FIN_CGA, H4, sys.d(), GATE_RUN, qs, bH + nh * 2 * 192.0);
        run_sweep(OP_CGX, SF64, SX, sys.d(), GATE_RUN, qs, sweep_bytes(SX, 6 * 192));
        run_sweep(ns > 0 ? OP_CGPM : OP_CGP, SF64, SP, sys.d(), GATE_RUN, qs,
                  sweep_bytes(SP, 3 * 192 + 4 * 192 * active_shifts));
    };
    std::shared_ptr<ChunkGraph> graph;
    if (graphs_on())
        graph = cached_graph(g, launch_key("cgm", poll, ns, 0, sys.d(), H1, H2, H3, H4, SX, SP), [&](hipStream_t qs) {
            for (int k = 0; k < poll; k++) iterate(ns, qs);
        });
    auto fetch_shifts = [&]() {
        if (ns == 0) return;
        const size_t n1 = sizeof(ShiftScal) * ns;
        void* stg = pinned(n1);
        WD_CHECK_HIP(hipMemcpyAsync(stg, d_sh, n1, hipMemcpyDeviceToHost, st));
        WD_CHECK_HIP(hipStreamSynchronize(st));
        std::memcpy(sh.data(), stg, n1);
    };
    int active_shifts = ns;
    long host_iters = 0;
    const long host_cap = (long)P.max_iter + 16L * poll + 64;
    while (sys.h[0].status == ST_RUNNING && host_iters <= host_cap) {
        if (graph) graph->launch(st);
        else
            for (int k = 0; k < poll; k++) iterate(active_shifts, st);
        host_iters += poll;
        sys.download(st);
        fetch_shifts();
        active_shifts = 0;
        for (int k = 0; k < ns; k++) active_shifts += sh[k].active;
    }
    int status;
    switch (sys.h[0].status) {
    case ST_CONVERGED: status = WD_OK; break;
    case ST_MAXIT: status = WD_ERR_NOCONV; break;
    case ST_BREAKDOWN: status = WD_ERR_BREAKDOWN; break;
    case ST_NAN: status = WD_ERR_NAN; break;
    default: status = WD_ERR_NOCONV;
    }
    fetch_shifts();
    const int iters = sys.h[0].iter;
    const double t1 = now_s();

    // true residual b_e - (A + sigma_i) x_i of every system, one launch per step for all of them
    // (one reduction group per system; the residual fields are not kept), then unpack
    {
        const size_t pstride = (size_t)NRED * (2 * geo.stride / BLOCK + 1);
        SysArray rs;
        rs.alloc(n, g->raw["cgm.rsys"]);
        double* rpart = (double*)g->rawbuf("cgm.rpartials", sizeof(double) * pstride * n);
        for (int i = 0; i < n; i++) {
            std::memset(&rs.h[i], 0, sizeof(SysState));
            rs.h[i].partials = rpart + pstride * i;
        }
        std::vector<Field> RT(n), RV(n), RR(n);
        for (int i = 0; i < n; i++) {
            RT[i] = g->field("cgm.RT" + std::to_string(i), SF64, 1);
            RV[i] = g->field("cgm.RV" + std::to_string(i), SF64, 1);
            RR[i] = g->field("cgm.RR" + std::to_string(i), SF64, 1);
        }
        JobTable<SweepJob> Bs;
        JobTable<HopJob> Q1, Q2, Q3, Q4;
        const void* d0 = g->slk(L64, 0);
        const void* d1 = g->slk(L64, 1);
        const long lcs = g->lcs();
        for (int i = 0; i < n; i++) {
            SweepJob sj = sweep_job(i, nh);
            sj.f[R_F0] = RR[i].all();
            sj.f[R_F1] = B.half(0);
            sj.f[R_F2] = X[i].half(0);
            sj.c[0] = 1.0;
            sj.c[1] = -sigmas[i];
            Bs.host.push_back(sj);
            HopJob h = hop_job(geo, 1, i, X[i].half(0), RT[i].all(), d1, lcs, 1.0);
            h.tg = g->tg;
            h.nc = g->nc;
            Q1.host.push_back(h);
            h = hop_job(geo, 0, i, RT[i].all(), RV[i].all(), d0, lcs, -0.25);
            h.tg = g->tg;
            h.nc = g->nc;
            h.x0 = X[i].half(0);
            h.c0 = a2;
            Q2.host.push_back(h);
            Q3.host.push_back(hop_job(geo, 1, i, RV[i].all(), RT[i].all(), d1, lcs, 1.0));
            h = hop_job(geo, 0, i, RT[i].all(), RR[i].all(), d0, lcs, 0.25);
            h.x0 = RR[i].all();
            h.c0 = 1.0;
            h.x1 = RV[i].all();
            h.c1 = -a2;
            Q4.host.push_back(h);
        }
        for (auto* t : {&Q1, &Q2, &Q3, &Q4}) {
            for (auto& h : t->host) {
                set_tile(h, tz64);
                h.nc = g->nc;
            }
            layout(*t);
        }
        layout(Bs);
        upload_tables(st, g->raw["cgm.rtables"], {&Bs, &Q1, &Q2, &Q3, &Q4});
        rs.upload(st);
        run_sweep(OP_AXPY, SF64, Bs, rs.d(), 0, st, sweep_bytes(Bs, 3 * 192.0));
        run_hop(SF64, L64, false, RED_NONE, FIN_STORE, Q1, rs.d(), 0, st, hop_bytes(Q1, SF64, L64, 0));
        run_hop(SF64, L64, false, RED_NONE, FIN_STORE, Q2, rs.d(), 0, st, hop_bytes(Q2, SF64, L64, 1));
        run_hop(SF64, L64, true, RED_NONE, FIN_STORE, Q3, rs.d(), 0, st, hop_bytes(Q3, SF64, L64, 0));
        run_hop(SF64, L64, true, RED_NORM, FIN_STORE, Q4, rs.d(), 0, st, hop_bytes(Q4, SF64, L64, 2));
        for (int i = 0; i < n; i++)
            WD_CHECK_HIP(launch_unpack_spinor(SF64, x[i], geo, X[i].half(0), X[i].half(1), 0, 1.0, st, g->gm(), g->nc));
        rs.download(st);
        if (stats)
            for (int i = 0; i < n; i++) {
                stats[i].iters = i == base ? iters : (sh[shift_of[i]].active ? iters : sh[shift_of[i]].conv_iter);
                stats[i].reliable_updates = 0;
                stats[i].true_rel_res = !std::isfinite(bb) ? std::nan("") : bb > 0 ? std::sqrt(rs.h[i].red[2] / bb) : 0.0;
                stats[i].status = status;
                stats[i].seconds = t1 - t0;
            }
    }
    return (wd_status)status;
}

wd_status solve_normal(wd_gauge* g, double kappa, int n, const double* sigmas, double* const* x, const double* b,
                       int method, int guess, const wd_solver_params& P, wd_solver_stats* stats, hipStream_t st)
{
    WD_REQUIRE(n >= 1 && n <= 32, "number of shifts must be in 1..32");
    WD_REQUIRE(kappa > 0, "kappa must be positive");
    for (int i = 0; i < n; i++) WD_REQUIRE(std::isfinite(sigmas[i]) && sigmas[i] >= 0, "shifts must be >= 0");
    WD_REQUIRE(P.dagger == 0, "the normal equations take dagger = 0");
    WD_REQUIRE(guess == WD_GUESS_NONE || guess == WD_GUESS_POLY, "normal equations: guess must be NONE or POLY");
    if (method == WD_METHOD_MULTISHIFT) return cgm_solve(g, kappa, n, sigmas, x, b, P, stats, st, kPoll);
    WD_REQUIRE(method == WD_METHOD_SEQUENTIAL || method == WD_METHOD_BATCHED, "unknown method");
    auto fill = [&](int i, const CgSys& e, wd_status& worst) {
        if (stats) {
            stats[i].iters = e.iters;
            stats[i].reliable_updates = e.reliable;
            stats[i].status = e.final_status;
            stats[i].true_rel_res = e.true_rel;
            stats[i].seconds = e.t1 - e.t0;
        }
        if (e.final_status != WD_OK && worst == WD_OK) worst = (wd_status)e.final_status;
    };
    EoSource src;
    prepare_source(g, "nm.", b, 0, src, st);
    wd_status worst = WD_OK;
    auto make = [&](int i) {
        CgSys e;
        e.g = g;
        e.kappa = kappa;
        e.sigma = sigmas[i];
        e.b = b;
        e.x = x[i];
        e.src = src;
        return e;
    };
    if (method == WD_METHOD_BATCHED) {
        // all shifts iterate together, one launch per solver step (no start guesses)
        std::vector<CgSys> S;
        for (int i = 0; i < n; i++) {
            S.push_back(make(i));
            S.back().slot = i;
        }
        cg_solve(S, P, st, kPoll);
        for (int i = 0; i < n; i++) fill(i, S[i], worst);
        return worst;
    }
    // largest shift (best conditioned) first; each start vector is the Lagrange extrapolation in
    // sigma of the solutions found so far (the analogue of Sec. 6.2.1 and Sec. 7)
    std::vector<int> order(n);
    for (int i = 0; i < n; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int p, int q) { return sigmas[p] > sigmas[q]; });
    // every shift keeps its FP64 solution and its final FP64 residual for the later start vectors
    std::vector<Field> X(n), R(n);
    for (int i = 0; i < n; i++) {
        X[i] = g->field("nm.X" + std::to_string(i), SF64, 2);
        R[i] = g->field("nm.R" + std::to_string(i), SF64, 1);
    }
    std::vector<char> res_ok(n, 0);
    SysState* dummy = (SysState*)g->rawbuf("apply.sys", sizeof(SysState));
    std::vector<int> done;
    double be2 = -1;
    for (int idx : order) {
        CgSys e = make(idx);
        e.slot = 0;
        e.X64 = X[idx];
        e.RH = R[idx];
        e.be2 = be2;
        const int kall = (int)done.size();
        const int k = P.guess_order > 0 ? std::min(P.guess_order, kall) : kall;
        const int j_first = kall - k;
        if (guess == WD_GUESS_POLY && k > 0) {
            // Lagrange weights over the distinct shifts among the previous ones (the latest
            // solution of a repeated shift); a shift solved before is its own guess
            const double s = sigmas[idx];
            std::vector<bool> use(k, true);
            int same = -1;
            for (int jj = 0; jj < k; jj++) {
                const double sj = sigmas[done[j_first + jj]];
                for (int ii = jj + 1; ii < k; ii++)
                    if (sigmas[done[j_first + ii]] == sj) use[jj] = false;
                if (use[jj] && sj == s) same = jj;
            }
            std::vector<double> c(k, 0.0);
            for (int jj = 0; jj < k; jj++) {
                if (same >= 0) c[jj] = jj == same ? 1.0 : 0.0;
                else if (use[jj]) {
                    const double sj = sigmas[done[j_first + jj]];
                    double w = 1.0;
                    for (int ii = 0; ii < k; ii++) {
                        if (ii == jj || !use[ii]) continue;
                        const double si = sigmas[done[j_first + ii]];
                        w *= (s - si) / (sj - si);
                    }
                    c[jj] = w;
                }
            }
            WD_CHECK_HIP(hipMemsetAsync(X[idx].base(), 0, X[idx].mem->bytes, st));
            bool fused = true;
            for (int jj = 0; jj < k; jj++)
                if (c[jj] != 0.0 && !res_ok[done[j_first + jj]]) fused = false;
            // x0 = sum_j c_j x_j and, since (A + s_j) x_j = b_e - r_j, its residual
            // b_e - (A + s) x0 = (1 - sum c_j) b_e + sum_j c_j (s_j - s) x_j + sum_j c_j r_j in one
            // pass over the stored solutions and residuals (k_guess; no operator application)
            double sum_c = 0.0;
            for (int jj = 0; jj < k; jj++) sum_c += c[jj];
            for (int j0 = 0; j0 < k && fused; j0 += GUESS_MAX) {
                GuessArgs A;
                std::memset(&A, 0, sizeof(A));
                A.x0 = X[idx].half(0);
                A.r0 = R[idx].all();
                A.n = R[idx].nsites();
                A.acc = j0 > 0;
                if (j0 == 0) {
                    A.be = e.src.B64.half(0);
                    A.cb = 1.0 - sum_c;
                }
                A.k = std::min(GUESS_MAX, k - j0);
                for (int jj = 0; jj < A.k; jj++) {
                    const int j = done[j_first + j0 + jj];
                    A.xs[jj] = X[j].half(0);
                    A.rs[jj] = R[j].all();
                    A.c[jj] = c[j0 + jj];
                    A.cx[jj] = c[j0 + jj] * (sigmas[j] - s);
                }
                WD_CHECK_HIP(launch_guess(A, st));
            }
            if (fused) e.r_ready = true;
            // otherwise x0 = sum_j c_j x_j over the even half (7 inputs per sweep), and the solver
            // computes its residual with the FP64 operator
            for (int j0 = 0; j0 < k && !fused; j0 += 7) {
                JobTable<SweepJob> L;
                SweepJob sj = sweep_job(0, X[idx].stride);
                sj.f[R_F0] = X[idx].half(0);
                const int mc = std::min(7, k - j0);
                for (int jj = 0; jj < mc; jj++) {
                    sj.f[1 + jj] = X[done[j_first + j0 + jj]].half(0);
                    sj.c[jj] = c[j0 + jj];
                }
                sj.flags = (mc << 8) | (j0 > 0 ? 1 : 0);
                L.host.push_back(sj);
                layout(L);
                upload_tables(st, g->raw["nm.tables"], {&L});
                run_sweep(OP_LINCOMB, SF64, L, dummy, 0, st, sweep_bytes(L, (mc + 1 + (j0 > 0)) * 192.0));
            }
            e.x_ready = true;
        }
        std::vector<CgSys> S{e};
        cg_solve(S, P, st, kPoll);
        be2 = S[0].be2;
        fill(idx, S[0], worst);
        res_ok[idx] = S[0].final_status == WD_OK && S[0].reliable > 0;
        done.push_back(idx);
    }
    return worst;
}

} // namespace wd
