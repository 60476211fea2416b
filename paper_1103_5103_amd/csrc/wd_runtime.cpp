// Runtime pieces of libwdirac: device memory, workspace fields, link preparation, job-table
// upload, launch helpers with optional HIP-event timing, and the thread-local error message.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "wd_host.hpp"

namespace wd {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
const std::string& last_error() { return g_last_error; }

DevMem::DevMem(size_t n) : bytes(n)
{
    if (n == 0) return;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        throw Error{WD_ERR_OOM, "hipMalloc of " + std::to_string(n) + " bytes failed"};
    }
}
DevMem::~DevMem()
{
    if (p) (void)hipFree(p);
}

size_t field_bytes(int sf, int halves, long stride)
{
    size_t n = (size_t)16 * spinor_chunks(sf) * halves * stride;
    if (sf == SF16) n += (size_t)4 * halves * stride;
    return n;
}

int spinor_fmt_of(wd_prec p)
{
    switch (p) {
    case WD_F64: return SF64;
    case WD_F32: return SF32;
    case WD_F16: return SF16;
    default: throw Error{WD_ERR_UNSUPPORTED, "spinor storage must be F64, F32 or F16"};
    }
}

int link_fmt_of(wd_prec p, int recon)
{
    if (recon != 8 && recon != 12 && recon != 18) throw Error{WD_ERR_ARG, "recon must be 8, 12 or 18"};
    if (recon == 8) {
        if (p != WD_F16) throw Error{WD_ERR_UNSUPPORTED, "8-real links are stored in FP16 only"};
        return L16_8;
    }
    if (p == WD_F64) return recon == 12 ? L64_12 : L64_18;
    if (recon == 18) throw Error{WD_ERR_UNSUPPORTED, "18-real links are stored in FP64 only"};
    switch (p) {
    case WD_F32: return L32_12;
    case WD_F16: return L16_12;
    case WD_BF16: return LB16_12;
    default: throw Error{WD_ERR_ARG, "bad link precision"};
    }
}

// ---------------------------------------------------------------- pinned staging
void* pinned(size_t bytes)
{
    static std::mutex mu;
    static void* buf = nullptr;
    static size_t cap = 0;
    std::lock_guard<std::mutex> lk(mu);
    if (bytes > cap) {
        if (buf) (void)hipHostFree(buf);
        size_t n = std::max(bytes, (size_t)1 << 20);
        WD_CHECK_HIP(hipHostMalloc(&buf, n, hipHostMallocDefault));
        cap = n;
    }
    return buf;
}

// ---------------------------------------------------------------- timing
Timer& timer()
{
    static Timer t;
    return t;
}
hipEvent_t Timer::get()
{
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    // The events only time: they are read after a device synchronisation, so they skip the
    // system-scope fence (an L2 writeback and invalidate) that a default event performs, which
    // would otherwise cost each timed launch its L2 contents and add to its measured duration.
    hipEvent_t e;
    WD_CHECK_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    return e;
}
int* Timer::slot()
{
    if (!dflags) {
        cap = 1 << 16;
        WD_CHECK_HIP(hipMalloc(&dflags, cap * sizeof(int)));
        WD_CHECK_HIP(hipMemset(dflags, 0, cap * sizeof(int)));
    }
    if (pending.size() >= cap) flush();
    return dflags + pending.size();
}

// Launches that every system skipped (gated iterations after convergence) are not counted:
// their kernels ran for a few microseconds and moved no data. A launch in which only some jobs
// ran is credited that fraction of its bytes (exact when the jobs have equal sizes).
void Timer::flush()
{
    if (pending.empty()) return;
    std::vector<int> done(pending.size(), 1);
    WD_CHECK_HIP(hipDeviceSynchronize());
    if (dflags) {
        WD_CHECK_HIP(hipMemcpy(done.data(), dflags, done.size() * sizeof(int), hipMemcpyDeviceToHost));
        WD_CHECK_HIP(hipMemset(dflags, 0, done.size() * sizeof(int)));
    }
    for (size_t k = 0; k < pending.size(); k++) {
        Rec& r = pending[k];
        if (r.slot < 0 || done[k]) {
            float t = 0;
            WD_CHECK_HIP(hipEventElapsedTime(&t, r.a, r.b));
            ms[r.cls] += t;
            const double frac = (r.slot < 0 || r.njobs <= 0) ? 1.0 : std::min(1.0, (double)done[k] / r.njobs);
            bytes[r.cls] += r.bytes * frac;
            launches[r.cls] += 1;
            if (r.cls2 >= 0) {
                ms[r.cls2] += t;
                bytes[r.cls2] += r.bytes * frac;
                launches[r.cls2] += 1;
            }
        }
        pool.push_back(r.a);
        pool.push_back(r.b);
    }
    pending.clear();
}

// Pinned staging for job tables: chunks are handed out in order and the arena is recycled only
// after the device has drained (one device synchronisation per wrap-around), so uploads do not
// wait for the stream.
char* stage_alloc(size_t n)
{
    static std::mutex mu;
    static char* buf = nullptr;
    static size_t cap = 0, off = 0;
    std::lock_guard<std::mutex> lk(mu);
    n = (n + 255) / 256 * 256;
    if (!buf) {
        cap = (size_t)32 << 20;
        WD_CHECK_HIP(hipHostMalloc((void**)&buf, cap, hipHostMallocDefault));
    }
    if (n > cap) throw Error{WD_ERR_ARG, "job table too large"};
    if (off + n > cap) {
        WD_CHECK_HIP(hipDeviceSynchronize());
        off = 0;
    }
    char* p = buf + off;
    off += n;
    return p;
}

static int job_blocks_factor(const HopJob& j) { return j.ilv > 1 && j.rhs < 2 ? j.ilv : 1; }
static int job_blocks_factor(const SweepJob&) { return 1; }

template <class J>
size_t JobTable<J>::prepare()
{
    // finisher list: the systems of this launch in order of first appearance
    fin.clear();
    for (auto& j : host) {
        bool seen = false;
        for (auto& f : fin) seen = seen || f.sys == j.sys;
        if (!seen) fin.push_back(FinJob{j.sys, j.rnblk});
    }
    nblocks = 0;
    for (auto& j : host) nblocks = std::max<long>(nblocks, (long)j.blk0 + (long)j.nblk * job_blocks_factor(j));
    return (fin_offset() + fin.size() * sizeof(FinJob) + 255) / 256 * 256;
}

template <class J>
void JobTable<J>::write(char* dst) const
{
    std::memcpy(dst, host.data(), host.size() * sizeof(J));
    std::memcpy(dst + fin_offset(), fin.data(), fin.size() * sizeof(FinJob));
}

template <class J>
void JobTable<J>::upload(hipStream_t s)
{
    // in place when the table's slot is large enough (also inside a buffer shared with other
    // tables), else into a buffer of its own
    const size_t n = prepare();
    if (!dev || n > cap) {
        dev = std::make_shared<DevMem>(std::max(n, sizeof(J)));
        off = 0;
        cap = std::max(n, sizeof(J));
    }
    char* stage = stage_alloc(n);
    write(stage);
    WD_CHECK_HIP(hipMemcpyAsync((char*)dev->p + off, stage, n, hipMemcpyHostToDevice, s));
}

void upload_tables(hipStream_t s, std::shared_ptr<DevMem>& mem, std::initializer_list<JobTableBase*> tables)
{
    size_t total = 0;
    std::vector<size_t> offs;
    for (JobTableBase* t : tables) {
        offs.push_back(total);
        total += t->prepare();
    }
    if (total == 0) return;
    if (!mem || mem->bytes < total) mem = std::make_shared<DevMem>(total);
    char* stage = stage_alloc(total);
    size_t k = 0;
    for (JobTableBase* t : tables) {
        t->write(stage + offs[k]);
        t->dev = mem;
        t->off = offs[k];
        t->cap = (k + 1 < offs.size() ? offs[k + 1] : total) - offs[k];
        k++;
    }
    WD_CHECK_HIP(hipMemcpyAsync(mem->p, stage, total, hipMemcpyHostToDevice, s));
}
template struct JobTable<HopJob>;
template struct JobTable<SweepJob>;

template <class J>
static void run_finish(int nr, int fin, const JobTable<J>& t, SysState* sys, int gated, hipStream_t s)
{
    Timer& T = timer();
    // a timed launch passes its events to the launch, which records the kernel's own start and end
    const bool timed = T.on && !t.fin.empty();
    hipEvent_t a = nullptr, b = nullptr;
    if (timed) {
        a = T.get();
        b = T.get();
    }
    WD_CHECK_HIP(launch_finish(nr, fin, t.fin_d(), (int)t.fin.size(), sys, gated, s, a, b));
    if (timed) T.pending.push_back({TK_FINISH, a, b, 0.0, -1, 0, -1});
}

void run_hop(int sf, int lf, bool dag, int red, int fin, const JobTable<HopJob>& t, SysState* sys, int gated,
             hipStream_t s, double bytes, int stage, int ntl_force)
{
    Timer& T = timer();
    hipEvent_t a = nullptr, b = nullptr;
    const int cls = sf == SF64 ? TK_HOP_F64 : TK_HOP_LO;
    int* flag = nullptr;
    const bool timed = T.on && t.nblocks > 0;  // (a launcher with no blocks launches nothing)
    if (timed) {
        flag = T.slot();
        a = T.get();
        b = T.get();
    }
    // Non-temporal link loads keep the links from evicting the neighbour spinors in L2. They pay
    // off when the links cannot stay in the 256 MB Infinity Cache between hops anyway (more than
    // 64 MB of links in the launch), and not when interleaved systems read the shared links from L2.
    int tg = 0, ntl = 1;
    double link_bytes = 0;
    for (auto& j : t.host) {
        tg |= j.tg;
        if (j.ilv > 1) ntl = 0;
        link_bytes += (double)j.g.Vh * 8 * link_chunks(lf) * link_chunk_bytes(lf);
    }
    if (link_bytes <= 64.0 * (1 << 20)) ntl = 0;
    if (ntl_force >= 0) ntl = ntl_force != 0;
    if (!t.host.empty() && t.host[0].rhs >= 2) {
        int kmax = 1;
        for (auto& j : t.host) kmax = std::max(kmax, j.ilv);
        const int kt = mrhs_kt(kmax);
        if (kt == 0 || sf == SF64) throw Error{WD_ERR_UNSUPPORTED, "multi-RHS hop: unsupported group or format"};
        WD_CHECK_HIP(launch_hop_mrhs(sf, lf, dag, red, kt, t.d(), t.n(), t.nblocks, sys, gated, s, flag, a, b));
    } else {
        WD_CHECK_HIP(launch_hop(sf, lf, dag, red, fin, t.d(), t.n(), t.nblocks, sys, gated, s, flag, stage, tg, ntl, a, b));
    }
    if (timed)
        T.pending.push_back({cls, a, b, bytes, (int)(flag - T.dflags), t.n(), cls == TK_HOP_LO ? TK_HOP_LO_RED + red : -1});
    if (red != RED_NONE) run_finish(3, fin, t, sys, gated, s);
}

void run_sweep(int op, int sfl, const JobTable<SweepJob>& t, SysState* sys, int gated, hipStream_t s, double bytes)
{
    Timer& T = timer();
    hipEvent_t a = nullptr, b = nullptr;
    int* flag = nullptr;
    const bool timed = T.on && t.nblocks > 0;
    if (timed) {
        flag = T.slot();
        a = T.get();
        b = T.get();
    }
    WD_CHECK_HIP(launch_sweep(op, sfl, t.d(), t.n(), t.nblocks, sys, gated, s, flag, a, b));
    if (timed) T.pending.push_back({TK_SWEEP, a, b, bytes, (int)(flag - T.dflags), t.n(), -1});
    switch (op) {
    case OP_XR: run_finish(3, FIN_ALPHA, t, sys, gated, s); break;
    case OP_SHIFT: run_finish(0, FIN_END, t, sys, gated, s); break;  // OP_S: committed in FIN_ALPHA
    case OP_INIT:
    case OP_MSINIT: run_finish(3, FIN_RESTART, t, sys, gated, s); break;
    case OP_NORM: run_finish(3, FIN_STORE, t, sys, gated, s); break;
    case OP_CGX: run_finish(3, FIN_CGB, t, sys, gated, s); break;
    case OP_CGPM: run_finish(0, FIN_CGEND, t, sys, gated, s); break;  // OP_CGP: committed in FIN_CGB
    default: break;
    }
}

} // namespace wd

// ---------------------------------------------------------------- gauge handle
using namespace wd;

const void* wd_gauge::lk(int lf, int parity) const
{
    const DevMem* m = links[lf].get();
    if (!m) throw Error{WD_ERR_ARG, "link format not prepared"};
    size_t half = m->bytes / 2;
    return (const char*)m->p + (size_t)parity * half;
}

const void* wd_gauge::slk(int lf, int parity) const
{
    if (!tg) return lk(lf, parity);
    const DevMem* m = fixed[lf].get();
    if (!m) throw Error{WD_ERR_ARG, "link format not prepared"};
    return (const char*)m->p + (size_t)parity * (m->bytes / 2);
}

static size_t link_bytes(int lf, long stride)
{
    return (size_t)2 * 8 * link_chunks(lf) * link_chunk_bytes(lf) * stride;
}

void wd_gauge::ensure_links(int lf, hipStream_t s)
{
    if (links[lf]) return;
    if (lf == L16_8) {
        if (recon_err > 1e-6)
            throw Error{WD_ERR_UNSUPPORTED, "links are not SU(3): the 8-real format would change the operator"};
        // row 1 is rebuilt by dividing by 1 - |u00|^2: refuse links (nearly) diagonal in row 0
        if (u00_max > 1.0 - 1e-6)
            throw Error{WD_ERR_UNSUPPORTED, "a link has |u00| = 1 to within 1e-6 (e.g. unit links): the 8-real "
                                            "format cannot rebuild it; use recon 12"};
    }
    auto m = std::make_unique<DevMem>(link_bytes(lf, geo.stride));
    const size_t half = m->bytes / 2;
    for (int p = 0; p < 2; p++)
        WD_CHECK_HIP(launch_convert_links(lf, L64_18, lk(L64_18, p), (char*)m->p + p * half, geo.Vh, geo.stride, s));
    links[lf] = std::move(m);
}

void wd_gauge::ensure_slinks(int lf, hipStream_t s)
{
    if (!tg) {
        ensure_links(lf, s);
        return;
    }
    if (lf == L16_8)
        throw Error{WD_ERR_UNSUPPORTED, "the temporal gauge makes time links unit matrices, which the 8-real "
                                        "format cannot rebuild; use recon 12"};
    if (fixed[lf]) return;
    // every other format is converted from the transformed 12-real FP64 links (exact for SU(3))
    auto m = std::make_unique<DevMem>(link_bytes(lf, geo.stride));
    const size_t half = m->bytes / 2;
    for (int p = 0; p < 2; p++)
        WD_CHECK_HIP(launch_convert_links(lf, L64_12, slk(L64_12, p), (char*)m->p + p * half, geo.Vh, geo.stride, s));
    fixed[lf] = std::move(m);
}

void wd_gauge::build_temporal_gauge(const double* U, hipStream_t s)
{
    const size_t gbytes = (size_t)V * 9 * 16;
    gmat = std::make_unique<DevMem>(gbytes);
    {
        DevMem Uf((size_t)4 * V * 9 * 16);
        DevMem f18(link_bytes(L64_18, geo.stride));
        WD_CHECK_HIP(hipMemsetAsync(f18.p, 0, f18.bytes, s));
        WD_CHECK_HIP(launch_temporal_gauge(U, geo, (double*)gmat->p, (double*)Uf.p, s));
        WD_CHECK_HIP(launch_pack_links((const double*)Uf.p, geo, f18.p, (char*)f18.p + f18.bytes / 2, geo.stride, s));
        auto m = std::make_unique<DevMem>(link_bytes(L64_12, geo.stride));
        const size_t half = m->bytes / 2;
        for (int p = 0; p < 2; p++)
            WD_CHECK_HIP(launch_convert_links(L64_12, L64_18, (const char*)f18.p + p * (f18.bytes / 2),
                                              (char*)m->p + p * half, geo.Vh, geo.stride, s));
        fixed[L64_12] = std::move(m);
        WD_CHECK_HIP(hipStreamSynchronize(s));  // the temporaries are freed on return
    }
    tg = true;
}

Field& wd_gauge::field(const std::string& key, int sf, int halves)
{
    auto it = ws.find(key);
    if (it != ws.end() && it->second.sf == sf && it->second.halves == halves) return it->second;
    Field f;
    f.sf = sf;
    f.halves = halves;
    f.stride = geo.stride;
    f.mem = std::make_shared<DevMem>(field_bytes(sf, halves, geo.stride));
    WD_CHECK_HIP(hipMemset(f.mem->p, 0, f.mem->bytes));
    ws[key] = f;
    return ws[key];
}

void* wd_gauge::rawbuf(const std::string& key, size_t bytes)
{
    auto it = raw.find(key);
    if (it != raw.end() && it->second->bytes >= bytes) return it->second->p;
    auto m = std::make_shared<DevMem>(bytes);
    WD_CHECK_HIP(hipMemset(m->p, 0, m->bytes));
    raw[key] = m;
    return m->p;
}

size_t wd_gauge::device_bytes() const
{
    size_t n = 0;
    for (auto& l : links)
        if (l) n += l->bytes;
    for (auto& l : fixed)
        if (l) n += l->bytes;
    if (gmat) n += gmat->bytes;
    for (auto& kv : ws) n += kv.second.mem->bytes;
    for (auto& kv : raw) n += kv.second->bytes;
    return n;
}
