// C ABI of libwdirac (declared in include/wdirac.h). Every entry point validates its arguments,
// converts C++ exceptions into wd_status codes and records a thread-local message.
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "wd_host.hpp"

namespace wd {
const std::string& last_error();
wd_status solve_single(wd_gauge* g, double kappa, double* x, const double* b, const wd_solver_params& P,
                       wd_solver_stats* stats, hipStream_t st);
wd_status solve_multishift(wd_gauge* g, int n, const double* kappas, double* const* x, const double* b,
                           const wd_solver_params& P, wd_solver_stats* stats, hipStream_t st);
wd_status solve_batch(int nsys, const wd_system* sys, const wd_solver_params& P, wd_solver_stats* stats,
                      hipStream_t st);
wd_status solve_normal(wd_gauge* g, double kappa, int n, const double* sigmas, double* const* x, const double* b,
                       int method, int guess, const wd_solver_params& P, wd_solver_stats* stats, hipStream_t st);
wd_status apply_prec(wd_gauge* g, double kappa, double* out, const double* in, const wd_solver_params& P,
                     const wd_op_variant& v, double* dots, hipStream_t st);
wd_status solve_multimass(wd_gauge* g, int n, const double* kappas, double* const* x, const double* b, int method,
                          int guess, const wd_solver_params& P, wd_solver_stats* stats, hipStream_t st);
void set_graphs(bool on);
} // namespace wd

using namespace wd;

template <class F>
static wd_status guarded(F&& f)
{
    try {
        return f();
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception& e) {
        set_error(e.what());
        return WD_ERR_HIP;
    } catch (...) {
        set_error("unknown exception");
        return WD_ERR_HIP;
    }
}

static void require_ptr(const void* p, const char* what)
{
    if (!p) throw Error{WD_ERR_ARG, std::string(what) + " is NULL"};
    if (((uintptr_t)p) & 15) throw Error{WD_ERR_ARG, std::string(what) + " is not 16-byte aligned"};
}

static void check_params(const wd_solver_params* p)
{
    if (!p) throw Error{WD_ERR_ARG, "params is NULL"};
    if (!(p->tol > 0) || !std::isfinite(p->tol)) throw Error{WD_ERR_ARG, "tol must be positive"};
    if (p->max_iter < 1) throw Error{WD_ERR_ARG, "max_iter must be >= 1"};
    if (p->mixed) {
        if (p->spinor_store != WD_F32 && p->spinor_store != WD_F16 && p->spinor_store != WD_F64)
            throw Error{WD_ERR_UNSUPPORTED, "spinor_store must be WD_F64, WD_F32 or WD_F16"};
        (void)link_fmt_of(p->link_store, p->recon);
        if (!(p->delta_reliable > 0 && p->delta_reliable < 1)) throw Error{WD_ERR_ARG, "delta_reliable must be in (0,1)"};
        if (p->mixed_mode != WD_MIXED_RELIABLE && p->mixed_mode != WD_MIXED_DEFECT)
            throw Error{WD_ERR_ARG, "mixed_mode must be WD_MIXED_RELIABLE or WD_MIXED_DEFECT"};
    }
}

extern "C" {

void wd_params_default(wd_solver_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->tol = 1e-8;
    p->max_iter = 5000;
    p->mixed = 1;
    p->spinor_store = WD_F32;
    p->link_store = WD_F16;
    p->recon = 12;
    p->eo = 1;
    p->delta_reliable = 0.1;
    p->use_x0 = 0;
    p->dagger = 0;
    p->mixed_mode = WD_MIXED_RELIABLE;
}

const char* wd_status_str(wd_status s)
{
    switch (s) {
    case WD_OK: return "WD_OK";
    case WD_ERR_ARG: return "WD_ERR_ARG";
    case WD_ERR_HIP: return "WD_ERR_HIP";
    case WD_ERR_OOM: return "WD_ERR_OOM";
    case WD_ERR_NOCONV: return "WD_ERR_NOCONV";
    case WD_ERR_BREAKDOWN: return "WD_ERR_BREAKDOWN";
    case WD_ERR_NAN: return "WD_ERR_NAN";
    case WD_ERR_UNSUPPORTED: return "WD_ERR_UNSUPPORTED";
    }
    return "unknown";
}

wd_status wd_last_error(char* buf, size_t n)
{
    if (!buf || n == 0) return WD_ERR_ARG;
    const std::string& m = last_error();
    size_t k = std::min(n - 1, m.size());
    std::memcpy(buf, m.data(), k);
    buf[k] = 0;
    return WD_OK;
}

wd_status wd_gauge_create(wd_gauge** out, const wd_geom* geom, const double* U, const wd_solver_params* hint,
                          void* stream)
{
    return guarded([&]() -> wd_status {
        if (!out || !geom) throw Error{WD_ERR_ARG, "NULL handle or geometry"};
        require_ptr(U, "U");
        for (int i = 0; i < 4; i++)
            if (geom->dims[i] < 2 || (geom->dims[i] & 1))
                throw Error{WD_ERR_ARG, "lattice extents must be even and >= 2"};
        const long V = (long)geom->dims[0] * geom->dims[1] * geom->dims[2] * geom->dims[3];
        if (V / 2 > (1L << 30)) throw Error{WD_ERR_ARG, "lattice too large"};
        hipStream_t s = (hipStream_t)stream;
        auto g = std::make_unique<wd_gauge>();
        g->V = V;
        Geo& G = g->geo;
        G.X = geom->dims[0];
        G.Y = geom->dims[1];
        G.Z = geom->dims[2];
        G.T = geom->dims[3];
        G.Xh = G.X / 2;
        G.Vh = (int)(V / 2);
        G.stride = (int)(((V / 2) + BLOCK - 1) / BLOCK * BLOCK);
        G.anti = geom->antiperiodic_t ? 1 : 0;
        g->stream = s;
        const size_t lb = (size_t)2 * 8 * link_chunks(L64_18) * link_chunk_bytes(L64_18) * G.stride;
        g->links[L64_18] = std::make_unique<DevMem>(lb);
        WD_CHECK_HIP(hipMemsetAsync(g->links[L64_18]->p, 0, lb, s));
        WD_CHECK_HIP(launch_pack_links(U, G, g->links[L64_18]->p, (char*)g->links[L64_18]->p + lb / 2, G.stride, s));
        {
            // decide whether the 12-real FP64 format is exact for these links
            const int nb = (G.Vh + BLOCK - 1) / BLOCK;
            DevMem bm(sizeof(double) * nb);
            double e = 0.0;
            std::vector<double> h(nb);
            for (int p = 0; p < 2; p++) {
                WD_CHECK_HIP(launch_recon_check(g->lk(L64_18, p), G.Vh, G.stride, (double*)bm.p, s));
                WD_CHECK_HIP(hipMemcpyAsync(h.data(), bm.p, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
                WD_CHECK_HIP(hipStreamSynchronize(s));
                for (double v : h) e = std::max(e, std::isfinite(v) ? v : 1.0);
            }
            g->recon_err = e;
            double u = 0.0;
            for (int p = 0; p < 2; p++) {
                WD_CHECK_HIP(launch_recon_check(g->lk(L64_18, p), G.Vh, G.stride, (double*)bm.p, s, 1));
                WD_CHECK_HIP(hipMemcpyAsync(h.data(), bm.p, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
                WD_CHECK_HIP(hipStreamSynchronize(s));
                for (double v : h) u = std::max(u, std::isfinite(v) ? v : 1.0);
            }
            g->u00_max = u;
            const bool tg_on = hint && hint->temporal_gauge;
            if (e < 1e-12) {
                if (tg_on) g->build_temporal_gauge(U, s);
                else g->ensure_links(L64_12, s);
            }
        }
        if (hint && hint->gamma_basis != 0 && hint->gamma_basis != 1)
            throw Error{WD_ERR_ARG, "gamma_basis must be 0 (chiral) or 1 (non-chiral)"};
        g->nc = hint && hint->gamma_basis == 1 ? 1 : 0;
        if (hint && hint->mixed) g->ensure_slinks(link_fmt_of(hint->link_store, hint->recon), s);
        WD_CHECK_HIP(hipStreamSynchronize(s));
        *out = g.release();
        return WD_OK;
    });
}

wd_status wd_gauge_destroy(wd_gauge* g)
{
    return guarded([&]() -> wd_status {
        if (!g) return WD_ERR_ARG;
        if (g->stream) (void)hipStreamSynchronize(g->stream);
        (void)hipDeviceSynchronize();
        delete g;
        return WD_OK;
    });
}

size_t wd_gauge_device_bytes(const wd_gauge* g) { return g ? g->device_bytes() : 0; }

static wd_status apply_impl(wd_gauge* g, double kappa, double* out, const double* in, void* stream, bool dag)
{
    return guarded([&]() -> wd_status {
        if (!g) throw Error{WD_ERR_ARG, "NULL gauge"};
        require_ptr(out, "out");
        require_ptr(in, "in");
        if (out == in) throw Error{WD_ERR_ARG, "in and out must be distinct"};
        if (!(kappa > 0)) throw Error{WD_ERR_ARG, "kappa must be positive"};
        hipStream_t s = (hipStream_t)stream;
        Field& A = g->field("apply.in", SF64, 2);
        Field& B = g->field("apply.out", SF64, 2);
        char key[64];
        std::snprintf(key, sizeof(key), "apply.%.17g.%d", kappa, (int)dag);
        auto it = g->hop_tables.find(key);
        if (it == g->hop_tables.end()) {
            JobTable<HopJob> t;
            int b0 = 0;
            for (int p = 0; p < 2; p++) {
                HopJob j;
                std::memset(&j, 0, sizeof(j));
                j.g = g->geo;
                j.parity = p;
                j.in = A.half(1 - p);
                j.out = B.half(p);
                j.x0 = A.half(p);
                j.c0 = 1.0 / (2.0 * kappa);
                j.c2 = -0.5;
                j.links = g->lk(L64_18, p);
                j.lcs = g->lcs();
                j.nblk = (g->geo.Vh + BLOCK - 1) / BLOCK;
                j.blk0 = b0;
                j.rblk0 = b0;
                b0 += j.nblk;
                t.host.push_back(j);
            }
            for (auto& j : t.host) j.rnblk = b0;
            t.upload(s);
            if (g->hop_tables.size() > 64) g->hop_tables.clear();
            it = g->hop_tables.emplace(key, t).first;
        }
        SysState* dummy = (SysState*)g->rawbuf("apply.sys", sizeof(SysState));
        WD_CHECK_HIP(launch_pack_spinor(SF64, in, g->geo, A.half(0), A.half(1), 0, 1.0, s));
        run_hop(SF64, L64_18, dag, RED_NONE, FIN_STORE, it->second, dummy, 0, s, (double)g->geo.Vh * 2 * (192 * 3 + 1152));
        WD_CHECK_HIP(launch_unpack_spinor(SF64, out, g->geo, B.half(0), B.half(1), 0, 1.0, s));
        return WD_OK;
    });
}

wd_status wd_apply(wd_gauge* g, double kappa, double* out, const double* in, void* stream)
{
    return apply_impl(g, kappa, out, in, stream, false);
}
wd_status wd_apply_dag(wd_gauge* g, double kappa, double* out, const double* in, void* stream)
{
    return apply_impl(g, kappa, out, in, stream, true);
}

wd_status wd_apply_noalloc(wd_gauge* g, double kappa, double* out, const double* in, int dagger, void* stream)
{
    return guarded([&]() -> wd_status {
        if (!g) throw Error{WD_ERR_ARG, "NULL gauge"};
        require_ptr(out, "out");
        require_ptr(in, "in");
        if (out == in) throw Error{WD_ERR_ARG, "in and out must be distinct"};
        if (!(kappa > 0)) throw Error{WD_ERR_ARG, "kappa must be positive"};
        apply_noalloc(g, kappa, out, in, dagger != 0, (hipStream_t)stream);
        return WD_OK;
    });
}

wd_status bicgstab_solve(wd_gauge* g, double kappa, double* x, const double* b, const wd_solver_params* params,
                         wd_solver_stats* stats, void* stream)
{
    return guarded([&]() -> wd_status {
        if (!g) throw Error{WD_ERR_ARG, "NULL gauge"};
        require_ptr(x, "x");
        require_ptr(b, "b");
        check_params(params);
        if (stats) std::memset(stats, 0, sizeof(*stats));
        return solve_single(g, kappa, x, b, *params, stats, (hipStream_t)stream);
    });
}

wd_status bicgstab_m_solve(wd_gauge* g, int n, const double* kappas, double* const* x, const double* b,
                           const wd_solver_params* params, wd_solver_stats* stats, void* stream)
{
    return guarded([&]() -> wd_status {
        if (!g || !kappas || !x) throw Error{WD_ERR_ARG, "NULL argument"};
        if (n < 1 || n > 32) throw Error{WD_ERR_ARG, "n must be in 1..32"};
        require_ptr(b, "b");
        for (int i = 0; i < n; i++) require_ptr(x[i], "x[i]");
        check_params(params);
        if (stats) std::memset(stats, 0, sizeof(*stats) * n);
        return solve_multishift(g, n, kappas, x, b, *params, stats, (hipStream_t)stream);
    });
}

wd_status wd_multimass_solve(wd_gauge* g, int n, const double* kappas, double* const* x, const double* b, int method,
                             int guess, const wd_solver_params* params, wd_solver_stats* stats, void* stream)
{
    return guarded([&]() -> wd_status {
        if (!g || !kappas || !x) throw Error{WD_ERR_ARG, "NULL argument"};
        if (n < 1 || n > 32) throw Error{WD_ERR_ARG, "n must be in 1..32"};
        require_ptr(b, "b");
        for (int i = 0; i < n; i++) require_ptr(x[i], "x[i]");
        check_params(params);
        if (stats) std::memset(stats, 0, sizeof(*stats) * n);
        return solve_multimass(g, n, kappas, x, b, method, guess, *params, stats, (hipStream_t)stream);
    });
}

wd_status wd_normal_solve(wd_gauge* g, double kappa, int n, const double* sigmas, double* const* x, const double* b,
                          int method, int guess, const wd_solver_params* params, wd_solver_stats* stats, void* stream)
{
    return guarded([&]() -> wd_status {
        if (!g || !sigmas || !x) throw Error{WD_ERR_ARG, "NULL argument"};
        if (n < 1 || n > 32) throw Error{WD_ERR_ARG, "n must be in 1..32"};
        if (!(kappa > 0)) throw Error{WD_ERR_ARG, "kappa must be positive"};
        require_ptr(b, "b");
        for (int i = 0; i < n; i++) {
            require_ptr(x[i], "x[i]");
            if (!(sigmas[i] >= 0) || !std::isfinite(sigmas[i])) throw Error{WD_ERR_ARG, "shifts must be finite and >= 0"};
        }
        check_params(params);
        if (stats) std::memset(stats, 0, sizeof(*stats) * n);
        return solve_normal(g, kappa, n, sigmas, x, b, method, guess, *params, stats, (hipStream_t)stream);
    });
}

wd_status wd_batch_solve(int nsys, const wd_system* sys, const wd_solver_params* params, wd_solver_stats* stats,
                         void* stream)
{
    return guarded([&]() -> wd_status {
        if (!sys) throw Error{WD_ERR_ARG, "NULL systems"};
        if (nsys < 1 || nsys > 1024) throw Error{WD_ERR_ARG, "nsys must be in 1..1024"};
        for (int i = 0; i < nsys; i++) {
            require_ptr(sys[i].x, "sys[i].x");
            require_ptr(sys[i].b, "sys[i].b");
        }
        check_params(params);
        if (stats) std::memset(stats, 0, sizeof(*stats) * nsys);
        return solve_batch(nsys, sys, *params, stats, (hipStream_t)stream);
    });
}

void wd_op_variant_default(wd_op_variant* v)
{
    if (!v) return;
    std::memset(v, 0, sizeof(*v));
    v->red = WD_RED_NONE;
    v->stage = -1;
    v->nontemporal = -1;
    v->tile = -1;
    v->copies = 1;
    v->rhs_per_thread = -1;
    v->dagger = 0;
}

wd_status wd_apply_prec(wd_gauge* g, double kappa, double* out, const double* in, const wd_solver_params* params,
                        const wd_op_variant* v, double* dots, void* stream)
{
    return guarded([&]() -> wd_status {
        if (!g) throw Error{WD_ERR_ARG, "NULL gauge"};
        require_ptr(out, "out");
        require_ptr(in, "in");
        check_params(params);
        wd_op_variant var;
        wd_op_variant_default(&var);
        if (v) var = *v;
        if (var.copies < 1 || var.copies > 64) throw Error{WD_ERR_ARG, "copies must be in 1..64"};
        const size_t bytes = (size_t)g->V * 24 * sizeof(double) * var.copies;
        const char *o = (const char*)out, *i = (const char*)in;
        if (o < i + bytes && i < o + bytes) throw Error{WD_ERR_ARG, "in and out overlap"};
        return apply_prec(g, kappa, out, in, *params, var, dots, (hipStream_t)stream);
    });
}

wd_status wd_gauge_grad(wd_gauge* g, const double* x, const double* lam, double* dU, int project, void* stream)
{
    return guarded([&]() -> wd_status {
        if (!g) throw Error{WD_ERR_ARG, "NULL gauge"};
        require_ptr(x, "x");
        require_ptr(lam, "lam");
        require_ptr(dU, "dU");
        WD_CHECK_HIP(launch_grad(x, lam, g->geo, g->lk(L64_18, 0), g->lk(L64_18, 1), g->lcs(), dU, project ? 1 : 0,
                                 (hipStream_t)stream));
        return WD_OK;
    });
}

void wd_set_graphs(int on) { set_graphs(on != 0); }

void wd_timing_enable(int on)
{
    try {
        Timer& t = timer();
        if (!on) t.flush();
        t.on = on != 0;
    } catch (...) {
    }
}

void wd_timing_reset(void)
{
    try {
        Timer& t = timer();
        t.flush();
        for (int k = 0; k < NTK; k++) {
            t.ms[k] = 0;
            t.bytes[k] = 0;
            t.launches[k] = 0;
        }
    } catch (...) {
    }
}

wd_status wd_timing_get(int cls, double* total_ms, long* launches, double* bytes)
{
    return guarded([&]() -> wd_status {
        if (cls < 0 || cls >= NTK) throw Error{WD_ERR_ARG, "bad kernel class"};
        Timer& t = timer();
        t.flush();
        if (total_ms) *total_ms = t.ms[cls];
        if (launches) *launches = t.launches[cls];
        if (bytes) *bytes = t.bytes[cls];
        return WD_OK;
    });
}

} // extern "C"
