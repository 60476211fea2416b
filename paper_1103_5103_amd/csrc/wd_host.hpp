// Host-side internals of libwdirac: the gauge handle, workspace fields, job tables and the
// error/timing plumbing shared by the solver drivers and the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/wdirac.h"
#include "wd_kernels.hpp"

namespace wd {

// ---------------------------------------------------------------- errors
struct Error {
    wd_status code;
    std::string msg;
};
void set_error(const std::string& msg);
#define WD_CHECK_HIP(call)                                                                                       \
    do {                                                                                                         \
        hipError_t e_ = (call);                                                                                  \
        if (e_ != hipSuccess)                                                                                    \
            throw ::wd::Error{WD_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)};                    \
    } while (0)
#define WD_REQUIRE(cond, msg)                                                                                    \
    do {                                                                                                         \
        if (!(cond)) throw ::wd::Error{WD_ERR_ARG, msg};                                                         \
    } while (0)

// ---------------------------------------------------------------- device memory
struct DevMem {
    void* p = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    explicit DevMem(size_t n);
    ~DevMem();
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
};

// An internal spinor field: one half (one parity) or a full field (both halves).
struct Field {
    std::shared_ptr<DevMem> mem;
    int sf = SF64;
    int halves = 1;
    long stride = 0;  // sites per half
    char* base() const { return (char*)mem->p; }
    float* nrm() const { return sf == SF16 ? (float*)(base() + (size_t)16 * spinor_chunks(sf) * halves * stride) : nullptr; }
    long cs() const { return stride * halves; }
    // view of parity p (a full field) or of the single half
    SpinorRef half(int p) const
    {
        SpinorRef r;
        r.p = base() + (size_t)p * stride * 16 * (AOSOA ? spinor_chunks(sf) : 1);
        float* n = nrm();
        r.nrm = n ? n + (size_t)p * stride : nullptr;
        r.cs = cs();
        return r;
    }
    SpinorRef all() const { return SpinorRef{base(), nrm(), cs()}; }
    long nsites() const { return stride * halves; }
};
size_t field_bytes(int sf, int halves, long stride);

// ---------------------------------------------------------------- timing
// TK_HOP_LO_RED + r: the low-precision hops with fused reduction r (RED_NONE .. RED_NORM), also
// counted in TK_HOP_LO
enum { TK_HOP_LO = 0, TK_HOP_F64 = 1, TK_SWEEP = 2, TK_FINISH = 3, TK_HOP_LO_RED = 4, NTK = 8 };
struct Timer {
    bool on = false;
    struct Rec { int cls; hipEvent_t a, b; double bytes; int slot; int njobs; int cls2; };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    int* dflags = nullptr;  // per pending launch: set by the kernel when it did work
    size_t cap = 0;
    int* slot();
    double ms[NTK] = {};
    double bytes[NTK] = {};
    long launches[NTK] = {};
    hipEvent_t get();
    void flush();
};
Timer& timer();

// ---------------------------------------------------------------- job tables
// A launch's job list (and the list of systems its finisher reduces) in device memory. A table
// owns its device copy (upload), or several tables share one buffer and one copy (upload_tables).
struct JobTableBase {
    std::shared_ptr<DevMem> dev;
    size_t off = 0;  // byte offset of this table in dev
    size_t cap = 0;  // bytes reserved for this table at off
    long nblocks = 0;
    virtual ~JobTableBase() = default;
    virtual size_t prepare() = 0;          // finisher list, nblocks; returns the image size
    virtual void write(char* dst) const = 0;  // the image: jobs, then the finisher list
};

template <class J>
struct JobTable : JobTableBase {
    std::vector<J> host;
    std::vector<FinJob> fin;  // one entry per system, for the finisher kernel
    void upload(hipStream_t s);
    size_t prepare() override;
    void write(char* dst) const override;
    int n() const { return (int)host.size(); }
    const J* d() const { return (const J*)((const char*)dev->p + off); }
    const FinJob* fin_d() const { return (const FinJob*)((const char*)dev->p + off + fin_offset()); }
    size_t fin_offset() const { return (host.size() * sizeof(J) + 255) / 256 * 256; }
};

// Upload several non-empty tables with one host-to-device copy into mem (grown when too small;
// tables still holding the previous buffer keep it alive).
void upload_tables(hipStream_t s, std::shared_ptr<DevMem>& mem, std::initializer_list<JobTableBase*> tables);

// ---------------------------------------------------------------- gauge handle
} // namespace wd

struct wd_gauge {
    wd::Geo geo;
    long V = 0;
    std::unique_ptr<wd::DevMem> links[wd::NLINKFMT];  // both output parities, [parity][8][chunks][stride]
    // Solvers work in temporal gauge when the links are SU(3) to rounding: sources are rotated by
    // g(n) on the way in, solutions by g(n)^dag on the way out, and the solver link formats are
    // built from the transformed links (links[] keeps the caller's gauge for wd_apply and the
    // gradient).
    bool tg = false;
    // Solvers work in the non-chiral spin basis (gamma_4 diagonal) when the handle was created with
    // that option: sources are rotated on the way in, solutions on the way out, and the hops take
    // the time direction in that basis (half-spinor neighbours). wd_apply, wd_apply_noalloc and the
    // gradient use the caller's basis.
    int nc = 0;
    std::unique_ptr<wd::DevMem> gmat;                   // g(n), canonical [V][3][3] complex128
    std::unique_ptr<wd::DevMem> fixed[wd::NLINKFMT];    // transformed links, same layouts
    const double* gm() const { return tg ? (const double*)gmat->p : nullptr; }
    const void* slk(int lf, int parity) const;          // links of format lf for the solvers
    void ensure_slinks(int lf, hipStream_t s);
    std::map<std::string, wd::Field> ws;              // cached workspace fields
    std::map<std::string, std::shared_ptr<wd::DevMem>> raw;
    std::map<std::string, wd::JobTable<wd::HopJob>> hop_tables;
    std::map<std::string, std::shared_ptr<void>> graphs;  // captured iteration chunks by launch key
    hipStream_t stream = nullptr;
    double recon_err = 1.0;  // max |row2 - conj(row0 x row1)| over the links
    double u00_max = 1.0;    // max |u00|^2 over the links (the 8-real format needs it below 1)
    // FP64 operator format of the solvers: 12-real when the links are SU(3) to rounding, else 18-real
    int f64_links() const { return recon_err < 1e-12 ? wd::L64_12 : wd::L64_18; }
    const void* lk(int lf, int parity) const;
    long lcs() const { return geo.stride; }
    wd::Field& field(const std::string& key, int sf, int halves);
    void* rawbuf(const std::string& key, size_t bytes);
    void ensure_links(int lf, hipStream_t s);
    void build_temporal_gauge(const double* U, hipStream_t s);  // U: the caller's canonical links
    size_t device_bytes() const;
};

namespace wd {

// pinned staging for small host<->device copies (one buffer: synchronise before reusing it)
void* pinned(size_t bytes);
// pinned ring for host-to-device copies: no synchronisation needed, since a region is only
// handed out again after the device has drained (the ring synchronises when it wraps)
char* stage_alloc(size_t bytes);

// wd_apply_noalloc: a fixed device array per GPU (kNoallocScratchBytes) holds the job table and a
// system record in its first kNoallocTableBytes, then the packed FP64 input and output fields
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
constexpr size_t kNoallocTableBytes = (size_t)64 << 10;
constexpr int kNoallocMaxDevices = 64;
size_t noalloc_scratch_need(long stride);
void apply_noalloc(wd_gauge* g, double kappa, double* out, const double* in, bool dag, hipStream_t s);

// launch helpers with optional timing
// stage / ntl: -1 the defaults (LDS staging as built; non-temporal link loads unless the launch's
// links are shared or small), else forced (0 off, 1 on)
void run_hop(int sf, int lf, bool dag, int red, int fin, const JobTable<HopJob>& t, SysState* sys, int gated,
             hipStream_t s, double bytes_per_site_total, int stage = -1, int ntl = -1);
void run_sweep(int op, int sfl, const JobTable<SweepJob>& t, SysState* sys, int gated, hipStream_t s,
               double bytes_total);

int spinor_fmt_of(wd_prec p);
int link_fmt_of(wd_prec p, int recon);

} // namespace wd
