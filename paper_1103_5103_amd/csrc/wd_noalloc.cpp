// wd_apply_noalloc: the operator application of wd_apply for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).
//
// wd_apply keeps its packed input and output fields and its job table in workspaces of the handle,
// allocated on first use. This variant keeps them in `scratch`, a fixed file-scope device array
// (one copy per GPU, held until the process ends), and builds its two-entry job table on the device
// from kernel arguments, so it calls no hipMalloc, hipFree, pinned-memory allocation or host-to-device
// copy. The kernels are those of wd_apply (pack, the FP64 18-real hop, unpack) with the same launch
// configuration, so the results are bitwise those of wd_apply.
//
// Host code never uses the name `scratch` as an address: on first use on a device (that device
// current) hipGetSymbolAddress gives the device address, kept per device, and only that address is
// passed to kernels. Every call on one GPU shares that GPU's array: calls that overlap on one GPU
// race (serialise them, e.g. on one stream).
#include <cstring>
#include <mutex>

#include "wd_host.hpp"

namespace wd {

static __device__ __align__(256) char scratch[kNoallocScratchBytes];

static std::mutex g_scratch_mu;
static char* g_scratch_addr[kNoallocMaxDevices];

// the device address of `scratch` on the current device
static char* scratch_address()
{
    int dev = 0;
    WD_CHECK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoallocMaxDevices) throw Error{WD_ERR_ARG, "device index out of range"};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        WD_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error{WD_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array"};
        g_scratch_addr[dev] = (char*)p;
    }
    return g_scratch_addr[dev];
}

struct JobPair {
    HopJob j[2];
};

// the job table of one launch, written into device memory by the device itself
__global__ void k_store_jobs(HopJob* __restrict__ dst, JobPair src)
{
    if (threadIdx.x < 2) dst[threadIdx.x] = src.j[threadIdx.x];
}

// view of parity p of an FP64 field of two halves at `base` (the layout of Field::half)
static SpinorRef f64_half(char* base, long stride, int p)
{
    SpinorRef r;
    r.p = base + (size_t)p * stride * 16 * spinor_chunks(SF64);
    r.nrm = nullptr;
    r.cs = 2 * stride;
    return r;
}

size_t noalloc_scratch_need(long stride)
{
    return kNoallocTableBytes + 2 * field_bytes(SF64, 2, stride);
}

void apply_noalloc(wd_gauge* g, double kappa, double* out, const double* in, bool dag, hipStream_t s)
{
    const Geo& G = g->geo;
    const size_t need = noalloc_scratch_need(G.stride);
    if (need > kNoallocScratchBytes)
        throw Error{WD_ERR_ARG, "lattice too large for wd_apply_noalloc: needs " + std::to_string(need) +
                                    " bytes of scratch, the library holds " + std::to_string(kNoallocScratchBytes)};
    char* base = scratch_address();
    HopJob* jobs = (HopJob*)base;
    SysState* sys = (SysState*)(base + kNoallocTableBytes / 2);  // not read: ungated, no reduction
    char* fa = base + kNoallocTableBytes;
    char* fb = fa + field_bytes(SF64, 2, G.stride);
    JobPair jp;
    std::memset(&jp, 0, sizeof(jp));
    const int nb = (G.Vh + BLOCK - 1) / BLOCK;
    double link_bytes = 0;
    for (int p = 0; p < 2; p++) {
        HopJob& j = jp.j[p];
        j.g = G;
        j.parity = p;
        j.sys = 0;
        j.in = f64_half(fa, G.stride, 1 - p);
        j.out = f64_half(fb, G.stride, p);
        j.x0 = f64_half(fa, G.stride, p);
        j.c0 = 1.0 / (2.0 * kappa);
        j.c2 = -0.5;
        j.links = g->lk(L64_18, p);
        j.lcs = g->lcs();
        j.nblk = nb;
        j.blk0 = p * nb;
        j.rblk0 = p * nb;
        j.rnblk = 2 * nb;
        j.ilv = 1;
        link_bytes += (double)G.Vh * 8 * link_chunks(L64_18) * link_chunk_bytes(L64_18);
    }
    // the load policy wd_apply's launch takes (non-temporal links above 64 MB)
    const int ntl = link_bytes > 64.0 * (1 << 20) ? 1 : 0;
    WD_CHECK_HIP(launch_pack_spinor(SF64, in, G, f64_half(fa, G.stride, 0), f64_half(fa, G.stride, 1), 0, 1.0, s));
    hipLaunchKernelGGL(k_store_jobs, dim3(1), dim3(64), 0, s, jobs, jp);
    WD_CHECK_HIP(hipGetLastError());
    WD_CHECK_HIP(launch_hop(SF64, L64_18, dag, RED_NONE, FIN_STORE, jobs, 2, 2L * nb, sys, 0, s, nullptr, -1, 0, ntl));
    WD_CHECK_HIP(launch_unpack_spinor(SF64, out, G, f64_half(fb, G.stride, 0), f64_half(fb, G.stride, 1), 0, 1.0, s));
}

} // namespace wd
