// Device-side building blocks of libwdirac: storage formats, complex arithmetic, spinor and
// link loads/stores, lattice geometry and deterministic block reductions.
//
// Internal layout (structure of arrays, site index innermost, as the paper argues in Sec. 3-4
// for coalesced access; the chunking is our own, chosen so that each lane issues 8- or 16-byte
// loads on gfx950):
//   * a "half field" holds the sites of one parity in checkerboard order
//       cb = (x >> 1) + (X/2) * (y + Y * (z + Z * t));
//     even sites first, then odd ones, as in the even-first site map of Sec. 4;
//   * a spinor of 12 complex numbers (colour c, spin s, index c*4 + s) is split into chunks:
//       F64: 12 x double2 (one complex each)  F32: 6 x float4 (two complex each)
//       F16: 3 x half8 (four complex each) plus one float per site holding the largest
//            |component|, by which the stored values are divided;
//     the chunks of 64 consecutive sites are stored together: chunk j of site i lives at
//     base[((i / 64) * nchunks + j) * 64 + i % 64] (see chunk_at), so a wavefront's loads of one
//     site quantity fall into one contiguous region;
//   * links are stored per output parity and per output site: 8 matrices per site, slots 0..3
//     the forward links U_mu(n), slots 4..7 the backward links already daggered,
//     U_mu(n - mu)^dag, so every hop reads its 8 links fully coalesced. 12-real formats keep rows
//     0 and 1 and rebuild row 2 = conj(row0 x row1), exact for SU(3); the 8-real FP16 format
//     keeps 6 elements and 2 phases in one 16-byte chunk per link (recon8).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wd {

// threads (= sites) per block of the site-parallel kernels
constexpr int BLOCK_SITES = 256;

// ---------------------------------------------------------------- formats
enum SpinorFmt { SF64 = 0, SF32 = 1, SF16 = 2 };
enum LinkFmt { L64_18 = 0, L64_12 = 1, L32_12 = 2, L16_12 = 3, LB16_12 = 4, L32_18 = 5, L16_8 = 6, NLINKFMT = 7 };

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__host__ __device__ constexpr int spinor_chunks(int f) { return f == SF64 ? 12 : (f == SF32 ? 6 : 3); }
__host__ __device__ constexpr int spinor_chunk_bytes(int f) { return 16; }
__host__ __device__ constexpr int link_chunks(int f)
{
    return f == L64_18 ? 9 : f == L64_12 ? 6 : f == L32_18 ? 0 : f == L16_8 ? 1 : 3;
}
__host__ __device__ constexpr int link_chunk_bytes(int f)
{
    return (f == L64_18 || f == L64_12 || f == L32_12 || f == L16_8) ? 16 : 8;
}
__host__ __device__ constexpr bool link_recon12(int f) { return f != L64_18 && f != L32_18; }
// 16-byte chunks per site holding all 8 links of that site
__host__ __device__ constexpr int link_site_chunks(int f) { return 8 * link_chunks(f) * link_chunk_bytes(f) / 16; }

// ---------------------------------------------------------------- complex
template <class T>
struct cx {
    T re, im;
};
template <class T> __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <class T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T> __device__ __forceinline__ cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
template <class T> __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T> __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <class T> __device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.re, -a.im}; }
// fused multiply-add in the precision of T
__device__ __forceinline__ float fmaf_t(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fmaf_t(double a, double b, double c) { return fma(a, b, c); }
// conj(a) * b
template <class T> __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b)
{
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// multiply by the unit i^k (k = 0..3), free of arithmetic
template <int K, class T> __device__ __forceinline__ cx<T> mul_ik(cx<T> a)
{
    constexpr int k = ((K % 4) + 4) % 4;
    if constexpr (k == 0) return a;
    else if constexpr (k == 1) return {-a.im, a.re};
    else if constexpr (k == 2) return {-a.re, -a.im};
    else return {a.im, -a.re};
}

// ---------------------------------------------------------------- geometry
struct Geo {
    int X, Y, Z, T;
    int Xh;     // X / 2
    int Vh;     // sites per parity
    int stride; // sites per parity rounded up to the block size (allocation unit)
    int anti;   // antiperiodic in t
};

// site coordinates of checkerboard index cb of parity p
__host__ __device__ __forceinline__ void cb_coords(const Geo& g, int p, int cb, int& x, int& y, int& z, int& t)
{
    unsigned u = (unsigned)cb;
    const unsigned xh = u % (unsigned)g.Xh;
    u /= (unsigned)g.Xh;
    y = (int)(u % (unsigned)g.Y);
    u /= (unsigned)g.Y;
    z = (int)(u % (unsigned)g.Z);
    t = (int)(u / (unsigned)g.Z);
    x = 2 * (int)xh + ((p + y + z + t) & 1);
}
__host__ __device__ __forceinline__ int cb_index(const Geo& g, int x, int y, int z, int t)
{
    return (x >> 1) + g.Xh * (y + g.Y * (z + g.Z * t));
}
// checkerboard index of the neighbour of (x, y, z, t) in direction MU, forward (D = 0) or backward
// (D = 1), with periodic wrap (the time boundary sign is applied by the hop, not here)
template <int MU, int D>
__host__ __device__ __forceinline__ int nb_index(const Geo& g, int x, int y, int z, int t)
{
    if constexpr (MU == 0) x = D == 0 ? (x + 1 == g.X ? 0 : x + 1) : (x == 0 ? g.X - 1 : x - 1);
    if constexpr (MU == 1) y = D == 0 ? (y + 1 == g.Y ? 0 : y + 1) : (y == 0 ? g.Y - 1 : y - 1);
    if constexpr (MU == 2) z = D == 0 ? (z + 1 == g.Z ? 0 : z + 1) : (z == 0 ? g.Z - 1 : z - 1);
    if constexpr (MU == 3) t = D == 0 ? (t + 1 == g.T ? 0 : t + 1) : (t == 0 ? g.T - 1 : t - 1);
    return cb_index(g, x, y, z, t);
}
// The same neighbour index from the site's own checkerboard index cb = (x >> 1) + Xh (y + Y (z + Z t)):
// an x step changes x >> 1 by 0 or +-1, a y, z or t step moves by a whole row, plane or slice
// (a uniform stride), with the periodic wrap. Cheaper than nb_index (no per-lane multiplies).
template <int MU, int D>
__host__ __device__ __forceinline__ int nb_from_cb(const Geo& g, int cb, int x, int y, int z, int t)
{
    if constexpr (MU == 0) {
        const int xn = D == 0 ? (x + 1 == g.X ? 0 : x + 1) : (x == 0 ? g.X - 1 : x - 1);
        return cb - (x >> 1) + (xn >> 1);
    } else {
        const int L = MU == 1 ? g.Y : MU == 2 ? g.Z : g.T;
        const int c = MU == 1 ? y : MU == 2 ? z : t;
        const int s = MU == 1 ? g.Xh : MU == 2 ? g.Xh * g.Y : g.Xh * g.Y * g.Z;
        if constexpr (D == 0) return c + 1 == L ? cb - s * (L - 1) : cb + s;
        else return c == 0 ? cb + s * (L - 1) : cb - s;
    }
}

// ---------------------------------------------------------------- chunk addressing
// Fields and links are stored in blocks of AOSOA_B sites with all chunks of a block contiguous
// (chunk j of site i at ((i / B) * nchunks + j) * B + i % B), so one wavefront's loads of a site
// quantity fall into one contiguous region and a kernel keeps a few DRAM streams open instead of
// one per chunk (measured on MI355X: hops +6%, sweeps +10% over one array per chunk).
constexpr long AOSOA_B = 64;  // sites per block (a power of two dividing 256)
constexpr bool AOSOA = true;
__host__ __device__ __forceinline__ long chunk_at(int nchunks, long cs, long i, int j)
{
    return ((i / AOSOA_B) * nchunks + j) * AOSOA_B + (i % AOSOA_B);
}

// ---------------------------------------------------------------- global-memory accessors
// Device pointers reach the kernels through job tables in memory, so the compiler cannot tell
// they are global and would emit flat loads; these casts make every field and link access a
// global load or store.
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
template <class V>
__device__ __forceinline__ V gld(const void* base, long idx)
{
    typedef __attribute__((address_space(1))) const V GV;
    return *((GV*)base + idx);
}
// NT: a non-temporal load, for data that the kernel reads once (it does not displace lines that
// other sites of the launch are about to re-read from L2)
template <class V, bool NT>
__device__ __forceinline__ V gldt(const void* base, long idx)
{
    typedef __attribute__((address_space(1))) const V GV;
    if constexpr (NT) return __builtin_nontemporal_load((GV*)base + idx);
    else return *((GV*)base + idx);
}
template <class V, bool NT = false>
__device__ __forceinline__ void gst(void* base, long idx, V v)
{
    typedef __attribute__((address_space(1))) V GV;
    if constexpr (NT) __builtin_nontemporal_store(v, (GV*)base + idx);
    else *((GV*)base + idx) = v;
}

// ---------------------------------------------------------------- field views
struct SpinorRef {
    void* p;     // chunk 0 of site 0 of this view
    float* nrm;  // F16 only: per-site scale
    long cs;     // chunk stride in sites
};

template <int SF> struct SReal { using T = float; };
template <> struct SReal<SF64> { using T = double; };

template <int SF, class T, bool NT = false>
__device__ __forceinline__ void load_spinor(const SpinorRef& r, long i, cx<T> v[12])
{
    if constexpr (SF == SF64) {
#pragma unroll
        for (int j = 0; j < 12; j++) {
            d2v q = gldt<d2v, NT>(r.p, chunk_at(12, r.cs, i, j));
            v[j] = mk<T>((T)q[0], (T)q[1]);
        }
    } else if constexpr (SF == SF32) {
#pragma unroll
        for (int j = 0; j < 6; j++) {
            f4v q = gldt<f4v, NT>(r.p, chunk_at(6, r.cs, i, j));
            v[2 * j] = mk<T>((T)q[0], (T)q[1]);
            v[2 * j + 1] = mk<T>((T)q[2], (T)q[3]);
        }
    } else {
        const float n = gldt<float, NT>(r.nrm, i);
#pragma unroll
        for (int j = 0; j < 3; j++) {
            h8 q = gldt<h8, NT>(r.p, chunk_at(3, r.cs, i, j));
#pragma unroll
            for (int k = 0; k < 4; k++) v[4 * j + k] = mk<T>((T)((float)q[2 * k] * n), (T)((float)q[2 * k + 1] * n));
        }
    }
}

// FP16 spinor without its per-site scale (returned): the hop applies the scale after the spin
// projection and the link multiply, which are linear, folding it into its accumulation.
template <class T>
__device__ __forceinline__ float load_spinor16_raw(const SpinorRef& r, long i, cx<T> v[12])
{
    const float n = gld<float>(r.nrm, i);
#pragma unroll
    for (int j = 0; j < 3; j++) {
        h8 q = gld<h8>(r.p, chunk_at(3, r.cs, i, j));
#pragma unroll
        for (int k = 0; k < 4; k++) v[4 * j + k] = mk<T>((T)(float)q[2 * k], (T)(float)q[2 * k + 1]);
    }
    return n;
}

// FP16 spinor storage divides a site's 24 values by their largest magnitude m. A site with m below
// the smallest normal float (where 1/m would overflow to infinity and 0 * inf give NaN) is stored
// as zero; so is m = 0. An infinite or NaN m keeps its scale (inv = 0): the load then yields NaN,
// which the solver reports.
__host__ __device__ __forceinline__ float f16_site_inv(float m)
{
    return m >= 1.17549435e-38f && m <= 3.40282347e+38f ? 1.0f / m : 0.0f;
}

// NT: non-temporal stores (a hop's output is not read again within the launch)
template <int SF, class T, bool NT = false>
__device__ __forceinline__ void store_spinor(const SpinorRef& r, long i, const cx<T> v[12])
{
    if constexpr (SF == SF64) {
#pragma unroll
        for (int j = 0; j < 12; j++)
            gst<d2v, NT>(r.p, chunk_at(12, r.cs, i, j), d2v{(double)v[j].re, (double)v[j].im});
    } else if constexpr (SF == SF32) {
#pragma unroll
        for (int j = 0; j < 6; j++)
            gst<f4v, NT>(r.p, chunk_at(6, r.cs, i, j),
                         f4v{(float)v[2 * j].re, (float)v[2 * j].im, (float)v[2 * j + 1].re, (float)v[2 * j + 1].im});
    } else {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 12; k++) m = fmaxf(m, fmaxf(fabsf((float)v[k].re), fabsf((float)v[k].im)));
        const float inv = f16_site_inv(m);
        gst<float, NT>(r.nrm, i, inv == 0.f && m < 1.0f ? 0.f : m);
#pragma unroll
        for (int j = 0; j < 3; j++) {
            h8 q;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                q[2 * k] = (_Float16)((float)v[4 * j + k].re * inv);
                q[2 * k + 1] = (_Float16)((float)v[4 * j + k].im * inv);
            }
            gst<h8, NT>(r.p, chunk_at(3, r.cs, i, j), q);
        }
    }
}

// ---------------------------------------------------------------- LDS staging of input sites
// A hop block covers BLOCK consecutive checkerboard sites, i.e. whole rows of constant (y, z, t)
// when Xh divides BLOCK. Its x neighbours lie in the same rows and its y neighbours one row up
// or down, so the block first copies the input sites [cb0 - H, cb0 + BLOCK + H) with H = Xh
// (when Xh <= STG_H_MAX) into LDS with coalesced direct global -> LDS loads (stage_window), and
// the four x and y directions then read LDS instead of gathering from memory. Neighbours outside that window
// (the periodic wrap in y, or H = 0) are loaded from memory as before.
constexpr int STG_H_MAX = 32;
constexpr int STG_SLOTS = BLOCK_SITES + 2 * STG_H_MAX;
template <int SF, bool ON> struct Stg {
    int unused;
};
template <> struct Stg<SF64, true> {
    d2v c[12][STG_SLOTS];
};
template <> struct Stg<SF32, true> {
    f4v c[6][STG_SLOTS];
};
template <> struct Stg<SF16, true> {
    h8 c[3][STG_SLOTS];
    float n[STG_SLOTS];
};

// Stage the window [base, base + nsl) with direct global -> LDS loads: each wave covers 64
// consecutive slots, lane l filling slot k0 + l (the hardware writes lane l's bytes at the wave's
// LDS address plus l times the access size), so the data does not pass through registers. Sites
// outside the lattice are skipped (their slots are never read). The loads are asynchronous:
// stage_wait() before the block's barrier completes them (one wait after several windows).
__device__ __forceinline__ void lds_load16(const void* g, void* lds)
{
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)g,
                                     (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}
__device__ __forceinline__ void lds_load4(const void* g, void* lds)
{
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)g,
                                     (__attribute__((address_space(3))) void*)lds, 4, 0, 0);
}
template <int SF>
__device__ __forceinline__ void stage_window(Stg<SF, true>& L, const SpinorRef& r, int base, int nsl, int Vh)
{
    const int lane = threadIdx.x & 63;
    for (int k0 = (int)(threadIdx.x & ~63u); k0 < nsl; k0 += BLOCK_SITES) {
        const int k = k0 + lane, i = base + k;
        if (k < nsl && i >= 0 && i < Vh) {
            if constexpr (SF == SF64) {
#pragma unroll
                for (int j = 0; j < 12; j++) lds_load16((const d2v*)r.p + chunk_at(12, r.cs, i, j), &L.c[j][k0]);
            } else if constexpr (SF == SF32) {
#pragma unroll
                for (int j = 0; j < 6; j++) lds_load16((const f4v*)r.p + chunk_at(6, r.cs, i, j), &L.c[j][k0]);
            } else {
                lds_load4(r.nrm + i, &L.n[k0]);
#pragma unroll
                for (int j = 0; j < 3; j++) lds_load16((const h8*)r.p + chunk_at(3, r.cs, i, j), &L.c[j][k0]);
            }
        }
    }
}
__device__ __forceinline__ void stage_wait() { __builtin_amdgcn_s_waitcnt(0); }

template <int SF, class T>
__device__ __forceinline__ void load_spinor_stg(const Stg<SF, true>& L, int k, cx<T> v[12])
{
    if constexpr (SF == SF64) {
#pragma unroll
        for (int j = 0; j < 12; j++) {
            const d2v q = L.c[j][k];
            v[j] = mk<T>((T)q[0], (T)q[1]);
        }
    } else if constexpr (SF == SF32) {
#pragma unroll
        for (int j = 0; j < 6; j++) {
            const f4v q = L.c[j][k];
            v[2 * j] = mk<T>((T)q[0], (T)q[1]);
            v[2 * j + 1] = mk<T>((T)q[2], (T)q[3]);
        }
    } else {
        const float n = L.n[k];
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const h8 q = L.c[j][k];
#pragma unroll
            for (int m = 0; m < 4; m++) v[4 * j + m] = mk<T>((T)((float)q[2 * m] * n), (T)((float)q[2 * m + 1] * n));
        }
    }
}

template <class T>
__device__ __forceinline__ float load_spinor16_stg_raw(const Stg<SF16, true>& L, int k, cx<T> v[12])
{
#pragma unroll
    for (int j = 0; j < 3; j++) {
        const h8 q = L.c[j][k];
#pragma unroll
        for (int m = 0; m < 4; m++) v[4 * j + m] = mk<T>((T)(float)q[2 * m], (T)(float)q[2 * m + 1]);
    }
    return L.n[k];
}

// ---------------------------------------------------------------- streaming loads
// A hop of one system reads each link exactly once: non-temporal loads keep the links from
// evicting the neighbour spinors that other sites of the same XCD are about to re-read from L2.
// When several systems share the links (interleaved groups) ordinary loads let them hit in L2.
template <bool NT = true, class V>
__device__ __forceinline__ V ld_stream(const V* p)
{
    typedef __attribute__((address_space(1))) const V GV;
    if constexpr (NT) return __builtin_nontemporal_load((GV*)p);
    else return *(GV*)p;
}

// ---------------------------------------------------------------- links
__device__ __forceinline__ float bf16_to_f32(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }
// round to nearest even; inputs are finite link entries
__device__ __forceinline__ unsigned short f32_to_bf16(float f)
{
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

// 16-bit link formats pair the forward and backward link of one direction: chunk j (0..2) of pair
// mu is 16 bytes, the first 8 from slot mu (forward) and the last 8 from slot 4 + mu (backward),
// so a hop reads both links of a direction with three 16-byte loads.
__host__ __device__ constexpr bool link_paired(int f) { return f == L16_12 || f == LB16_12; }

// conj(a b - c d) as two chains of fused multiply-adds (1 multiply + 3 FMAs per component, where
// forming the two products first and subtracting takes 2 + 2 + 1)
template <class T>
__device__ __forceinline__ cx<T> conj_cross(cx<T> a, cx<T> b, cx<T> c, cx<T> d)
{
    T re = c.im * d.im;
    re = fmaf_t(-c.re, d.re, re);
    re = fmaf_t(-a.im, b.im, re);
    re = fmaf_t(a.re, b.re, re);
    T im = c.im * d.re;
    im = fmaf_t(c.re, d.im, im);
    im = fmaf_t(-a.im, b.re, im);
    im = fmaf_t(-a.re, b.im, im);
    return {re, im};
}

template <class T>
__device__ __forceinline__ void recon_row2(cx<T> W[9])
{
    // row 2 = conj(row0 x row1)
    W[6] = conj_cross(W[1], W[5], W[2], W[4]);
    W[7] = conj_cross(W[2], W[3], W[0], W[5]);
    W[8] = conj_cross(W[0], W[4], W[1], W[3]);
}

// sum_b W[r][b] h[b] (row r of a 3x3 complex matrix times a colour vector) as one chain of fused
// multiply-adds per component: 1 multiply + 5 FMAs, where summing three complex products formed
// separately takes 8 instructions per component
template <class T>
__device__ __forceinline__ cx<T> row_dot(const cx<T> W[9], int r, const cx<T> h[3])
{
    const cx<T> a = W[r * 3], b = W[r * 3 + 1], c = W[r * 3 + 2];
    T re = -c.im * h[2].im;
    re = fmaf_t(c.re, h[2].re, re);
    re = fmaf_t(-b.im, h[1].im, re);
    re = fmaf_t(b.re, h[1].re, re);
    re = fmaf_t(-a.im, h[0].im, re);
    re = fmaf_t(a.re, h[0].re, re);
    T im = c.im * h[2].re;
    im = fmaf_t(c.re, h[2].im, im);
    im = fmaf_t(b.im, h[1].re, im);
    im = fmaf_t(b.re, h[1].im, im);
    im = fmaf_t(a.im, h[0].re, im);
    im = fmaf_t(a.re, h[0].im, im);
    return {re, im};
}

// 8-real FP16 links: one 16-byte chunk per link holding u01, u02, u10 and the phases of u00 and
// u20 in units of pi. For U in SU(3) the rows are orthonormal and the inverse is the adjugate, so
// |u00|^2 = 1 - |u01|^2 - |u02|^2, |u20|^2 = |u01|^2 + |u02|^2 - |u10|^2, and row 1 solves the
// two linear conditions <row1, row0> = 0 and conj(u20) = u01 u12 - u02 u11, whose determinant is
// N = |u01|^2 + |u02|^2; row 2 then follows as for the 12-real formats. The host refuses fields
// with N near zero on some link (row 1 is not determined there).
template <class T>
__device__ __forceinline__ void recon8(const u16x8& q, cx<T> W[9])
{
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; k++) v[k] = (float)__builtin_bit_cast(_Float16, (unsigned short)q[k]);
    const cx<float> a = {v[0], v[1]}, b = {v[2], v[3]}, c = {v[4], v[5]};
    const float n = a.re * a.re + a.im * a.im + b.re * b.re + b.im * b.im;
    const float m00 = __builtin_amdgcn_sqrtf(fmaxf(1.0f - n, 0.0f));
    const float m20 = __builtin_amdgcn_sqrtf(fmaxf(n - c.re * c.re - c.im * c.im, 0.0f));
    // the hardware sine and cosine take revolutions: angle / (2 pi) = (angle / pi) / 2
    const float t0 = 0.5f * v[6], t2 = 0.5f * v[7];
    const cx<float> u00 = {m00 * __builtin_amdgcn_cosf(t0), m00 * __builtin_amdgcn_sinf(t0)};
    const cx<float> u20 = {m20 * __builtin_amdgcn_cosf(t2), m20 * __builtin_amdgcn_sinf(t2)};
    const float inv = __builtin_amdgcn_rcpf(n);
    const cx<float> r1 = -(c * cconj(u00)), r2 = cconj(u20);
    const cx<float> u11 = inv * (r1 * a - cmulc(b, r2));
    const cx<float> u12 = inv * (cmulc(a, r2) + b * r1);
    W[0] = mk<T>((T)u00.re, (T)u00.im);
    W[1] = mk<T>((T)a.re, (T)a.im);
    W[2] = mk<T>((T)b.re, (T)b.im);
    W[3] = mk<T>((T)c.re, (T)c.im);
    W[4] = mk<T>((T)u11.re, (T)u11.im);
    W[5] = mk<T>((T)u12.re, (T)u12.im);
}

template <int LF, class T>
__device__ __forceinline__ void unpack16(unsigned short a, unsigned short b, cx<T>& z)
{
    if constexpr (LF == L16_12) {
        z = mk<T>((T)(float)__builtin_bit_cast(_Float16, a), (T)(float)__builtin_bit_cast(_Float16, b));
    } else {
        z = mk<T>((T)bf16_to_f32(a), (T)bf16_to_f32(b));
    }
}

// Load link slot k (0..3 forward U_mu(n), 4..7 backward U_mu(n-mu)^dag) of output site i into
// W[3][3]. Unpaired formats: chunk j of slot k at base[(k * nchunks + j) * lcs + i].
template <int LF, class T, bool NT = true>
__device__ __forceinline__ void load_link(const void* base, long lcs, int k, long i, cx<T> W[9])
{
    constexpr int NCT = link_site_chunks(LF);
    if constexpr (LF == L64_18 || LF == L64_12) {
        constexpr int nc = link_chunks(LF);
        const d2v* p = (const d2v*)base;
#pragma unroll
        for (int j = 0; j < nc; j++) {
            d2v q = ld_stream<NT>(p + chunk_at(NCT, lcs, i, k * nc + j));
            W[j] = mk<T>((T)q[0], (T)q[1]);
        }
    } else if constexpr (LF == L32_12) {
        const f4v* p = (const f4v*)base;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            f4v q = ld_stream<NT>(p + chunk_at(NCT, lcs, i, k * 3 + j));
            W[2 * j] = mk<T>((T)q[0], (T)q[1]);
            W[2 * j + 1] = mk<T>((T)q[2], (T)q[3]);
        }
    } else if constexpr (link_paired(LF)) {
        const u16x4* p = (const u16x4*)base;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            u16x4 q = ld_stream<NT>(p + 2 * chunk_at(NCT, lcs, i, (k & 3) * 3 + j) + (k >> 2));
            unpack16<LF, T>(q[0], q[1], W[2 * j]);
            unpack16<LF, T>(q[2], q[3], W[2 * j + 1]);
        }
    } else if constexpr (LF == L16_8) {
        recon8<T>(ld_stream<NT>((const u16x8*)base + chunk_at(NCT, lcs, i, k)), W);
    }
    if constexpr (link_recon12(LF)) recon_row2(W);
}

// Both links of direction mu: forward U_mu(n) into Wf, backward U_mu(n-mu)^dag into Wb.
template <int LF, class T, bool NT = true>
__device__ __forceinline__ void load_link_pair(const void* base, long lcs, int mu, long i, cx<T> Wf[9], cx<T> Wb[9])
{
    if constexpr (link_paired(LF)) {
        const u16x8* p = (const u16x8*)base;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            u16x8 q = ld_stream<NT>(p + chunk_at(12, lcs, i, mu * 3 + j));
            unpack16<LF, T>(q[0], q[1], Wf[2 * j]);
            unpack16<LF, T>(q[2], q[3], Wf[2 * j + 1]);
            unpack16<LF, T>(q[4], q[5], Wb[2 * j]);
            unpack16<LF, T>(q[6], q[7], Wb[2 * j + 1]);
        }
        recon_row2(Wf);
        recon_row2(Wb);
    } else {
        load_link<LF, T, NT>(base, lcs, mu, i, Wf);
        load_link<LF, T, NT>(base, lcs, 4 + mu, i, Wb);
    }
}

template <int LF>
__device__ __forceinline__ void store_link(void* base, long lcs, int k, long i, const cx<double> W[9])
{
    constexpr int NCT = link_site_chunks(LF);
    if constexpr (LF == L64_18 || LF == L64_12) {
        constexpr int nc = link_chunks(LF);
        double2* p = (double2*)base;
#pragma unroll
        for (int j = 0; j < nc; j++) p[chunk_at(NCT, lcs, i, k * nc + j)] = make_double2(W[j].re, W[j].im);
    } else if constexpr (LF == L32_12) {
        float4* p = (float4*)base;
#pragma unroll
        for (int j = 0; j < 3; j++)
            p[chunk_at(NCT, lcs, i, k * 3 + j)] = make_float4((float)W[2 * j].re, (float)W[2 * j].im, (float)W[2 * j + 1].re,
                                     (float)W[2 * j + 1].im);
    } else if constexpr (LF == L16_12) {
        h4* p = (h4*)base;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            h4* pj = p + 2 * chunk_at(NCT, lcs, i, (k & 3) * 3 + j) + (k >> 2);
            h4 q;
            q[0] = (_Float16)(float)W[2 * j].re;
            q[1] = (_Float16)(float)W[2 * j].im;
            q[2] = (_Float16)(float)W[2 * j + 1].re;
            q[3] = (_Float16)(float)W[2 * j + 1].im;
            *pj = q;
        }
    } else if constexpr (LF == LB16_12) {
        u16x4* p = (u16x4*)base;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            u16x4* pj = p + 2 * chunk_at(NCT, lcs, i, (k & 3) * 3 + j) + (k >> 2);
            u16x4 q;
            q[0] = f32_to_bf16((float)W[2 * j].re);
            q[1] = f32_to_bf16((float)W[2 * j].im);
            q[2] = f32_to_bf16((float)W[2 * j + 1].re);
            q[3] = f32_to_bf16((float)W[2 * j + 1].im);
            *pj = q;
        }
    } else if constexpr (LF == L16_8) {
        h8 q;
        q[0] = (_Float16)(float)W[1].re;
        q[1] = (_Float16)(float)W[1].im;
        q[2] = (_Float16)(float)W[2].re;
        q[3] = (_Float16)(float)W[2].im;
        q[4] = (_Float16)(float)W[3].re;
        q[5] = (_Float16)(float)W[3].im;
        q[6] = (_Float16)(float)(atan2(W[0].im, W[0].re) * 0.31830988618379067154);
        q[7] = (_Float16)(float)(atan2(W[6].im, W[6].re) * 0.31830988618379067154);
        ((h8*)base)[chunk_at(NCT, lcs, i, k)] = q;
    }
}

// ---------------------------------------------------------------- reductions
constexpr int BLOCK = BLOCK_SITES;
constexpr int NRED = 4;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum NR values over the block in a fixed order; result valid in thread 0.
template <int NR>
__device__ __forceinline__ void block_sum(double v[NR], double* lds /* [NR][BLOCK/64] */)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NR; k++) {
        double s = wave_sum(v[k]);
        if (lane == 0) lds[k * (BLOCK / 64) + wid] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NR; k++) {
            double s = 0;
            for (int w = 0; w < BLOCK / 64; w++) s += lds[k * (BLOCK / 64) + w];
            v[k] = s;
        }
    }
}

} // namespace wd
