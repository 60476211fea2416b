// The Wilson hopping term on gfx950 (CDNA4, wave64): device building blocks shared by the
// single-system hop (k_hop) and the multi-RHS hop (k_hop_mrhs), the k_hop kernel template and the
// dispatch macros of its launchers. Instantiated in wd_hop_lo.hip (FP32 / FP16 spinors) and
// wd_hop64.hip (FP64).
#pragma once
#include "wd_kernels.hpp"

namespace wd {

// MI355X has 8 XCDs, each with its own L2; consecutive workgroups go to consecutive XCDs. This
// bijection on [0, nb) hands each XCD one contiguous eighth of the blocks, so the neighbour
// sites a block gathers were mostly loaded by blocks of the same XCD and hit in its L2.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int x = b & 7, i = b >> 3, q = nb >> 3, r = nb & 7;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// Block reduction of NR partial sums; thread 0 stores the block's partial at slot rb.
template <int NR>
__device__ __forceinline__ void write_partials(double v[NRED], SysState* S, int rb)
{
    __shared__ double lds[NRED * (BLOCK / 64)];
    block_sum<NR>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NR; k++) S->partials[(long)rb * NRED + k] = v[k];
    }
}

// job of block b: jobs are sorted by blk0
template <class J>
__device__ __forceinline__ int find_job(const J* jobs, int njobs, int b)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].blk0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ================================================================ hop

// Projection data of Table 1: with the hop's spin matrix written P = v1 v1^dag + v2 v2^dag,
// v1^dag has a 1 in spin slot 3 and the unit e = i^E in slot I1, v2^dag has a 1 in slot 2 and
// f = i^F in slot I2. For 1 - gamma_mu (forward hop of M):
//   mu = x: e = i,  f = i   (I1 = 0, I2 = 1)      mu = y: e = -1, f = 1  (I1 = 0, I2 = 1)
//   mu = z: e = -i, f = i   (I1 = 1, I2 = 0)      mu = t: e = 1,  f = 1  (I1 = 1, I2 = 0)
// and 1 + gamma_mu negates e and f. Shrink: h1 = psi_3 + conj(e) psi_I1, h2 = psi_2 + conj(f) psi_I2;
// expand: col3 += g1, col I1 += e g1, col2 += g2, col I2 += f g2 with g = U h (colour multiply).
template <int MU> struct Proj;
template <> struct Proj<0> { static constexpr int E = 1, F = 1, I1 = 0, I2 = 1; };
template <> struct Proj<1> { static constexpr int E = 2, F = 0, I1 = 0, I2 = 1; };
template <> struct Proj<2> { static constexpr int E = 3, F = 1, I1 = 1, I2 = 0; };
template <> struct Proj<3> { static constexpr int E = 0, F = 0, I1 = 1, I2 = 0; };

// Where a hop reads its input sites: memory, or (STG) an LDS copy of the window [base, base + nsl)
// of input sites for the x and y directions.
template <int SF, bool STG>
struct HopIn {
    const SpinorRef& in;
    const Stg<SF, STG>& L;
    int base, nsl;
    bool tg;  // temporal gauge: unit time links inside the lattice
    bool nc;  // spinors in the non-chiral basis (the time hop of hop_t_nc)
};

template <int MU, int D, bool DAG, int SFI, bool STG, class T>
__device__ __forceinline__ void hop_dir(const Geo& g, int cb, int x, int y, int z, int t, const HopIn<SFI, STG>& in,
                                        const cx<T> W[9], cx<T> acc[12], int dep, bool unit)
{
    const int nb = nb_from_cb<MU, D>(g, cb, x, y, z, t) + dep;

    cx<T> psi[12];
    T sc = T(1);  // FP16 input: the site's scale, applied in the accumulation
    if constexpr (SFI == SF16) {
        if constexpr (STG && MU < 2) {
            const int k = nb - in.base;
            if ((unsigned)k < (unsigned)in.nsl) sc = (T)load_spinor16_stg_raw<T>(in.L, k, psi);
            else sc = (T)load_spinor16_raw<T>(in.in, nb, psi);
        } else {
            sc = (T)load_spinor16_raw<T>(in.in, nb, psi);
        }
    } else if constexpr (STG && MU < 2) {
        const int k = nb - in.base;
        if ((unsigned)k < (unsigned)in.nsl) load_spinor_stg<SFI, T>(in.L, k, psi);
        else load_spinor<SFI, T>(in.in, nb, psi);
    } else {
        load_spinor<SFI, T>(in.in, nb, psi);
    }
    constexpr bool minus = (D == 0) != DAG;  // projector 1 - gamma
    constexpr int E = Proj<MU>::E + (minus ? 0 : 2);
    constexpr int F = Proj<MU>::F + (minus ? 0 : 2);
    constexpr int I1 = Proj<MU>::I1, I2 = Proj<MU>::I2;
    cx<T> h1[3], h2[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        h1[c] = psi[c * 4 + 3] + mul_ik<-E>(psi[c * 4 + I1]);
        h2[c] = psi[c * 4 + 2] + mul_ik<-F>(psi[c * 4 + I2]);
    }
    cx<T> g1[3], g2[3];
    if (unit) {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            g1[a] = h1[a];
            g2[a] = h2[a];
        }
    } else {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            g1[a] = row_dot(W, a, h1);
            g2[a] = row_dot(W, a, h2);
        }
    }
    if constexpr (MU == 3) {
        const bool flip = g.anti && (D == 0 ? (t == g.T - 1) : (t == 0));
        if (flip) {
#pragma unroll
            for (int a = 0; a < 3; a++) { g1[a] = -g1[a]; g2[a] = -g2[a]; }
        }
    }
    if constexpr (SFI == SF16) {
        // acc += sc * g as fused multiply-adds (mul_ik only swaps and negates components)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const cx<T> e1 = mul_ik<E>(g1[c]), e2 = mul_ik<F>(g2[c]);
            acc[c * 4 + 3] = {fmaf(sc, g1[c].re, acc[c * 4 + 3].re), fmaf(sc, g1[c].im, acc[c * 4 + 3].im)};
            acc[c * 4 + 2] = {fmaf(sc, g2[c].re, acc[c * 4 + 2].re), fmaf(sc, g2[c].im, acc[c * 4 + 2].im)};
            acc[c * 4 + I1] = {fmaf(sc, e1.re, acc[c * 4 + I1].re), fmaf(sc, e1.im, acc[c * 4 + I1].im)};
            acc[c * 4 + I2] = {fmaf(sc, e2.re, acc[c * 4 + I2].re), fmaf(sc, e2.im, acc[c * 4 + I2].im)};
        }
    } else {
#pragma unroll
        for (int c = 0; c < 3; c++) {
            acc[c * 4 + 3] = acc[c * 4 + 3] + g1[c];
            acc[c * 4 + 2] = acc[c * 4 + 2] + g2[c];
            acc[c * 4 + I1] = acc[c * 4 + I1] + mul_ik<E>(g1[c]);
            acc[c * 4 + I2] = acc[c * 4 + I2] + mul_ik<F>(g2[c]);
        }
    }
}

// Directions whose loads may be scheduled together (2: the two of one axis). Larger groups let the
// compiler issue more loads at once but spill registers (FP64) or lose occupancy.
// Spin components s0, s0 + 1 of the three colours of input site i: h[a][c] = psi[c * 4 + s0 + a]
// (two of the four spin components: half the bytes of a full spinor). FP16: the stored values
// and the site's scale, returned separately (applied in the accumulation).
template <int SF, int S0, class T>
__device__ __forceinline__ T load_spin_pair(const SpinorRef& r, long i, cx<T> h[2][3])
{
    if constexpr (SF == SF64) {
#pragma unroll
        for (int c = 0; c < 3; c++)
#pragma unroll
            for (int a = 0; a < 2; a++) {
                const d2v q = gld<d2v>(r.p, chunk_at(12, r.cs, i, c * 4 + S0 + a));
                h[a][c] = mk<T>((T)q[0], (T)q[1]);
            }
        return T(1);
    } else if constexpr (SF == SF32) {
        // chunk 2c + S0/2 holds spins S0, S0 + 1 of colour c
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const f4v q = gld<f4v>(r.p, chunk_at(6, r.cs, i, 2 * c + S0 / 2));
            h[0][c] = mk<T>((T)q[0], (T)q[1]);
            h[1][c] = mk<T>((T)q[2], (T)q[3]);
        }
        return T(1);
    } else {
        // chunk c holds the four spins of colour c (8 halves): read the 8 bytes of spins S0, S0 + 1
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const h4 q = gld<h4>(r.p, 2 * chunk_at(3, r.cs, i, c) + S0 / 2);
            h[0][c] = mk<T>((T)(float)q[0], (T)(float)q[1]);
            h[1][c] = mk<T>((T)(float)q[2], (T)(float)q[3]);
        }
        return (T)gld<float>(r.nrm, i);
    }
}

// The time hop in the non-chiral basis, where gamma_4 = diag(1, 1, -1, -1): 1 - gamma_4 =
// 2 diag(0, 0, 1, 1) and 1 + gamma_4 = 2 diag(1, 1, 0, 0), so the hop reads two of the neighbour's
// spin components (S0 = 2 for the projector 1 - gamma_4, 0 for 1 + gamma_4), multiplies them by the
// link and adds twice the product to the same two components of the output: no projection sums,
// half the expansion, half the neighbour bytes of the chiral time hop.
template <int D, bool DAG, int SFI, class T>
__device__ __forceinline__ void hop_t_nc(const Geo& g, int cb, int x, int y, int z, int t, const SpinorRef& in,
                                         const cx<T> W[9], cx<T> acc[12], int dep, bool unit)
{
    constexpr bool minus = (D == 0) != DAG;  // projector 1 - gamma_4
    constexpr int S0 = minus ? 2 : 0;
    const int nb = nb_from_cb<3, D>(g, cb, x, y, z, t) + dep;
    cx<T> h[2][3];
    const T sc = load_spin_pair<SFI, S0, T>(in, nb, h);
    cx<T> gg[2][3];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int c = 0; c < 3; c++)
            gg[a][c] = unit ? h[a][c] : row_dot(W, c, h[a]);
    // twice the product, with the boundary sign and (FP16 input) the site's scale
    const bool flip = g.anti && (D == 0 ? (t == g.T - 1) : (t == 0));
    const T f = (flip ? T(-2) : T(2)) * sc;
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            cx<T>& o = acc[c * 4 + S0 + a];
            o = {fmaf_t(f, gg[a][c].re, o.re), fmaf_t(f, gg[a][c].im, o.im)};
        }
}

template <int SF> struct HopGroup { static constexpr int G = 2; };

// Between groups of directions: an empty asm that reads every accumulator and then "writes"
// the zero offset used by the next group's addresses. The volatile asms keep their order, so
// the next group's loads cannot be issued before this group's results exist, which bounds the
// number of live load registers (the FP64 hop otherwise spills).
template <class T>
__device__ __forceinline__ void order_after(cx<T> acc[12], int& dep)
{
#pragma unroll
    for (int k = 0; k < 12; k += 3)
        asm volatile("" ::"v"(acc[k].re), "v"(acc[k].im), "v"(acc[k + 1].re), "v"(acc[k + 1].im), "v"(acc[k + 2].re),
                     "v"(acc[k + 2].im));
    asm volatile("" : "+v"(dep));
}

template <int D, int G, class T>
__device__ __forceinline__ void group_barrier(cx<T> acc[12], int& dep)
{
    // after direction D (0..7): close the group
    if constexpr (G < 8 && ((D + 1) % G) == 0 && D < 7) order_after(acc, dep);
}

// Both directions of axis MU; the two links are loaded together (one 16-byte load per chunk for
// the paired 16-bit formats). G = directions per ordering group. NTL: non-temporal link loads.
template <int MU, int G, bool DAG, int SFI, int LF, bool STG, bool NTL, class T>
__device__ __forceinline__ void hop_axis(const Geo& g, int cb, int x, int y, int z, int t, const HopIn<SFI, STG>& in,
                                         const void* links, long lcs, cx<T> acc[12], int& dep)
{
    cx<T> Wf[9], Wb[9];
    // temporal gauge: U_t(n) is the unit matrix unless t = T - 1, U_t(n - t)^dag unless t = 0
    const bool unit_f = MU == 3 && in.tg && t != g.T - 1;
    const bool unit_b = MU == 3 && in.tg && t != 0;
    if (!(unit_f && unit_b)) {
        load_link_pair<LF, T, NTL>(links, lcs, MU, cb + dep, Wf, Wb);
    }
    if (MU == 3 && in.nc) {
        hop_t_nc<0, DAG, SFI, T>(g, cb, x, y, z, t, in.in, Wf, acc, dep, unit_f);
        group_barrier<2 * MU, G>(acc, dep);
        hop_t_nc<1, DAG, SFI, T>(g, cb, x, y, z, t, in.in, Wb, acc, dep, unit_b);
        group_barrier<2 * MU + 1, G>(acc, dep);
        return;
    }
    hop_dir<MU, 0, DAG, SFI, STG, T>(g, cb, x, y, z, t, in, Wf, acc, dep, unit_f);
    group_barrier<2 * MU, G>(acc, dep);
    hop_dir<MU, 1, DAG, SFI, STG, T>(g, cb, x, y, z, t, in, Wb, acc, dep, unit_b);
    group_barrier<2 * MU + 1, G>(acc, dep);
}

template <bool DAG, int SFI, int LF, bool STG, bool NTL, class T>
__device__ __forceinline__ void hop_site(const Geo& g, int p, int cb, const HopIn<SFI, STG>& in, const void* links,
                                         long lcs, cx<T> acc[12])
{
    constexpr int G = HopGroup<SFI>::G;
    int x, y, z, t;
    cb_coords(g, p, cb, x, y, z, t);
#pragma unroll
    for (int k = 0; k < 12; k++) acc[k] = mk<T>(T(0), T(0));
    int dep = 0;
    hop_axis<0, G, DAG, SFI, LF, STG, NTL, T>(g, cb, x, y, z, t, in, links, lcs, acc, dep);
    hop_axis<1, G, DAG, SFI, LF, STG, NTL, T>(g, cb, x, y, z, t, in, links, lcs, acc, dep);
    hop_axis<2, G, DAG, SFI, LF, STG, NTL, T>(g, cb, x, y, z, t, in, links, lcs, acc, dep);
    hop_axis<3, G, DAG, SFI, LF, STG, NTL, T>(g, cb, x, y, z, t, in, links, lcs, acc, dep);
}

// Job-local block order. With tz > 0 the blocks walk t fastest inside groups of tz z-planes, so a
// block's t +- 1 neighbours were (or are about to be) loaded by blocks running on the same XCD at
// nearly the same time, while the site order would put them a whole t-slice apart.
__device__ __forceinline__ int tiled_block(const HopJob& J, int lb)
{
    if (J.tz <= 0) return lb;
    const int q = lb % J.bpp;
    int r = lb / J.bpp;
    const int zz = r % J.tz;
    r /= J.tz;
    const int t = r % J.g.T;
    const int zg = r / J.g.T;
    return q + J.bpp * ((zg * J.tz + zz) + J.g.Z * t);
}

// TG: some job of the launch has temporal-gauge links (TG = false compiles the unit-link paths out).
// NTL: the links are loaded non-temporally, so that they do not evict the neighbour spinors from
// L2; launches with interleaved systems (links shared through L2) take ordinary loads. The same
// variant loads the epilogue's own-site fields (x0, x1, z), which are read once, non-temporally and
// stores the output non-temporally, except the low-precision plain hop (D_oe of M_prec), whose
// output the next hop gathers at once (measured: that hop 102.5 -> 97.5 us at 32^3x64 with FP32
// spinors; the FP64 plain hop is faster with non-temporal stores). A compile-time choice: as a
// run-time branch the compiler merges the two identical loads and drops the hint.
template <int SF, int LF, bool DAG, int RED, int FIN, bool STG, bool NTL, bool TG>
__global__ __launch_bounds__(BLOCK) void k_hop(
    const HopJob* __restrict__ jobs, int njobs, SysState* __restrict__ sys, int gated, int* exec)
{
    using T = typename SReal<SF>::T;
    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    int jx = find_job(jobs, njobs, b);
    int lb = b - jobs[jx].blk0;
    if (jobs[jx].ilv > 1) {
        // interleaved group: find_job returned its last job
        const int K = jobs[jx].ilv;
        jx = jx - jobs[jx].ilv_pos + lb % K;
        lb /= K;
    }
    const HopJob& J = jobs[jx];
    SysState* S = sys + J.sys;
    if (gated && !((gated >> S->status) & 1)) return;  // gated: mask of the statuses that run
    if (exec && lb == 0 && threadIdx.x == 0) atomicAdd(exec, 1);  // timing: jobs that did work
    const int cb0 = tiled_block(J, lb) * BLOCK;
    const int cb = cb0 + threadIdx.x;
    __shared__ Stg<SF, STG> stg;
    int base = 0, nsl = 0;
    if constexpr (STG) {
        const int H = J.g.Xh <= STG_H_MAX ? J.g.Xh : 0;
        base = cb0 - H;
        nsl = BLOCK + 2 * H;
        stage_window<SF>(stg, J.in, base, nsl, J.g.Vh);
        stage_wait();
        __syncthreads();
    }
    const HopIn<SF, STG> hin{J.in, stg, base, nsl, TG && J.tg != 0, J.nc != 0};
    double v[NRED] = {0.0, 0.0, 0.0, 0.0};
    if (cb < J.g.Vh) {
        cx<T> acc[12];
        hop_site<DAG, SF, LF, STG, NTL, T>(J.g, J.parity, cb, hin, J.links, J.lcs, acc);
        const T c2 = (T)J.c2;
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k] = c2 * acc[k];
        cx<T> x0[12];
        if (J.x0.p) {
            load_spinor<SF, T, NTL>(J.x0, cb, x0);
            const T c0 = (T)J.c0;
#pragma unroll
            for (int k = 0; k < 12; k++) acc[k] = acc[k] + c0 * x0[k];
        }
        if (J.x1.p) {
            cx<T> x1[12];
            load_spinor<SF, T, NTL>(J.x1, cb, x1);
            const T c1 = (T)J.c1;
#pragma unroll
            for (int k = 0; k < 12; k++) acc[k] = acc[k] + c1 * x1[k];
        }
        store_spinor<SF, T, NTL && (RED != RED_NONE || SF == SF64)>(J.out, cb, acc);
        if constexpr (RED == RED_ZDOT) {
            cx<T> z[12];
            load_spinor<SF, T, NTL>(J.z, cb, z);
#pragma unroll
            for (int k = 0; k < 12; k++) {
                v[0] += (double)z[k].re * acc[k].re + (double)z[k].im * acc[k].im;
                v[1] += (double)z[k].re * acc[k].im - (double)z[k].im * acc[k].re;
            }
        } else if constexpr (RED == RED_OUTX) {
#pragma unroll
            for (int k = 0; k < 12; k++) {
                v[0] += (double)acc[k].re * x0[k].re + (double)acc[k].im * x0[k].im;
                v[1] += (double)acc[k].re * x0[k].im - (double)acc[k].im * x0[k].re;
                v[2] += (double)acc[k].re * acc[k].re + (double)acc[k].im * acc[k].im;
            }
        } else if constexpr (RED == RED_NORM) {
#pragma unroll
            for (int k = 0; k < 12; k++) v[2] += (double)acc[k].re * acc[k].re + (double)acc[k].im * acc[k].im;
        }
    }
    if constexpr (RED != RED_NONE) write_partials<3>(v, S, J.rblk0 + lb);
}

// ================================================================ launch dispatch

static inline dim3 grid1(long nblk) { return dim3((unsigned)nblk); }

#define HOP_LAUNCH(SF_, LF_, DAG_, RED_, FIN_, STG_, TG_)                                                          \
    if (ntl) hipExtLaunchKernelGGL((k_hop<SF_, LF_, DAG_, RED_, FIN_, STG_, true, TG_>), grid1(nblocks), dim3(BLOCK), 0, s, \
                                   ev0, ev1, 0, jobs, njobs, sys, gated, exec);                                    \
    else hipExtLaunchKernelGGL((k_hop<SF_, LF_, DAG_, RED_, FIN_, STG_, false, TG_>), grid1(nblocks), dim3(BLOCK), 0, s, \
                               ev0, ev1, 0, jobs, njobs, sys, gated, exec)
// The kernel does not depend on the finisher run after it (FIN_ names the instantiation only): the
// launch is chosen by the reduction kind.
#define HOP_CASE(SF_, LF_, DAG_, RED_, FIN_)                                                                        \
    if (sf == SF_ && lf == LF_ && dag == DAG_ && red == RED_) {                                                    \
        const bool stg_ = (SF_ != SF64 ? stage : stage64) != 0;                                                    \
        if (stg_ && tg) HOP_LAUNCH(SF_, LF_, DAG_, RED_, FIN_, true, !DAG_);                                       \
        else if (stg_) HOP_LAUNCH(SF_, LF_, DAG_, RED_, FIN_, true, false);                                        \
        else if (tg) HOP_LAUNCH(SF_, LF_, DAG_, RED_, FIN_, false, !DAG_);                                         \
        else HOP_LAUNCH(SF_, LF_, DAG_, RED_, FIN_, false, false);                                                 \
        return hipGetLastError();                                                                                  \
    }
#define HOP_REDS(SF_, LF_, DAG_)                                                                                   \
    HOP_CASE(SF_, LF_, DAG_, RED_NONE, FIN_STORE)                                                                  \
    HOP_CASE(SF_, LF_, DAG_, RED_NORM, FIN_STORE)                                                                  \
    HOP_CASE(SF_, LF_, DAG_, RED_ZDOT, FIN_BETA)                                                                   \
    HOP_CASE(SF_, LF_, DAG_, RED_OUTX, FIN_CHI)
// the adjoint hops of the normal equations (CG): the iteration's two, plus the FP64 residual's
#define HOP_DAG_LO(SF_, LF_)                                                                                       \
    HOP_CASE(SF_, LF_, true, RED_NONE, FIN_STORE)                                                                  \
    HOP_CASE(SF_, LF_, true, RED_ZDOT, FIN_BETA)
#define HOP_DAG_64(LF_) HOP_DAG_LO(SF64, LF_) HOP_CASE(SF64, LF_, true, RED_NORM, FIN_STORE)

} // namespace wd
