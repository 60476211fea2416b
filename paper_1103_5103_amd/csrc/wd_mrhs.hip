// Multi-RHS hop (the link reuse across right-hand sides that Sec. 4 discusses as data reuse per
// thread): one thread per output site applies the hopping term to the K systems of a group that
// share one gauge field, loading each of the site's 8 links once for all of them. Per output site
// and system the compulsory traffic drops from 2 spinors + 8 links to 2 spinors + 8 links / K.
//
// The K accumulators stay in registers (24 K floats); each link is rebuilt once and multiplied
// into the K projected neighbours. After every axis an ordering point consumes the accumulators,
// so the next axis's loads cannot all be hoisted at once (which would exceed the register file). The epilogue (out = c0 x0 + c1 x1 + c2 hop) and the fused FP64 reductions
// are those of k_hop, per system.
//
// Every system's x/y window is staged in LDS, as in k_hop. Besides saving the x/y gathers this
// sizes the launch for the L2: a block holds K systems' sites, so the neighbour spinors that
// blocks in flight on one XCD re-read from L2 grow K-fold; K windows of LDS per block cut the
// blocks per CU to about 1/K of k_hop's, which keeps that working set near k_hop's (without it
// the FP32 hop with K = 2 ran 1.65 times slower per system than one system per thread).
#include "wd_hop.hpp"

namespace wd {

template <int KT, class T>
__device__ __forceinline__ void order_after_k(cx<T> acc[KT][12], int& dep)
{
#pragma unroll
    for (int k = 0; k < KT; k++)
#pragma unroll
        for (int c = 0; c < 12; c += 3)
            asm volatile("" ::"v"(acc[k][c].re), "v"(acc[k][c].im), "v"(acc[k][c + 1].re), "v"(acc[k][c + 1].im),
                         "v"(acc[k][c + 2].re), "v"(acc[k][c + 2].im));
    asm volatile("" : "+v"(dep));
}

// both directions of axis MU for every running system of the group; stg[k]: system k's LDS
// window [base, base + nsl) of input sites. One ordering group per axis: the block's LDS windows
// already hold the occupancy at about 8 / K waves per CU, so the registers for both links and the
// 2 K neighbour spinors of an axis are free, and more loads are in flight per wave.
template <int MU, bool DAG, int SF, int LF, int KT, class T>
__device__ __forceinline__ void mrhs_axis(const HopJob* __restrict__ jobs, int j0, const bool run[KT], const Geo& g,
                                          int cb, int x, int y, int z, int t, bool tg, const Stg<SF, true>* stg,
                                          int base, int nsl, cx<T> acc[KT][12], int& dep)
{
    const HopJob& J0 = jobs[j0];
    // temporal gauge: U_t(n) is the unit matrix unless t = T - 1, U_t(n - t)^dag unless t = 0
    const bool unit_f = MU == 3 && tg && t != g.T - 1;
    const bool unit_b = MU == 3 && tg && t != 0;
    cx<T> Wf[9], Wb[9];
    if (!(unit_f && unit_b)) load_link_pair<LF, T, true>(J0.links, J0.lcs, MU, cb + dep, Wf, Wb);
    const bool nc = MU == 3 && J0.nc != 0;  // the systems of a group share one handle, hence its basis
#pragma unroll
    for (int k = 0; k < KT; k++)
        if (run[k]) {
            if (nc) {
                hop_t_nc<0, DAG, SF, T>(g, cb, x, y, z, t, jobs[j0 + k].in, Wf, acc[k], dep, unit_f);
                hop_t_nc<1, DAG, SF, T>(g, cb, x, y, z, t, jobs[j0 + k].in, Wb, acc[k], dep, unit_b);
                continue;
            }
            const HopIn<SF, true> in{jobs[j0 + k].in, stg[k], base, nsl, tg, false};
            hop_dir<MU, 0, DAG, SF, true, T>(g, cb, x, y, z, t, in, Wf, acc[k], dep, unit_f);
            hop_dir<MU, 1, DAG, SF, true, T>(g, cb, x, y, z, t, in, Wb, acc[k], dep, unit_b);
        }
    order_after_k<KT, T>(acc, dep);
}

template <int SF, int LF, bool DAG, int RED, int KT>
__global__ __launch_bounds__(BLOCK) void k_hop_mrhs(const HopJob* __restrict__ jobs, int njobs,
                                                    SysState* __restrict__ sys, int gated, int* exec)
{
    using T = float;
    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int jl = find_job(jobs, njobs, b);  // the last job of the group (all share blk0)
    const int K = jobs[jl].ilv;
    const int j0 = jl - jobs[jl].ilv_pos;
    const HopJob& J0 = jobs[j0];
    const int lb = b - J0.blk0;
    bool run[KT];
    bool any = false;
#pragma unroll
    for (int k = 0; k < KT; k++) {
        run[k] = k < K && (!gated || ((gated >> sys[jobs[j0 + k].sys].status) & 1));  // gated: mask of statuses
        any = any || run[k];
    }
    if (!any) return;
    if (exec && lb == 0 && threadIdx.x == 0)
        for (int k = 0; k < KT; k++)
            if (run[k]) atomicAdd(exec, 1);  // timing: jobs that did work
    const int cb0 = tiled_block(J0, lb) * BLOCK;
    const int cb = cb0 + threadIdx.x;
    // each running system's window of input sites: the block's rows and one row above and below
    __shared__ Stg<SF, true> stg[KT];
    const int H = J0.g.Xh <= STG_H_MAX ? J0.g.Xh : 0;
    const int base = cb0 - H, nsl = BLOCK + 2 * H;
#pragma unroll
    for (int k = 0; k < KT; k++)
        if (run[k]) stage_window<SF>(stg[k], jobs[j0 + k].in, base, nsl, J0.g.Vh);
    stage_wait();
    __syncthreads();
    double v[KT][NRED];
#pragma unroll
    for (int k = 0; k < KT; k++)
#pragma unroll
        for (int r = 0; r < NRED; r++) v[k][r] = 0.0;
    if (cb < J0.g.Vh) {
        const Geo& g = J0.g;
        int x, y, z, t;
        cb_coords(g, J0.parity, cb, x, y, z, t);
        const bool tg = J0.tg != 0;
        cx<T> acc[KT][12];
#pragma unroll
        for (int k = 0; k < KT; k++)
#pragma unroll
            for (int c = 0; c < 12; c++) acc[k][c] = mk<T>(T(0), T(0));
        int dep = 0;
        mrhs_axis<0, DAG, SF, LF, KT, T>(jobs, j0, run, g, cb, x, y, z, t, tg, stg, base, nsl, acc, dep);
        mrhs_axis<1, DAG, SF, LF, KT, T>(jobs, j0, run, g, cb, x, y, z, t, tg, stg, base, nsl, acc, dep);
        mrhs_axis<2, DAG, SF, LF, KT, T>(jobs, j0, run, g, cb, x, y, z, t, tg, stg, base, nsl, acc, dep);
        mrhs_axis<3, DAG, SF, LF, KT, T>(jobs, j0, run, g, cb, x, y, z, t, tg, stg, base, nsl, acc, dep);
#pragma unroll
        for (int k = 0; k < KT; k++) {
            if (!run[k]) continue;
            const HopJob& J = jobs[j0 + k];
            const T c2 = (T)J.c2;
#pragma unroll
            for (int c = 0; c < 12; c++) acc[k][c] = c2 * acc[k][c];
            cx<T> x0[12];
            if (J.x0.p) {
                load_spinor<SF, T>(J.x0, cb, x0);
                const T c0 = (T)J.c0;
#pragma unroll
                for (int c = 0; c < 12; c++) acc[k][c] = acc[k][c] + c0 * x0[c];
            }
            if (J.x1.p) {
                cx<T> x1[12];
                load_spinor<SF, T>(J.x1, cb, x1);
                const T c1 = (T)J.c1;
#pragma unroll
                for (int c = 0; c < 12; c++) acc[k][c] = acc[k][c] + c1 * x1[c];
            }
            // the output is not read again within the launch
            store_spinor<SF, T, true>(J.out, cb, acc[k]);
            if constexpr (RED == RED_ZDOT) {
                cx<T> zz[12];
                load_spinor<SF, T>(J.z, cb, zz);
#pragma unroll
                for (int c = 0; c < 12; c++) {
                    v[k][0] += (double)zz[c].re * acc[k][c].re + (double)zz[c].im * acc[k][c].im;
                    v[k][1] += (double)zz[c].re * acc[k][c].im - (double)zz[c].im * acc[k][c].re;
                }
            } else if constexpr (RED == RED_OUTX) {
#pragma unroll
                for (int c = 0; c < 12; c++) {
                    v[k][0] += (double)acc[k][c].re * x0[c].re + (double)acc[k][c].im * x0[c].im;
                    v[k][1] += (double)acc[k][c].re * x0[c].im - (double)acc[k][c].im * x0[c].re;
                    v[k][2] += (double)acc[k][c].re * acc[k][c].re + (double)acc[k][c].im * acc[k][c].im;
                }
            } else if constexpr (RED == RED_NORM) {
#pragma unroll
                for (int c = 0; c < 12; c++)
                    v[k][2] += (double)acc[k][c].re * acc[k][c].re + (double)acc[k][c].im * acc[k][c].im;
            }
        }
    }
    if constexpr (RED != RED_NONE) {
        // block-uniform conditions: every thread of the block takes the same branches
#pragma unroll
        for (int k = 0; k < KT; k++)
            if (run[k]) write_partials<3>(v[k], sys + jobs[j0 + k].sys, jobs[j0 + k].rblk0 + lb);
    }
}

#define MRHS_LAUNCH(SF_, LF_, DAG_, RED_, KT_)                                                                      \
    if (sf == SF_ && lf == LF_ && dag == DAG_ && red == RED_ && kt == KT_) {                                      \
        hipExtLaunchKernelGGL((k_hop_mrhs<SF_, LF_, DAG_, RED_, KT_>), grid1(nblocks), dim3(BLOCK), 0, s, ev0, ev1, \
                              0, jobs, njobs, sys, gated, exec);                                                   \
        return hipGetLastError();                                                                                  \
    }
#define MRHS_REDS(SF_, LF_, KT_)                                                                                   \
    MRHS_LAUNCH(SF_, LF_, false, RED_NONE, KT_)                                                                    \
    MRHS_LAUNCH(SF_, LF_, false, RED_ZDOT, KT_)                                                                    \
    MRHS_LAUNCH(SF_, LF_, false, RED_OUTX, KT_)                                                                    \
    MRHS_LAUNCH(SF_, LF_, true, RED_NONE, KT_)                                                                     \
    MRHS_LAUNCH(SF_, LF_, true, RED_ZDOT, KT_)
#define MRHS_LINKS(SF_, KT_)                                                                                       \
    MRHS_REDS(SF_, L32_12, KT_) MRHS_REDS(SF_, L16_12, KT_) MRHS_REDS(SF_, LB16_12, KT_) MRHS_REDS(SF_, L16_8, KT_)

int mrhs_kt(int k) { return k <= 2 ? 2 : k <= 4 ? 4 : 0; }

hipError_t launch_hop_mrhs(int sf, int lf, bool dag, int red, int kt, const HopJob* jobs, int njobs, long nblocks,
                           SysState* sys, int gated, hipStream_t s, int* exec, hipEvent_t ev0, hipEvent_t ev1)
{
    if (nblocks <= 0) return hipSuccess;
    MRHS_LINKS(SF32, 2)
    MRHS_LINKS(SF16, 2)
    MRHS_LINKS(SF32, 4)
    MRHS_LINKS(SF16, 4)
    return hipErrorInvalidValue;
}

} // namespace wd
