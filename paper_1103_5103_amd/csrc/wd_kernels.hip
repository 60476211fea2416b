// Kernels of libwdirac for gfx950 (CDNA4, wave64).
//
//  * k_hop     : the Wilson hopping term between parities (Sec. 2, eq. 3-4; the paper's dslash,
//                Alg. 1) with the spin-projection trick of Table 1 and a fused epilogue
//                out = c0 x0 + c1 x1 + c2 * hop, optionally followed by FP64 reductions and a
//                finisher that updates the solver scalars; the adjoint (DAG) variant serves the
//                normal equations of CG / CG-M (Sec. 8).
//  * k_sweep   : the fused BiCGstab vector updates of one iteration (Sec. 5: the x <- x - beta s +
//                chi w update and its companions), the BiCGstab-M shift sweep (Sec. 6.1), and the
//                CG / CG-M updates.
//  * k_finish  : fixed-order sums of the block partials and the scalar recurrences.
//  * k_guess   : the sequential start vector (Sec. 6.2.1) and its residual without the operator.
//  * packing   : canonical complex128 layout <-> internal checkerboarded structure of arrays;
//                k_unpack_eo also rebuilds the odd half from eq. eo3.
//  * k_grad    : link derivative of Re<eta, M^{-1} b> (outer products of projected spinors).
#include "wd_hop.hpp"

#include <cstdlib>

namespace wd {

// LDS staging of the x and y neighbours in the hop (both the low-precision and the FP64 hop; a
// launch may turn it off, which changes no arithmetic)
int hop_stage_default() { return 1; }
int hop_stage64_default() { return 1; }

// ================================================================ finishers

__device__ __forceinline__ double2 c_div(double2 a, double2 b)
{
    double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double2 c_mul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 c_neg(double2 a) { return make_double2(-a.x, -a.y); }
__device__ __forceinline__ double2 c_real(double r) { return make_double2(r, 0.0); }
__device__ __forceinline__ double c_abs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ bool c_finite(double2 a) { return isfinite(a.x) && isfinite(a.y); }

template <int FIN>
__device__ void finish(SysState* S, const double* tot)
{
    for (int k = 0; k < NRED; k++) S->red[k] = tot[k];
    if constexpr (FIN == FIN_BETA) {
        const double2 rhAs = make_double2(tot[0], tot[1]);
        if (!c_finite(rhAs)) { S->status = ST_NAN; return; }
        if (c_abs2(rhAs) == 0.0) { S->status = ST_BREAKDOWN; return; }
        const double2 beta = c_neg(c_div(S->delta, rhAs));
        S->beta = beta;
        // shifted systems: zeta_{n+1} and beta^sigma_n from the collinearity of the residuals
        for (int i = 0; i < S->nshift; i++) {
            ShiftScal& q = S->sh[i];
            if (!q.active) continue;
            // den = beta alpha (zeta_prev - zeta) + zeta_prev beta_prev (1 - sigma beta)
            double2 den = c_add(c_mul(c_mul(beta, S->alpha), c_sub(q.zeta_prev, q.zeta)),
                                c_mul(c_mul(q.zeta_prev, S->beta_prev),
                                      c_sub(c_real(1.0), c_mul(c_real(q.sigma), beta))));
            q.zeta_next = c_div(c_mul(c_mul(q.zeta, q.zeta_prev), S->beta_prev), den);
            q.beta_s = c_div(c_mul(beta, q.zeta_next), q.zeta);
        }
    } else if constexpr (FIN == FIN_CHI) {
        const double2 aww = make_double2(tot[0], tot[1]);
        const double awaw = tot[2];
        if (!c_finite(aww) || !isfinite(awaw)) { S->status = ST_NAN; return; }
        if (awaw == 0.0) { S->status = ST_BREAKDOWN; return; }
        const double2 chi = make_double2(aww.x / awaw, aww.y / awaw);
        S->chi = chi;
        for (int i = 0; i < S->nshift; i++) {
            ShiftScal& q = S->sh[i];
            if (!q.active) continue;
            double2 d = c_add(c_real(1.0), c_mul(chi, c_real(q.sigma)));
            q.chi_s = c_div(chi, d);
            q.rho_next = c_div(q.rho, d);
        }
    } else if constexpr (FIN == FIN_ALPHA) {
        const double2 d1 = make_double2(tot[0], tot[1]);
        const double rr = tot[2];
        S->iter += 1;
        S->rr = rr;
        const double2 alpha = c_neg(c_div(c_mul(S->beta, d1), c_mul(S->delta, S->chi)));
        int pend = ST_RUNNING;
        if (!isfinite(rr) || !c_finite(d1)) pend = ST_NAN;
        else if (rr <= S->target2) pend = ST_CONVERGED;
        else if (S->mixed && rr < S->delta_rel2 * S->maxrr) pend = ST_RELIABLE;
        else if (S->iter >= S->maxit) pend = ST_MAXIT;
        else if (c_abs2(d1) == 0.0) pend = ST_BREAKDOWN;
        S->pending = pend;
        // no shifted scalars to rotate: commit now instead of in a separate end-of-iteration
        // finisher. The s update of this iteration is then gated off for a system that stops;
        // a solver that continues from s (reliable update) applies it before the update.
        if (S->nshift == 0) S->status = pend;
        if (!S->dc && rr > S->maxrr) S->maxrr = rr;
        for (int i = 0; i < S->nshift; i++) {
            ShiftScal& q = S->sh[i];
            if (!q.active) continue;
            // alpha^sigma_{n+1} = alpha_{n+1} zeta_{n+1} beta^sigma_n / (zeta_n beta_n)
            q.alpha_s = c_div(c_mul(c_mul(alpha, q.zeta_next), q.beta_s), c_mul(q.zeta, S->beta));
            double2 zr = c_mul(q.zeta_next, q.rho_next);
            if (c_abs2(zr) * rr < S->shift_target2) q.freeze = 1;
        }
        S->alpha = alpha;
        S->delta = d1;
    } else if constexpr (FIN == FIN_END) {
        S->status = S->pending;
        S->beta_prev = S->beta;
        for (int i = 0; i < S->nshift; i++) {
            ShiftScal& q = S->sh[i];
            if (!q.active) continue;
            q.zeta_prev = q.zeta;
            q.zeta = q.zeta_next;
            q.rho = q.rho_next;
            if (q.freeze) { q.active = 0; q.conv_iter = S->iter; }
        }
        if (S->nshift > 0) S->rsel ^= 1;
    } else if constexpr (FIN == FIN_RESTART) {
        S->delta = make_double2(tot[0], tot[1]);
        S->rr = tot[2];
        S->maxrr = tot[2];
        S->status = (isfinite(tot[2]) && c_finite(S->delta)) ? ST_RUNNING : ST_NAN;
        S->pending = S->status;
    } else if constexpr (FIN == FIN_CGA) {
        // CG: alpha_n = |r_n|^2 / <p_n, A p_n> (tot[0] = Re <p, A p>; A Hermitian positive definite)
        const double pAp = tot[0];
        if (!isfinite(pAp)) { S->status = ST_NAN; return; }
        if (!(pAp > 0.0)) { S->status = ST_BREAKDOWN; return; }
        const double alpha = S->rr / pAp;
        // CG-M: zeta_{n+1} from the collinearity of the shifted residuals, alpha^s_n = alpha_n zeta_{n+1} / zeta_n
        for (int i = 0; i < S->nshift; i++) {
            ShiftScal& q = S->sh[i];
            if (!q.active) continue;
            const double zp = q.zeta_prev.x, z = q.zeta.x;
            const double den = zp * S->cga_prev * (1.0 + alpha * q.sigma) + alpha * S->cgb * (zp - z);
            const double zn = z * zp * S->cga_prev / den;
            q.zeta_next = c_real(zn);
            q.alpha_s = c_real(alpha * zn / z);
        }
        S->cga = alpha;
    } else if constexpr (FIN == FIN_CGB) {
        // CG: beta_{n+1} = |r_{n+1}|^2 / |r_n|^2 (tot[2] = |r_{n+1}|^2) and the exit test
        const double rr = tot[2];
        S->iter += 1;
        const double beta = rr / S->rr;
        int pend = ST_RUNNING;
        if (!isfinite(rr)) pend = ST_NAN;
        else if (rr <= S->target2) pend = ST_CONVERGED;
        else if (S->mixed && rr < S->delta_rel2 * S->maxrr) pend = ST_RELIABLE;
        else if (S->iter >= S->maxit) pend = ST_MAXIT;
        S->pending = pend;
        // single system: commit now (the p update of a system that stops is gated off, and a
        // continuing reliable update applies it first); CG-M commits after its shift sweep
        if (S->nshift == 0) S->status = pend;
        if (!S->dc && rr > S->maxrr) S->maxrr = rr;
        for (int i = 0; i < S->nshift; i++) {
            ShiftScal& q = S->sh[i];
            if (!q.active) continue;
            const double g = q.zeta_next.x / q.zeta.x;
            q.beta_s = c_real(beta * g * g);
            if (q.zeta_next.x * q.zeta_next.x * rr <= S->shift_target2) q.freeze = 1;
        }
        S->rr = rr;
        S->cgb = beta;
        S->cga_prev = S->cga;
    } else if constexpr (FIN == FIN_CGEND) {
        S->status = S->pending;
        for (int i = 0; i < S->nshift; i++) {
            ShiftScal& q = S->sh[i];
            if (!q.active) continue;
            q.zeta_prev = q.zeta;
            q.zeta = q.zeta_next;
            if (q.freeze) { q.active = 0; q.conv_iter = S->iter; }
        }
    }
}

// One block per system: fixed-order sum of the partials of the preceding kernel, then the
// finisher. Gated launches skip systems that were not RUNNING (the preceding kernel skipped
// them too, since only finishers change the status).
template <int NR, int FIN>
__global__ __launch_bounds__(BLOCK) void k_finish(const FinJob* __restrict__ fin, SysState* __restrict__ sys,
                                                  int gated)
{
    __shared__ double lds[NRED * (BLOCK / 64)];
    const FinJob F = fin[blockIdx.x];
    SysState* S = sys + F.sys;
    if (gated && !((gated >> S->status) & 1)) return;  // gated: mask of the statuses that run
    double tot[NRED] = {0.0, 0.0, 0.0, 0.0};
    if constexpr (NR > 0) {
        for (int i = threadIdx.x; i < F.rnblk; i += BLOCK) {
#pragma unroll
            for (int k = 0; k < NR; k++) tot[k] += S->partials[(long)i * NRED + k];
        }
        block_sum<NR>(tot, lds);
    }
    if (threadIdx.x == 0) finish<FIN>(S, tot);
}

// ================================================================ sweeps

template <class T> __device__ __forceinline__ cx<T> cvt(double2 a) { return mk<T>((T)a.x, (T)a.y); }

template <int OP, int SFL>
__global__ __launch_bounds__(BLOCK) void k_sweep(const SweepJob* __restrict__ jobs, int njobs,
                                                 SysState* __restrict__ sys, int gated, int* exec)
{
    using T = typename SReal<SFL>::T;
    constexpr int SFX = SFL == SF64 ? SF64 : SF32;  // storage of the low-precision solution
    // A sweep reads every field once: non-temporal loads. Its outputs are stored non-temporally
    // too, except those of the low-precision x / r update, whose new residual the next sweep reads
    // at once (measured on the 32^3x64 mixed solves: sweeps 4.9 -> 5.2-5.6 TB/s, and the hops that
    // follow them 2% faster).
    constexpr bool NTS = !(OP == OP_XR && SFL != SF64);
    const int b = blockIdx.x;
    const SweepJob& J = jobs[find_job(jobs, njobs, b)];
    SysState* S = sys + J.sys;
    if (gated && !((gated >> S->status) & 1)) return;  // gated: mask of the statuses that run
    const int lb = b - J.blk0;
    if (exec && lb == 0 && threadIdx.x == 0) atomicAdd(exec, 1);
    const long i = (long)lb * BLOCK + threadIdx.x;
    const bool ok = i < J.n;
    double v[NRED] = {0.0, 0.0, 0.0, 0.0};
    const int rsel = S->rsel;
    const SpinorRef& Rcur = rsel ? J.f[R_F3] : J.f[R_F1];  // OP_W / OP_S / OP_SHIFT role layout
    const SpinorRef& Rnxt = rsel ? J.f[R_F1] : J.f[R_F3];

    if constexpr (OP == OP_W) {
        // w = r + beta A s
        if (ok) {
            const cx<T> beta = cvt<T>(S->beta);
            cx<T> r[12], as[12];
            load_spinor<SFL, T, true>(Rcur, i, r);
            load_spinor<SFL, T, true>(J.f[R_F2], i, as);
#pragma unroll
            for (int k = 0; k < 12; k++) r[k] = r[k] + beta * as[k];
            store_spinor<SFL, T, NTS>(J.f[R_F0], i, r);
        }
    } else if constexpr (OP == OP_XR) {
        // x <- x - beta s + chi w ; r_{n+1} = w - chi A w ; <rhat, r_{n+1}>, |r_{n+1}|^2
        if (ok) {
            const cx<T> beta = cvt<T>(S->beta), chi = cvt<T>(S->chi);
            cx<T> x[12], s[12], w[12];
            load_spinor<SFX, T, true>(J.f[R_F0], i, x);
            load_spinor<SFL, T, true>(J.f[R_F2], i, s);
            load_spinor<SFL, T, true>(J.f[R_F3], i, w);
#pragma unroll
            for (int k = 0; k < 12; k++) x[k] = x[k] - beta * s[k] + chi * w[k];
            store_spinor<SFX, T, NTS>(J.f[R_F0], i, x);
            cx<T> aw[12];
            load_spinor<SFL, T, true>(J.f[R_F4], i, aw);
#pragma unroll
            for (int k = 0; k < 12; k++) w[k] = w[k] - chi * aw[k];
            // the new residual goes to the buffer not holding r_n
            store_spinor<SFL, T, NTS>(rsel ? J.f[R_F1] : J.f[R_F6], i, w);
            cx<T> rh[12];
            load_spinor<SFL, T, true>(J.f[R_F5], i, rh);
#pragma unroll
            for (int k = 0; k < 12; k++) {
                v[0] += (double)rh[k].re * w[k].re + (double)rh[k].im * w[k].im;
                v[1] += (double)rh[k].re * w[k].im - (double)rh[k].im * w[k].re;
                v[2] += (double)w[k].re * w[k].re + (double)w[k].im * w[k].im;
            }
        }
        write_partials<3>(v, S, J.rblk0 + lb);
    } else if constexpr (OP == OP_S) {
        // s <- r_{n+1} + alpha (s - chi A s)
        if (ok) {
            const cx<T> alpha = cvt<T>(S->alpha), chi = cvt<T>(S->chi);
            cx<T> r[12], s[12], as[12];
            load_spinor<SFL, T, true>(Rnxt, i, r);
            load_spinor<SFL, T, true>(J.f[R_F0], i, s);
            load_spinor<SFL, T, true>(J.f[R_F2], i, as);
#pragma unroll
            for (int k = 0; k < 12; k++) s[k] = r[k] + alpha * (s[k] - chi * as[k]);
            store_spinor<SFL, T, NTS>(J.f[R_F0], i, s);
        }

    } else if constexpr (OP == OP_SHIFT) {
        // BiCGstab-M: base s update, then every active shifted system
        //   x^s <- x^s - beta^s s^s + chi^s rho_n zeta_{n+1} w
        //   s^s <- zeta_{n+1} rho_{n+1} r_{n+1} + alpha^s (s^s - (chi^s/beta^s) rho_n (zeta_{n+1} w - zeta_n r_n))
        if (ok) {
            const cx<T> alpha = cvt<T>(S->alpha), chi = cvt<T>(S->chi);
            cx<T> rn[12], r1[12], w[12], s[12], as[12];
            load_spinor<SFL, T, true>(Rcur, i, rn);
            load_spinor<SFL, T, true>(Rnxt, i, r1);
            load_spinor<SFL, T, true>(J.f[R_F4], i, w);
            load_spinor<SFL, T, true>(J.f[R_F0], i, s);
            load_spinor<SFL, T, true>(J.f[R_F2], i, as);
#pragma unroll
            for (int k = 0; k < 12; k++) s[k] = r1[k] + alpha * (s[k] - chi * as[k]);
            store_spinor<SFL, T, NTS>(J.f[R_F0], i, s);
            const int ns = S->nshift;
            for (int q = 0; q < ns; q++) {
                const ShiftScal& Q = S->sh[q];
                if (!Q.active) continue;
                const SpinorRef xr = S->shv[2 * q], sr = S->shv[2 * q + 1];
                const cx<T> bs = cvt<T>(Q.beta_s);
                const cx<T> cxw = cvt<T>(c_mul(c_mul(Q.chi_s, Q.rho), Q.zeta_next));
                const cx<T> zr1 = cvt<T>(c_mul(Q.zeta_next, Q.rho_next));
                const cx<T> as_ = cvt<T>(Q.alpha_s);
                const cx<T> cb_ = cvt<T>(c_mul(c_div(Q.chi_s, Q.beta_s), Q.rho));
                const cx<T> zn1 = cvt<T>(Q.zeta_next), zn = cvt<T>(Q.zeta);
                cx<T> xs[12], ss[12];
                load_spinor<SFL, T, true>(xr, i, xs);
                load_spinor<SFL, T, true>(sr, i, ss);
#pragma unroll
                for (int k = 0; k < 12; k++) {
                    xs[k] = xs[k] - bs * ss[k] + cxw * w[k];
                    ss[k] = zr1 * r1[k] + as_ * (ss[k] - cb_ * (zn1 * w[k] - zn * rn[k]));
                }
                store_spinor<SFL, T, NTS>(xr, i, xs);
                store_spinor<SFL, T, NTS>(sr, i, ss);
            }
        }

    } else if constexpr (OP == OP_INIT) {
        // r_lo = r_hi; optionally rhat = r_lo, s = r_lo (flags 1, 2), x_lo = 0 (flags 4); CG (flags 8):
        // p = r_lo + beta p with the beta the host set in the record; then <rhat, r_lo>, |r_lo|^2
        if (ok) {
            cx<T> r[12];
            {
                cx<double> rh[12];
                load_spinor<SF64, double, true>(J.f[R_F1], i, rh);
#pragma unroll
                for (int k = 0; k < 12; k++) r[k] = mk<T>((T)rh[k].re, (T)rh[k].im);
            }
            store_spinor<SFL, T, NTS>(J.f[R_F0], i, r);
            // the dot products use the values as stored
            load_spinor<SFL, T, true>(J.f[R_F0], i, r);
            if (J.flags & 1) store_spinor<SFL, T, NTS>(J.f[R_F2], i, r);
            if (J.flags & 2) store_spinor<SFL, T, NTS>(J.f[R_F3], i, r);
            if (J.flags & 8) {
                const T bt = (T)S->cgb;
                cx<T> pp[12];
                load_spinor<SFL, T, true>(J.f[R_F3], i, pp);
#pragma unroll
                for (int k = 0; k < 12; k++) pp[k] = r[k] + bt * pp[k];
                store_spinor<SFL, T, NTS>(J.f[R_F3], i, pp);
            }
            if (J.flags & 4) {
                cx<T> zero[12];
#pragma unroll
                for (int k = 0; k < 12; k++) zero[k] = mk<T>(T(0), T(0));
                store_spinor<SFX, T, NTS>(J.f[R_F4], i, zero);
            }
            cx<T> rh[12];
            if (J.flags & 1) {
#pragma unroll
                for (int k = 0; k < 12; k++) rh[k] = r[k];
            } else {
                load_spinor<SFL, T, true>(J.f[R_F2], i, rh);
            }
#pragma unroll
            for (int k = 0; k < 12; k++) {
                v[0] += (double)rh[k].re * r[k].re + (double)rh[k].im * r[k].im;
                v[1] += (double)rh[k].re * r[k].im - (double)rh[k].im * r[k].re;
                v[2] += (double)r[k].re * r[k].re + (double)r[k].im * r[k].im;
            }
        }
        write_partials<3>(v, S, J.rblk0 + lb);
    } else if constexpr (OP == OP_ACC) {
        // x_hi += x_lo  (flags & 1: then x_lo = 0)
        if (ok) {
            cx<double> xh[12];
            cx<T> xl[12];
            load_spinor<SF64, double, true>(J.f[R_F0], i, xh);
            load_spinor<SFX, T, true>(J.f[R_F1], i, xl);
#pragma unroll
            for (int k = 0; k < 12; k++) xh[k] = xh[k] + mk<double>((double)xl[k].re, (double)xl[k].im);
            store_spinor<SF64, double, NTS>(J.f[R_F0], i, xh);
            if (J.flags & 1) {
#pragma unroll
                for (int k = 0; k < 12; k++) xl[k] = mk<T>(T(0), T(0));
                store_spinor<SFX, T, NTS>(J.f[R_F1], i, xl);
            }
        }
    } else if constexpr (OP == OP_NORM) {
        // |f0|^2 in FP64
        if (ok) {
            cx<double> a[12];
            load_spinor<SF64, double, true>(J.f[R_F0], i, a);
#pragma unroll
            for (int k = 0; k < 12; k++) v[2] += a[k].re * a[k].re + a[k].im * a[k].im;
        }
        write_partials<3>(v, S, J.rblk0 + lb);
    } else if constexpr (OP == OP_AXPY) {
        // f0 = c0 f1 + c1 f2 (FP64)
        if (ok) {
            cx<double> a[12], bq[12];
            load_spinor<SF64, double, true>(J.f[R_F1], i, a);
            load_spinor<SF64, double, true>(J.f[R_F2], i, bq);
#pragma unroll
            for (int k = 0; k < 12; k++) a[k] = J.c[0] * a[k] + J.c[1] * bq[k];
            store_spinor<SF64, double, NTS>(J.f[R_F0], i, a);
        }
    } else if constexpr (OP == OP_LINCOMB) {
        // f0 (+)= sum_{j < m} c_j f_{1+j}, m = flags >> 8; flags & 1: accumulate into f0;
        // flags & 2: complex c_j = (c[2j], c[2j+1]) (m <= 4), else real c_j = c[j] (m <= 7)
        if (ok) {
            cx<double> acc[12], a[12];
            if (J.flags & 1) load_spinor<SF64, double, true>(J.f[R_F0], i, acc);
            else {
#pragma unroll
                for (int k = 0; k < 12; k++) acc[k] = mk<double>(0.0, 0.0);
            }
            const int m = J.flags >> 8;
            const bool cplx = (J.flags & 2) != 0;
            for (int j = 0; j < m; j++) {
                load_spinor<SF64, double, true>(J.f[1 + j], i, a);
                const cx<double> cj = cplx ? mk<double>(J.c[2 * j], J.c[2 * j + 1]) : mk<double>(J.c[j], 0.0);
#pragma unroll
                for (int k = 0; k < 12; k++) acc[k] = acc[k] + cj * a[k];
            }
            store_spinor<SF64, double, NTS>(J.f[R_F0], i, acc);
        }
    } else if constexpr (OP == OP_CGX) {
        // CG: x += alpha p ; r -= alpha A p ; |r|^2
        if (ok) {
            const T alpha = (T)S->cga;
            cx<T> x[12], p[12], r[12], ap[12];
            load_spinor<SFX, T, true>(J.f[R_F0], i, x);
            load_spinor<SFL, T, true>(J.f[R_F1], i, p);
#pragma unroll
            for (int k = 0; k < 12; k++) x[k] = x[k] + alpha * p[k];
            store_spinor<SFX, T, NTS>(J.f[R_F0], i, x);
            load_spinor<SFL, T, true>(J.f[R_F2], i, r);
            load_spinor<SFL, T, true>(J.f[R_F3], i, ap);
#pragma unroll
            for (int k = 0; k < 12; k++) r[k] = r[k] - alpha * ap[k];
            store_spinor<SFL, T, NTS>(J.f[R_F2], i, r);
            // the norm of the residual as stored
            load_spinor<SFL, T, true>(J.f[R_F2], i, r);
#pragma unroll
            for (int k = 0; k < 12; k++) v[2] += (double)r[k].re * r[k].re + (double)r[k].im * r[k].im;
        }
        write_partials<3>(v, S, J.rblk0 + lb);
    } else if constexpr (OP == OP_CGP || OP == OP_CGPM) {
        // CG: p = r + beta p ; CG-M, every active shifted system:
        //   x^s += alpha^s_n p^s ;  p^s = zeta_{n+1} r + beta^s_{n+1} p^s
        if (ok) {
            const T beta = (T)S->cgb;
            cx<T> r[12], p[12];
            load_spinor<SFL, T, true>(J.f[R_F1], i, r);
            load_spinor<SFL, T, true>(J.f[R_F0], i, p);
#pragma unroll
            for (int k = 0; k < 12; k++) p[k] = r[k] + beta * p[k];
            store_spinor<SFL, T, NTS>(J.f[R_F0], i, p);
            if constexpr (OP == OP_CGPM) {
                const int ns = S->nshift;
                for (int q = 0; q < ns; q++) {
                    const ShiftScal& Q = S->sh[q];
                    if (!Q.active) continue;
                    const SpinorRef xr = S->shv[2 * q], pr = S->shv[2 * q + 1];
                    const T as = (T)Q.alpha_s.x, bs = (T)Q.beta_s.x, zn = (T)Q.zeta_next.x;
                    cx<T> xs[12], ps[12];
                    load_spinor<SFL, T, true>(xr, i, xs);
                    load_spinor<SFL, T, true>(pr, i, ps);
#pragma unroll
                    for (int k = 0; k < 12; k++) {
                        xs[k] = xs[k] + as * ps[k];
                        ps[k] = zn * r[k] + bs * ps[k];
                    }
                    store_spinor<SFL, T, NTS>(xr, i, xs);
                    store_spinor<SFL, T, NTS>(pr, i, ps);
                }
            }
        }
    } else if constexpr (OP == OP_MSINIT) {
        // BiCGstab-M start: r = s = rhat = b, x = 0, x^sigma = 0, s^sigma = b; |b|^2
        if (ok) {
            cx<T> bb[12], zero[12];
            load_spinor<SFL, T, true>(J.f[R_F1], i, bb);
#pragma unroll
            for (int k = 0; k < 12; k++) zero[k] = mk<T>(T(0), T(0));
            store_spinor<SFL, T, NTS>(J.f[R_F0], i, bb);
            store_spinor<SFL, T, NTS>(J.f[R_F2], i, bb);
            store_spinor<SFL, T, NTS>(J.f[R_F3], i, bb);
            store_spinor<SFL, T, NTS>(J.f[R_F4], i, zero);
            for (int q = 0; q < S->nshift; q++) {
                store_spinor<SFL, T, NTS>(S->shv[2 * q], i, zero);
                store_spinor<SFL, T, NTS>(S->shv[2 * q + 1], i, bb);
            }
#pragma unroll
            for (int k = 0; k < 12; k++) {
                double n2 = (double)bb[k].re * bb[k].re + (double)bb[k].im * bb[k].im;
                v[0] += n2;
                v[2] += n2;
            }
        }
        write_partials<3>(v, S, J.rblk0 + lb);
    }
}

// ================================================================ start vector and its residual

// Sequential multi-mass start (Sec. 6.2.1) without applying the operator: for the even-odd system
// of mass a = 1/(2 kappa), with the earlier solutions x_j and their FP64 residuals
// r_j = b_prec(a_j) - M_prec(a_j) x_j (b_prec(a) = a b_e + h, M_prec(a) = a^2 - K, K independent
// of the mass),
//   x0 = sum_j c_j x_j,
//   r0 = b_prec(a) - M_prec(a) x0 = cb b_e + ch h + sum_j cx_j x_j + sum_j c_j r_j
// (and b_prec(a) itself when bp.p is set). The shifted normal equations (A + s) x = b_e use the same
// kernel without h: there r0 = (1 - sum c_j) b_e + sum_j c_j (s_j - s) x_j + sum_j c_j r_j.
// with cb = a - sum c_j a_j, ch = 1 - sum c_j, cx_j = c_j (a_j^2 - a^2), since K x_j =
// r_j - a_j b_e - h + a_j^2 x_j. FP64 half fields over n sites; acc = 1 adds to x0 and r0 (inputs
// in chunks of GUESS_MAX). Every input is read once: non-temporal loads.
__global__ __launch_bounds__(BLOCK) void k_guess(GuessArgs A)
{
    const long i = (long)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= A.n) return;
    cx<double> x0[12], r0[12], v[12];
    if (A.acc) {
        load_spinor<SF64, double, true>(A.x0, i, x0);
        load_spinor<SF64, double, true>(A.r0, i, r0);
    } else {
#pragma unroll
        for (int k = 0; k < 12; k++) x0[k] = r0[k] = mk<double>(0.0, 0.0);
    }
    if (A.be.p) {
        cx<double> hv[12];
        load_spinor<SF64, double, true>(A.be, i, v);
        if (A.h.p) load_spinor<SF64, double, true>(A.h, i, hv);
        else {
#pragma unroll
            for (int k = 0; k < 12; k++) hv[k] = mk<double>(0.0, 0.0);
        }
#pragma unroll
        for (int k = 0; k < 12; k++) r0[k] = r0[k] + A.cb * v[k] + A.ch * hv[k];
        if (A.bp.p) {
#pragma unroll
            for (int k = 0; k < 12; k++) v[k] = A.a * v[k] + hv[k];
            store_spinor<SF64, double>(A.bp, i, v);
        }
    }
    for (int j = 0; j < A.k; j++) {
        load_spinor<SF64, double, true>(A.xs[j], i, v);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            x0[k] = x0[k] + A.c[j] * v[k];
            r0[k] = r0[k] + A.cx[j] * v[k];
        }
        load_spinor<SF64, double, true>(A.rs[j], i, v);
#pragma unroll
        for (int k = 0; k < 12; k++) r0[k] = r0[k] + A.c[j] * v[k];
    }
    store_spinor<SF64, double>(A.x0, i, x0);
    store_spinor<SF64, double>(A.r0, i, r0);
}

// ================================================================ inner products of full fields

// <a, b_j> for j < m (m <= DOTS_MAX) over the real sites of two full FP64 fields in the internal
// layout (padding sites of each half skipped). Block partials [block][2 m], then one block sums
// them in a fixed order: deterministic.
__global__ __launch_bounds__(BLOCK) void k_dots(SpinorRef a, const SpinorRef* __restrict__ bs, int m, int Vh,
                                                int stride, double* __restrict__ partials)
{
    __shared__ double lds[BLOCK / 64];
    const long i = (long)blockIdx.x * BLOCK + threadIdx.x;  // site of the full field, [0, 2 stride)
    const bool ok = i < 2L * stride && (i % stride) < Vh;
    cx<double> va[12];
    if (ok) load_spinor<SF64, double>(a, i, va);
    for (int j = 0; j < m; j++) {
        double re = 0.0, im = 0.0;
        if (ok) {
            cx<double> vb[12];
            load_spinor<SF64, double>(bs[j], i, vb);
#pragma unroll
            for (int k = 0; k < 12; k++) {
                re += va[k].re * vb[k].re + va[k].im * vb[k].im;
                im += va[k].re * vb[k].im - va[k].im * vb[k].re;
            }
        }
        double v[2] = {re, im};
#pragma unroll
        for (int c = 0; c < 2; c++) {
            double s = wave_sum(v[c]);
            if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
            __syncthreads();
            if (threadIdx.x == 0) {
                double t = 0.0;
                for (int w = 0; w < BLOCK / 64; w++) t += lds[w];
                partials[(long)blockIdx.x * 2 * DOTS_MAX + 2 * j + c] = t;
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_dots_finish(const double* __restrict__ partials, int nblk, int m,
                                                       double* __restrict__ out)
{
    __shared__ double lds[BLOCK / 64];
    for (int c = 0; c < 2 * m; c++) {
        double t = 0.0;
        for (int b = threadIdx.x; b < nblk; b += BLOCK) t += partials[(long)b * 2 * DOTS_MAX + c];
        t = wave_sum(t);
        if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            double u = 0.0;
            for (int w = 0; w < BLOCK / 64; w++) u += lds[w];
            out[c] = u;
        }
        __syncthreads();
    }
}

// ================================================================ packing

// Spin basis of the solvers' internal fields on a non-chiral handle: psi' = psi S with
// S = (1/sqrt 2) [[1, 0, 1, 0], [0, 1, 0, 1], [-1, 0, 1, 0], [0, -1, 0, 1]] (spin index, fields
// multiplied from the right as in eq. 4), for which S^dag gamma_4 S = diag(1, 1, -1, -1) while the
// spatial gamma matrices of Sec. 2 are unchanged. Site values v[c * 4 + s].
__device__ __forceinline__ void spin_to_nc(cx<double> v[12])
{
    const double r = 0.70710678118654752440;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const cx<double> a0 = v[c * 4], a1 = v[c * 4 + 1], a2 = v[c * 4 + 2], a3 = v[c * 4 + 3];
        v[c * 4] = r * (a0 - a2);
        v[c * 4 + 1] = r * (a1 - a3);
        v[c * 4 + 2] = r * (a0 + a2);
        v[c * 4 + 3] = r * (a1 + a3);
    }
}
// psi = psi' S^dag
__device__ __forceinline__ void spin_from_nc(cx<double> v[12])
{
    const double r = 0.70710678118654752440;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const cx<double> a0 = v[c * 4], a1 = v[c * 4 + 1], a2 = v[c * 4 + 2], a3 = v[c * 4 + 3];
        v[c * 4] = r * (a0 + a2);
        v[c * 4 + 1] = r * (a1 + a3);
        v[c * 4 + 2] = r * (a2 - a0);
        v[c * 4 + 3] = r * (a3 - a1);
    }
}

// canonical [V][3][4] complex128 (lexicographic) <-> internal per-parity half fields.
// gamma5 != 0 multiplies spin components 2 and 3 by -1 on the way (gamma5 = diag(1,1,-1,-1)).
template <int SF>
// gm (may be NULL): colour rotation g(n) applied on the way, psi'(n) = g(n) psi(n) (temporal gauge)
// nc: then into the non-chiral basis (spin_to_nc)
__global__ __launch_bounds__(BLOCK) void k_pack_spinor(const double2* __restrict__ src, Geo g, SpinorRef even,
                                                       SpinorRef odd, int gamma5, double scale,
                                                       const double2* __restrict__ gm, int nc)
{
    const int p = blockIdx.y;
    const int cb = blockIdx.x * BLOCK + threadIdx.x;
    if (cb >= g.Vh) return;
    int x, y, z, t;
    cb_coords(g, p, cb, x, y, z, t);
    const long n = x + (long)g.X * (y + (long)g.Y * (z + (long)g.Z * t));
    cx<double> v[12];
#pragma unroll
    for (int k = 0; k < 12; k++) {
        double2 q = src[n * 12 + k];
        double sg = (gamma5 && (k & 3) >= 2) ? -scale : scale;
        v[k] = mk<double>(sg * q.x, sg * q.y);
    }
    if (gm) {
        cx<double> G[9], w[12];
#pragma unroll
        for (int k = 0; k < 9; k++) G[k] = mk<double>(gm[n * 9 + k].x, gm[n * 9 + k].y);
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int sp = 0; sp < 4; sp++)
                w[a * 4 + sp] = G[a * 3] * v[sp] + G[a * 3 + 1] * v[4 + sp] + G[a * 3 + 2] * v[8 + sp];
#pragma unroll
        for (int k = 0; k < 12; k++) v[k] = w[k];
    }
    if (nc) spin_to_nc(v);
    store_spinor<SF, double>(p ? odd : even, cb, v);
}

template <int SF>
// gm (may be NULL): psi(n) = g(n)^dag psi'(n) (back from temporal gauge)
// nc: out of the non-chiral basis first (spin_from_nc)
__global__ __launch_bounds__(BLOCK) void k_unpack_spinor(double2* __restrict__ dst, Geo g, SpinorRef even,
                                                         SpinorRef odd, int gamma5, double scale,
                                                         const double2* __restrict__ gm, int nc)
{
    const int p = blockIdx.y;
    const int cb = blockIdx.x * BLOCK + threadIdx.x;
    if (cb >= g.Vh) return;
    int x, y, z, t;
    cb_coords(g, p, cb, x, y, z, t);
    const long n = x + (long)g.X * (y + (long)g.Y * (z + (long)g.Z * t));
    using T = typename SReal<SF>::T;
    cx<T> v[12];
    load_spinor<SF, T>(p ? odd : even, cb, v);
    cx<double> w[12];
#pragma unroll
    for (int k = 0; k < 12; k++) w[k] = mk<double>((double)v[k].re, (double)v[k].im);
    if (nc) spin_from_nc(w);
    if (gm) {
        cx<double> G[9], u[12];
#pragma unroll
        for (int k = 0; k < 9; k++) G[k] = mk<double>(gm[n * 9 + k].x, gm[n * 9 + k].y);
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int sp = 0; sp < 4; sp++)
                u[a * 4 + sp] = cmulc(G[a], w[sp]) + cmulc(G[3 + a], w[4 + sp]) + cmulc(G[6 + a], w[8 + sp]);
#pragma unroll
        for (int k = 0; k < 12; k++) w[k] = u[k];
    }
#pragma unroll
    for (int k = 0; k < 12; k++) {
        double sg = (gamma5 && (k & 3) >= 2) ? -scale : scale;
        dst[n * 12 + k] = make_double2(sg * w[k].re, sg * w[k].im);
    }
}

// Canonical output of an even-odd solve in one pass, one thread per lattice site in canonical
// order (a wavefront writes contiguous sites): even sites from x_e, odd sites rebuilt from eq. eo3,
// x_o = c0 b_o + c1 T with T = D_oe x_e left by the last FP64 residual update (stored into xo too
// when xo.p is set), then the colour rotation, gamma5 and scale of k_unpack_spinor. FP64 fields.
__global__ __launch_bounds__(BLOCK) void k_unpack_eo(double2* __restrict__ dst, Geo g, SpinorRef xe, SpinorRef xo,
                                                     SpinorRef bo, SpinorRef T, double c0, double c1, int gamma5,
                                                     double scale, const double2* __restrict__ gm, int nc)
{
    const long n = (long)blockIdx.x * BLOCK + threadIdx.x;
    const long V = (long)g.X * g.Y * g.Z * g.T;
    if (n >= V) return;
    const int x = (int)(n % g.X);
    long r = n / g.X;
    const int y = (int)(r % g.Y);
    r /= g.Y;
    const int z = (int)(r % g.Z);
    const int t = (int)(r / g.Z);
    const int cb = cb_index(g, x, y, z, t);
    cx<double> w[12];
    if (((x + y + z + t) & 1) == 0) {
        load_spinor<SF64, double, true>(xe, cb, w);
    } else {
        cx<double> q[12];
        load_spinor<SF64, double, true>(bo, cb, w);
        load_spinor<SF64, double, true>(T, cb, q);
#pragma unroll
        for (int k = 0; k < 12; k++) w[k] = c0 * w[k] + c1 * q[k];
        if (xo.p) store_spinor<SF64, double>(xo, cb, w);
    }
    if (nc) spin_from_nc(w);
    if (gm) {
        cx<double> G[9], u[12];
#pragma unroll
        for (int k = 0; k < 9; k++) G[k] = mk<double>(gm[n * 9 + k].x, gm[n * 9 + k].y);
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int sp = 0; sp < 4; sp++)
                u[a * 4 + sp] = cmulc(G[a], w[sp]) + cmulc(G[3 + a], w[4 + sp]) + cmulc(G[6 + a], w[8 + sp]);
#pragma unroll
        for (int k = 0; k < 12; k++) w[k] = u[k];
    }
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const double sg = (gamma5 && (k & 3) >= 2) ? -scale : scale;
        dst[n * 12 + k] = make_double2(sg * w[k].re, sg * w[k].im);
    }
}

// canonical U[4][V][3][3] -> internal FP64 18-real links, 8 slots per output site
__global__ __launch_bounds__(BLOCK) void k_pack_links(const double2* __restrict__ U, Geo g, void* even, void* odd,
                                                      long lcs)
{
    const int p = blockIdx.y;
    const int cb = blockIdx.x * BLOCK + threadIdx.x;
    if (cb >= g.Vh) return;
    int x, y, z, t;
    cb_coords(g, p, cb, x, y, z, t);
    const long V = (long)g.X * g.Y * g.Z * g.T;
    const long n = x + (long)g.X * (y + (long)g.Y * (z + (long)g.Z * t));
    void* dst = p ? odd : even;
    for (int mu = 0; mu < 4; mu++) {
        cx<double> W[9];
        const double2* u = U + ((long)mu * V + n) * 9;
#pragma unroll
        for (int k = 0; k < 9; k++) W[k] = mk<double>(u[k].x, u[k].y);
        store_link<L64_18>(dst, lcs, mu, cb, W);
        int c[4] = {x, y, z, t};
        const int L[4] = {g.X, g.Y, g.Z, g.T};
        c[mu] = c[mu] == 0 ? L[mu] - 1 : c[mu] - 1;
        const long m = c[0] + (long)g.X * (c[1] + (long)g.Y * (c[2] + (long)g.Z * c[3]));
        const double2* ub = U + ((long)mu * V + m) * 9;
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int bb = 0; bb < 3; bb++) W[a * 3 + bb] = mk<double>(ub[bb * 3 + a].x, -ub[bb * 3 + a].y);
        store_link<L64_18>(dst, lcs, 4 + mu, cb, W);
    }
}

// internal FP64 18-real links -> another link format (same slot layout)
template <int SRC, int LF>
__global__ __launch_bounds__(BLOCK) void k_convert_links(const void* __restrict__ src, void* __restrict__ dst, int Vh,
                                                         long lcs)
{
    const int cb = blockIdx.x * BLOCK + threadIdx.x;
    const int k = blockIdx.y;
    if (cb >= Vh) return;
    cx<double> W[9];
    load_link<SRC, double>(src, lcs, k, cb, W);
    store_link<LF>(dst, lcs, k, cb, W);
}

// ---------------------------------------------------------------- temporal gauge
// Bandwidth saving named in Sec. 4: with g(x, 0) = 1 and g(x, t + 1) = g(x, t) U_t(x, t), the
// gauge transform U'_mu(n) = g(n) U_mu(n) g(n + mu)^dag, psi'(n) = g(n) psi(n) (M' = g M g^dag)
// turns every time link into the unit matrix except U'_t(x, T - 1) = g(x, T - 1) U_t(x, T - 1),
// so the hop loads and multiplies time links on the two boundary time slices only.
// One thread per spatial site walks t; gm: canonical [V][3][3].
__global__ __launch_bounds__(BLOCK) void k_temporal_g(const double2* __restrict__ U, Geo g, double2* __restrict__ gm)
{
    const long Vs = (long)g.X * g.Y * g.Z;
    const long s = (long)blockIdx.x * BLOCK + threadIdx.x;
    if (s >= Vs) return;
    const long V = Vs * g.T;
    cx<double> G[9];
#pragma unroll
    for (int k = 0; k < 9; k++) G[k] = mk<double>(k % 4 == 0 ? 1.0 : 0.0, 0.0);
    for (int t = 0; t < g.T; t++) {
        const long n = s + Vs * t;
#pragma unroll
        for (int k = 0; k < 9; k++) gm[n * 9 + k] = make_double2(G[k].re, G[k].im);
        const double2* u = U + (3 * V + n) * 9;
        cx<double> W[9], R[9];
#pragma unroll
        for (int k = 0; k < 9; k++) W[k] = mk<double>(u[k].x, u[k].y);
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) R[a * 3 + b] = G[a * 3] * W[b] + G[a * 3 + 1] * W[3 + b] + G[a * 3 + 2] * W[6 + b];
#pragma unroll
        for (int k = 0; k < 9; k++) G[k] = R[k];
    }
}

// U'_mu(n) = g(n) U_mu(n) g(n + mu)^dag, canonical [4][V][3][3]; time links inside the lattice are
// written as the exact unit matrix.
__global__ __launch_bounds__(BLOCK) void k_transform_links(const double2* __restrict__ U, const double2* __restrict__ gm,
                                                           Geo g, double2* __restrict__ Uf)
{
    const long V = (long)g.X * g.Y * g.Z * g.T;
    const long n = (long)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= V) return;
    int c[4];
    long r = n;
    c[0] = (int)(r % g.X); r /= g.X;
    c[1] = (int)(r % g.Y); r /= g.Y;
    c[2] = (int)(r % g.Z);
    c[3] = (int)(r / g.Z);
    const int L[4] = {g.X, g.Y, g.Z, g.T};
    cx<double> Gn[9];
#pragma unroll
    for (int k = 0; k < 9; k++) Gn[k] = mk<double>(gm[n * 9 + k].x, gm[n * 9 + k].y);
    for (int mu = 0; mu < 4; mu++) {
        double2* out = Uf + ((long)mu * V + n) * 9;
        if (mu == 3 && c[3] != g.T - 1) {
#pragma unroll
            for (int k = 0; k < 9; k++) out[k] = make_double2(k % 4 == 0 ? 1.0 : 0.0, 0.0);
            continue;
        }
        int d[4] = {c[0], c[1], c[2], c[3]};
        d[mu] = d[mu] + 1 == L[mu] ? 0 : d[mu] + 1;
        const long m = d[0] + (long)g.X * (d[1] + (long)g.Y * (d[2] + (long)g.Z * d[3]));
        const double2* u = U + ((long)mu * V + n) * 9;
        cx<double> A[9], B[9];
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++)
                A[a * 3 + b] = Gn[a * 3] * mk<double>(u[b].x, u[b].y) + Gn[a * 3 + 1] * mk<double>(u[3 + b].x, u[3 + b].y) +
                               Gn[a * 3 + 2] * mk<double>(u[6 + b].x, u[6 + b].y);
        // B = A g(m)^dag: B[a][b] = sum_k A[a][k] conj(g(m)[b][k])
        const double2* gmm = gm + m * 9;
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) {
                cx<double> t = mk<double>(0.0, 0.0);
#pragma unroll
                for (int k = 0; k < 3; k++) t = t + A[a * 3 + k] * cconj(mk<double>(gmm[b * 3 + k].x, gmm[b * 3 + k].y));
                B[a * 3 + b] = t;
            }
#pragma unroll
        for (int k = 0; k < 9; k++) out[k] = make_double2(B[k].re, B[k].im);
    }
}

// Per-block maximum over all stored links of
//   mode 0: the deviation of row 2 from conj(row0 x row1), which decides whether the 12-real
//           FP64 format reproduces the operator exactly;
//   mode 1: |u00|^2, which must stay below 1 for the 8-real format (row 1 is rebuilt by dividing
//           by |u01|^2 + |u02|^2 = 1 - |u00|^2).
__global__ __launch_bounds__(BLOCK) void k_recon_check(const void* __restrict__ lk, int Vh, long lcs,
                                                       double* __restrict__ blockmax, int mode)
{
    __shared__ double lds[BLOCK / 64];
    const int cb = blockIdx.x * BLOCK + threadIdx.x;
    double m = 0.0;
    if (cb < Vh) {
        for (int k = 0; k < 8; k++) {
            cx<double> W[9];
            load_link<L64_18, double>(lk, lcs, k, cb, W);
            if (mode == 1) {
                m = fmax(m, W[0].re * W[0].re + W[0].im * W[0].im);
                continue;
            }
            cx<double> R[9];
            for (int j = 0; j < 6; j++) R[j] = W[j];
            recon_row2(R);
            for (int j = 6; j < 9; j++) m = fmax(m, fmax(fabs(R[j].re - W[j].re), fabs(R[j].im - W[j].im)));
        }
    }
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < BLOCK / 64; w++) m = fmax(m, lds[w]);
        blockmax[blockIdx.x] = m;
    }
}

hipError_t launch_recon_check(const void* lk, int Vh, long lcs, double* blockmax, hipStream_t s, int mode)
{
    hipLaunchKernelGGL(k_recon_check, dim3((unsigned)((Vh + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, lk, Vh, lcs,
                       blockmax, mode);
    return hipGetLastError();
}

// out = sum_j c_j in_j over n complex numbers (FP64, any layout)
__global__ __launch_bounds__(BLOCK) void k_lincomb(double2* __restrict__ out, const double2* const* __restrict__ ins,
                                                   const double* __restrict__ c, int k, long n)
{
    const long i = (long)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    double2 s = make_double2(0.0, 0.0);
    for (int j = 0; j < k; j++) {
        double2 a = ins[j][i];
        s.x += c[j] * a.x;
        s.y += c[j] * a.y;
    }
    out[i] = s;
}

// ================================================================ link gradient

// G_mu(n) = 1/2 s [ lam_n (1 - gamma_mu) x_{n+mu}^dag + x_n (1 + gamma_mu) lam_{n+mu}^dag ]
// With 1 -/+ gamma = v1 v1^dag + v2 v2^dag (Table 1) each term is a sum of two colour outer
// products of projected vectors: psi P phi^dag = (psi v1)(phi v1)^dag + (psi v2)(phi v2)^dag.
template <int MU, bool MINUS>
__device__ __forceinline__ void proj2(const cx<double> psi[12], cx<double> h1[3], cx<double> h2[3])
{
    constexpr int E = Proj<MU>::E + (MINUS ? 0 : 2);
    constexpr int F = Proj<MU>::F + (MINUS ? 0 : 2);
#pragma unroll
    for (int c = 0; c < 3; c++) {
        h1[c] = psi[c * 4 + 3] + mul_ik<-E>(psi[c * 4 + Proj<MU>::I1]);
        h2[c] = psi[c * 4 + 2] + mul_ik<-F>(psi[c * 4 + Proj<MU>::I2]);
    }
}

template <int MU>
__device__ __forceinline__ void grad_mu(const Geo& g, long n, int x, int y, int z, int t, const double2* xs,
                                        const double2* lam, const cx<double> xn[12], const cx<double> ln[12],
                                        cx<double> G[9])
{
    int c[4] = {x, y, z, t};
    const int L[4] = {g.X, g.Y, g.Z, g.T};
    c[MU] = c[MU] + 1 == L[MU] ? 0 : c[MU] + 1;
    const long m = c[0] + (long)g.X * (c[1] + (long)g.Y * (c[2] + (long)g.Z * c[3]));
    cx<double> xm[12], lm[12];
#pragma unroll
    for (int k = 0; k < 12; k++) {
        xm[k] = mk<double>(xs[m * 12 + k].x, xs[m * 12 + k].y);
        lm[k] = mk<double>(lam[m * 12 + k].x, lam[m * 12 + k].y);
    }
    cx<double> a1[3], a2[3], b1[3], b2[3], c1[3], c2[3], d1[3], d2[3];
    proj2<MU, true>(ln, a1, a2);   // lam_n  with 1 - gamma
    proj2<MU, true>(xm, b1, b2);   // x_{n+mu} with 1 - gamma
    proj2<MU, false>(xn, c1, c2);  // x_n   with 1 + gamma
    proj2<MU, false>(lm, d1, d2);  // lam_{n+mu} with 1 + gamma
    const double s = (MU == 3 && g.anti && t == g.T - 1) ? -0.5 : 0.5;  // 1/2 times the boundary sign
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int bb = 0; bb < 3; bb++) {
            cx<double> v = cmulc(b1[bb], a1[a]) + cmulc(b2[bb], a2[a]) + cmulc(d1[bb], c1[a]) + cmulc(d2[bb], c2[a]);
            G[a * 3 + bb] = s * v;
        }
}

__global__ __launch_bounds__(BLOCK) void k_grad(const double2* __restrict__ xs, const double2* __restrict__ lam, Geo g,
                                                const void* __restrict__ lk_even, const void* __restrict__ lk_odd,
                                                long lcs, double2* __restrict__ out, int project)
{
    const long V = (long)g.X * g.Y * g.Z * g.T;
    const long n = (long)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= V) return;
    int x = (int)(n % g.X);
    long r = n / g.X;
    int y = (int)(r % g.Y);
    r /= g.Y;
    int z = (int)(r % g.Z);
    int t = (int)(r / g.Z);
    cx<double> xn[12], ln[12];
#pragma unroll
    for (int k = 0; k < 12; k++) {
        xn[k] = mk<double>(xs[n * 12 + k].x, xs[n * 12 + k].y);
        ln[k] = mk<double>(lam[n * 12 + k].x, lam[n * 12 + k].y);
    }
    const int p = (x + y + z + t) & 1;
    const int cb = cb_index(g, x, y, z, t);
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
        cx<double> G[9];
        if (mu == 0) grad_mu<0>(g, n, x, y, z, t, xs, lam, xn, ln, G);
        if (mu == 1) grad_mu<1>(g, n, x, y, z, t, xs, lam, xn, ln, G);
        if (mu == 2) grad_mu<2>(g, n, x, y, z, t, xs, lam, xn, ln, G);
        if (mu == 3) grad_mu<3>(g, n, x, y, z, t, xs, lam, xn, ln, G);
        if (project) {
            // F = (i/2) TA(U G^dag),  TA(Y) = (Y - Y^dag)/2 - tr(Y - Y^dag)/6
            cx<double> U[9], Y[9];
            load_link<L64_18, double>(p ? lk_odd : lk_even, lcs, mu, cb, U);
#pragma unroll
            for (int a = 0; a < 3; a++)
#pragma unroll
                for (int bb = 0; bb < 3; bb++)
                    Y[a * 3 + bb] = cmulc(G[bb * 3], U[a * 3]) + cmulc(G[bb * 3 + 1], U[a * 3 + 1]) +
                                    cmulc(G[bb * 3 + 2], U[a * 3 + 2]);
            cx<double> A[9];
#pragma unroll
            for (int a = 0; a < 3; a++)
#pragma unroll
                for (int bb = 0; bb < 3; bb++) A[a * 3 + bb] = 0.5 * (Y[a * 3 + bb] - cconj(Y[bb * 3 + a]));
            cx<double> tr = (1.0 / 3.0) * (A[0] + A[4] + A[8]);
            A[0] = A[0] - tr;
            A[4] = A[4] - tr;
            A[8] = A[8] - tr;
#pragma unroll
            for (int k = 0; k < 9; k++) G[k] = mk<double>(-0.5 * A[k].im, 0.5 * A[k].re);
        }
#pragma unroll
        for (int k = 0; k < 9; k++) out[((long)mu * V + n) * 9 + k] = make_double2(G[k].re, G[k].im);
    }
}

// ================================================================ host launchers

#define FIN_CASE(NR_, FIN_)                                                                                        \
    if (nr == NR_ && fin == FIN_) {                                                                                \
        hipExtLaunchKernelGGL((k_finish<NR_, FIN_>), dim3(nfin), dim3(BLOCK), 0, s, ev0, ev1, 0, fins, sys, gated); \
        return hipGetLastError();                                                                                  \
    }

hipError_t launch_finish(int nr, int fin, const FinJob* fins, int nfin, SysState* sys, int gated, hipStream_t s,
                         hipEvent_t ev0, hipEvent_t ev1)
{
    if (nfin <= 0) return hipSuccess;
    FIN_CASE(3, FIN_STORE)
    FIN_CASE(3, FIN_BETA)
    FIN_CASE(3, FIN_CHI)
    FIN_CASE(3, FIN_ALPHA)
    FIN_CASE(3, FIN_RESTART)
    FIN_CASE(0, FIN_END)
    FIN_CASE(3, FIN_CGA)
    FIN_CASE(3, FIN_CGB)
    FIN_CASE(0, FIN_CGEND)
    return hipErrorInvalidValue;
}

#define SWEEP_CASE(OP_, SF_)                                                                                       \
    if (op == OP_ && sfl == SF_) {                                                                                 \
        hipExtLaunchKernelGGL((k_sweep<OP_, SF_>), grid1(nblocks), dim3(BLOCK), 0, s, ev0, ev1, 0, jobs, njobs, sys, \
                              gated, exec);                                                                        \
        return hipGetLastError();                                                                                  \
    }
#define SWEEP_ALL(SF_)                                                                                             \
    SWEEP_CASE(OP_W, SF_)                                                                                          \
    SWEEP_CASE(OP_XR, SF_) SWEEP_CASE(OP_S, SF_) SWEEP_CASE(OP_INIT, SF_) SWEEP_CASE(OP_ACC, SF_)                 \
    SWEEP_CASE(OP_CGX, SF_) SWEEP_CASE(OP_CGP, SF_)

hipError_t launch_sweep(int op, int sfl, const SweepJob* jobs, int njobs, long nblocks, SysState* sys, int gated,
                        hipStream_t s, int* exec, hipEvent_t ev0, hipEvent_t ev1)
{
    if (nblocks <= 0) return hipSuccess;
    SWEEP_ALL(SF64)
    SWEEP_ALL(SF32)
    SWEEP_ALL(SF16)
    SWEEP_CASE(OP_SHIFT, SF64)
    SWEEP_CASE(OP_NORM, SF64)
    SWEEP_CASE(OP_MSINIT, SF64)
    SWEEP_CASE(OP_AXPY, SF64)
    SWEEP_CASE(OP_LINCOMB, SF64)
    SWEEP_CASE(OP_CGPM, SF64)
    return hipErrorInvalidValue;
}

hipError_t launch_pack_spinor(int sf, const double* src, const Geo& g, SpinorRef even, SpinorRef odd, int gamma5,
                              double scale, hipStream_t s, const double* gm, int nc)
{
    dim3 grid((unsigned)((g.Vh + BLOCK - 1) / BLOCK), 2);
    const double2* G = (const double2*)gm;
    if (sf == SF64) hipLaunchKernelGGL((k_pack_spinor<SF64>), grid, dim3(BLOCK), 0, s, (const double2*)src, g, even, odd, gamma5, scale, G, nc);
    else if (sf == SF32) hipLaunchKernelGGL((k_pack_spinor<SF32>), grid, dim3(BLOCK), 0, s, (const double2*)src, g, even, odd, gamma5, scale, G, nc);
    else hipLaunchKernelGGL((k_pack_spinor<SF16>), grid, dim3(BLOCK), 0, s, (const double2*)src, g, even, odd, gamma5, scale, G, nc);
    return hipGetLastError();
}

hipError_t launch_unpack_spinor(int sf, double* dst, const Geo& g, SpinorRef even, SpinorRef odd, int gamma5,
                                double scale, hipStream_t s, const double* gm, int nc)
{
    dim3 grid((unsigned)((g.Vh + BLOCK - 1) / BLOCK), 2);
    const double2* G = (const double2*)gm;
    if (sf == SF64) hipLaunchKernelGGL((k_unpack_spinor<SF64>), grid, dim3(BLOCK), 0, s, (double2*)dst, g, even, odd, gamma5, scale, G, nc);
    else if (sf == SF32) hipLaunchKernelGGL((k_unpack_spinor<SF32>), grid, dim3(BLOCK), 0, s, (double2*)dst, g, even, odd, gamma5, scale, G, nc);
    else hipLaunchKernelGGL((k_unpack_spinor<SF16>), grid, dim3(BLOCK), 0, s, (double2*)dst, g, even, odd, gamma5, scale, G, nc);
    return hipGetLastError();
}

hipError_t launch_pack_links(const double* U, const Geo& g, void* even, void* odd, long lcs, hipStream_t s)
{
    dim3 grid((unsigned)((g.Vh + BLOCK - 1) / BLOCK), 2);
    hipLaunchKernelGGL(k_pack_links, grid, dim3(BLOCK), 0, s, (const double2*)U, g, even, odd, lcs);
    return hipGetLastError();
}

#define CONVERT_CASES(SRC_)                                                                                        \
    switch (lf) {                                                                                                  \
    case L64_18: hipLaunchKernelGGL((k_convert_links<SRC_, L64_18>), grid, dim3(BLOCK), 0, s, src, dst, Vh, lcs); break; \
    case L64_12: hipLaunchKernelGGL((k_convert_links<SRC_, L64_12>), grid, dim3(BLOCK), 0, s, src, dst, Vh, lcs); break; \
    case L32_12: hipLaunchKernelGGL((k_convert_links<SRC_, L32_12>), grid, dim3(BLOCK), 0, s, src, dst, Vh, lcs); break; \
    case L16_12: hipLaunchKernelGGL((k_convert_links<SRC_, L16_12>), grid, dim3(BLOCK), 0, s, src, dst, Vh, lcs); break; \
    case LB16_12: hipLaunchKernelGGL((k_convert_links<SRC_, LB16_12>), grid, dim3(BLOCK), 0, s, src, dst, Vh, lcs); break; \
    case L16_8: hipLaunchKernelGGL((k_convert_links<SRC_, L16_8>), grid, dim3(BLOCK), 0, s, src, dst, Vh, lcs); break; \
    default: return hipErrorInvalidValue;                                                                          \
    }

hipError_t launch_convert_links(int lf, int src_lf, const void* src, void* dst, int Vh, long lcs, hipStream_t s)
{
    dim3 grid((unsigned)((Vh + BLOCK - 1) / BLOCK), 8);
    if (src_lf == L64_18) {
        CONVERT_CASES(L64_18)
    } else if (src_lf == L64_12) {
        CONVERT_CASES(L64_12)
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_temporal_gauge(const double* U, const Geo& g, double* gm, double* Uf, hipStream_t s)
{
    const long Vs = (long)g.X * g.Y * g.Z, V = Vs * g.T;
    hipLaunchKernelGGL(k_temporal_g, grid1((Vs + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, (const double2*)U, g,
                       (double2*)gm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_transform_links, grid1((V + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, (const double2*)U,
                       (const double2*)gm, g, (double2*)Uf);
    return hipGetLastError();
}

hipError_t launch_dots(SpinorRef a, const SpinorRef* bs, int m, const Geo& g, double* partials, double* out,
                       hipStream_t s)
{
    if (m < 1 || m > DOTS_MAX) return hipErrorInvalidValue;
    const int nb = (int)((2L * g.stride + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(k_dots, grid1(nb), dim3(BLOCK), 0, s, a, bs, m, g.Vh, g.stride, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dots_finish, dim3(1), dim3(BLOCK), 0, s, partials, nb, m, out);
    return hipGetLastError();
}

hipError_t launch_unpack_eo(double* dst, const Geo& g, SpinorRef xe, SpinorRef xo, SpinorRef bo, SpinorRef T,
                            double c0, double c1, int gamma5, double scale, hipStream_t s, const double* gm, int nc)
{
    const long V = (long)g.X * g.Y * g.Z * g.T;
    hipLaunchKernelGGL(k_unpack_eo, grid1((V + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, (double2*)dst, g, xe, xo, bo, T,
                       c0, c1, gamma5, scale, (const double2*)gm, nc);
    return hipGetLastError();
}

hipError_t launch_guess(const GuessArgs& a, hipStream_t s)
{
    if (a.k < 0 || a.k > GUESS_MAX || a.n <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_guess, grid1((a.n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_lincomb(double* out, const double* const* ins, const double* c, int k, long ncomplex, hipStream_t s)
{
    long nb = (ncomplex + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL(k_lincomb, grid1(nb), dim3(BLOCK), 0, s, (double2*)out, (const double2* const*)ins, c, k,
                       ncomplex);
    return hipGetLastError();
}

hipError_t launch_grad(const double* x, const double* lam, const Geo& g, const void* lk_even, const void* lk_odd,
                       long lcs, double* out, int project, hipStream_t s)
{
    const long V = (long)g.X * g.Y * g.Z * g.T;
    hipLaunchKernelGGL(k_grad, grid1((V + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, (const double2*)x,
                       (const double2*)lam, g, lk_even, lk_odd, lcs, (double2*)out, project);
    return hipGetLastError();
}

} // namespace wd
