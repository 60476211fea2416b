// Launchers of the libwdirac kernels (host side). Each returns the HIP error of the launch.
#pragma once
#include <hip/hip_ext.h>

#include "wd_types.hpp"

namespace wd {

enum HopRed { RED_NONE = 0, RED_ZDOT = 1, RED_OUTX = 2, RED_NORM = 3 };
enum SweepOp { OP_W = 0, OP_XR = 1, OP_S = 2, OP_SHIFT = 3, OP_INIT = 4, OP_ACC = 5, OP_NORM = 6, OP_MSINIT = 7, OP_AXPY = 8,
               OP_LINCOMB = 9, OP_CGX = 10, OP_CGP = 11, OP_CGPM = 12 };

// exec (may be NULL): incremented once per job that was not gated off. stage: LDS staging of the
// x/y neighbours (1 on, 0 off, -1 the defaults hop_stage_default() / hop_stage64_default()).
// tg: some job has temporal-gauge links (HopJob::tg); must be 0 for the adjoint hop. ntl:
// non-temporal link loads (for launches in which no two jobs share links through L2).
// ev0, ev1 (may be NULL): events that take the kernel's own start and end times (the launch is
// made with them, so the interval excludes the time between launches); a launcher that has
// nothing to launch (no blocks, no jobs) leaves them unrecorded.
hipError_t launch_hop(int sf, int lf, bool dag, int red, int fin, const HopJob* jobs, int njobs, long nblocks,
                      SysState* sys, int gated, hipStream_t s, int* exec = nullptr, int stage = -1, int tg = 0,
                      int ntl = 1, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Multi-RHS hop (tables whose jobs have rhs >= 2): kt = mrhs_kt(largest group), 2 or 4 systems per
// thread at most (0: unsupported group size). Low-precision spinors only.
int mrhs_kt(int k);
hipError_t launch_hop_mrhs(int sf, int lf, bool dag, int red, int kt, const HopJob* jobs, int njobs, long nblocks,
                           SysState* sys, int gated, hipStream_t s, int* exec = nullptr, hipEvent_t ev0 = nullptr,
                           hipEvent_t ev1 = nullptr);
int hop_stage_default();
int hop_stage64_default();
hipError_t launch_finish(int nr, int fin, const FinJob* fins, int nfin, SysState* sys, int gated, hipStream_t s,
                         hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_sweep(int op, int sfl, const SweepJob* jobs, int njobs, long nblocks, SysState* sys, int gated,
                        hipStream_t s, int* exec = nullptr, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// gm (may be NULL): canonical [V][3][3] colour rotation g(n): pack stores g(n) psi(n), unpack
// returns g(n)^dag psi'(n). nc: the internal field is in the non-chiral spin basis (pack rotates
// into it after gamma5 and g(n), unpack out of it before them)
hipError_t launch_pack_spinor(int sf, const double* src, const Geo& g, SpinorRef even, SpinorRef odd, int gamma5,
                              double scale, hipStream_t s, const double* gm = nullptr, int nc = 0);
hipError_t launch_unpack_spinor(int sf, double* dst, const Geo& g, SpinorRef even, SpinorRef odd, int gamma5,
                                double scale, hipStream_t s, const double* gm = nullptr, int nc = 0);
hipError_t launch_pack_links(const double* U, const Geo& g, void* even, void* odd, long lcs, hipStream_t s);
// canonical output of an even-odd solve: even sites from xe, odd sites c0 bo + c1 T (eq. eo3 with
// T = D_oe x_e), also stored into xo when xo.p is set; FP64 views of one parity each
hipError_t launch_unpack_eo(double* dst, const Geo& g, SpinorRef xe, SpinorRef xo, SpinorRef bo, SpinorRef T,
                            double c0, double c1, int gamma5, double scale, hipStream_t s, const double* gm = nullptr,
                            int nc = 0);
// internal links of format src_lf (L64_18 or L64_12) -> format lf, both output parities' halves
// separately (called per half)
hipError_t launch_convert_links(int lf, int src_lf, const void* src, void* dst, int Vh, long lcs, hipStream_t s);
// temporal gauge of canonical links U: gm = g(n) [V][3][3], Uf = transformed links [4][V][3][3]
hipError_t launch_temporal_gauge(const double* U, const Geo& g, double* gm, double* Uf, hipStream_t s);
hipError_t launch_recon_check(const void* lk, int Vh, long lcs, double* blockmax, hipStream_t s, int mode = 0);
// out[2 j], out[2 j + 1] = <a, bs[j]> (j < m <= DOTS_MAX) over the real sites of full FP64 fields;
// bs: device array of m views; partials: device, >= (2 stride / BLOCK + 1) * 2 * DOTS_MAX doubles
constexpr int DOTS_MAX = 8;
// start vector x0 = sum c_j x_j and its even-odd residual from the earlier solutions and their
// FP64 residuals (no operator application): see k_guess. be.p == nullptr: no b_e / h terms.
constexpr int GUESS_MAX = 8;
struct GuessArgs {
    SpinorRef x0, r0, be, h;
    SpinorRef bp;  // optional (first chunk): b_prec = a b_e + h
    double a;
    SpinorRef xs[GUESS_MAX], rs[GUESS_MAX];
    double c[GUESS_MAX], cx[GUESS_MAX];
    double cb, ch;
    long n;
    int k, acc;
};
hipError_t launch_guess(const GuessArgs& a, hipStream_t s);
hipError_t launch_dots(SpinorRef a, const SpinorRef* bs, int m, const Geo& g, double* partials, double* out,
                       hipStream_t s);
hipError_t launch_lincomb(double* out, const double* const* ins, const double* c, int k, long ncomplex, hipStream_t s);
hipError_t launch_grad(const double* x, const double* lam, const Geo& g, const void* lk_even, const void* lk_odd,
                       long lcs, double* out, int project, hipStream_t s);

} // namespace wd
