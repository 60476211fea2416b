/*
 * wdirac: Wilson-Dirac multi-mass BiCGstab solves on one AMD MI355X (gfx950).
 *
 * C ABI of libwdirac.so. Every entry point takes plain device pointers and sizes; no C++ or
 * framework types cross the boundary, and no exception escapes it.
 *
 * Paper: A. Alexandru, C. Pelissier, B. Gamari, F. Lee, "Multi-mass solvers for lattice QCD on GPUs".
 *
 * Conventions shared by every call
 * ---------------------------------
 * Lattice: extents X, Y, Z, T (dims[0..3]), all even and >= 2. Site order is x fastest:
 *   n = x + X*(y + Y*(z + Z*t)).  Directions mu = 0,1,2,3 are x,y,z,t (the paper's 1..4).
 *   Space is periodic; time is antiperiodic when geom.antiperiodic_t = 1 (periodic when 0).
 * Fermion field (paper Sec. 2, after eq. 3): 12 complex numbers per site, a 3x4 colour-by-spin
 *   matrix; device array of interleaved complex128 (double re, double im), shape [V][3][4],
 *   i.e. 24 doubles per site, colour major, spin minor. V = X*Y*Z*T.
 * Gauge field (Sec. 2, eq. 4): U_mu(n), the SU(3) link from n to n+mu; device array of complex128,
 *   shape [4][V][3][3] (mu, site, row, column).
 * Operator (Sec. 2, eq. 3 and eq. 4) with the paper's mass written through kappa,
 *   m a + 4 = 1/(2 kappa):
 *     (M psi)_n = psi_n/(2 kappa) - 1/2 sum_mu [ U_mu(n) psi_{n+mu} (1 - gamma_mu)
 *                                            + U_mu(n-mu)^dag psi_{n-mu} (1 + gamma_mu) ]
 *   with the chiral gamma matrices of Sec. 2 multiplying the 3x4 site matrix from the right, and
 *   a factor -1 on the time hops that cross the t boundary when antiperiodic.
 *   M^dag = gamma5 M gamma5, gamma5 = diag(1, 1, -1, -1) on the spin index.
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the default stream). Every kernel is
 *   launched on it. wd_apply, wd_apply_dag and wd_gauge_grad are asynchronous; the solvers
 *   return after the solve has finished (they synchronise the stream).
 * Ownership: the caller owns every field buffer (allocate and free them yourself, e.g. with
 *   torch). The library owns wd_gauge handles and their workspaces: created by
 *   wd_gauge_create, released by wd_gauge_destroy. A handle may be used from one host thread at
 *   a time; calls on one handle must not overlap.
 * Errors: every call returns a wd_status. WD_OK on success. On failure nothing is thrown;
 *   wd_last_error gives a thread-local message. Device pointers are not dereferenced on the
 *   host; NULL pointers and misaligned pointers (not 16-byte aligned) give WD_ERR_ARG.
 */
#ifndef WDIRAC_H
#define WDIRAC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WD_OK = 0,
    WD_ERR_ARG = 1,         /* invalid argument (shape, pointer, parameter)            */
    WD_ERR_HIP = 2,         /* a HIP runtime call failed                               */
    WD_ERR_OOM = 3,         /* device allocation failed                                */
    WD_ERR_NOCONV = 4,      /* max_iter reached; x holds the last iterate, stats filled */
    WD_ERR_BREAKDOWN = 5,   /* BiCGstab breakdown (<rhat, A s> or chi vanished) after one restart */
    WD_ERR_NAN = 6,         /* a NaN or Inf appeared in the iteration                   */
    WD_ERR_UNSUPPORTED = 7  /* combination of options not implemented                   */
} wd_status;

typedef enum { WD_F64 = 0, WD_F32 = 1, WD_F16 = 2, WD_BF16 = 3 } wd_prec;

typedef struct {
    int dims[4];        /* X, Y, Z, T: all even, >= 2 */
    int antiperiodic_t; /* 1: antiperiodic in time (default), 0: periodic */
} wd_geom;

typedef struct wd_gauge wd_gauge; /* opaque: geometry, packed links, workspaces */

typedef struct {
    double tol;            /* stop when |b - M x| < tol |b| (Sec. 6.1 exit criterion)                   */
    int max_iter;          /* iteration cap (per mass for sequential solves)                           */
    int mixed;             /* 0: FP64 throughout. 1: iterate with low-precision storage and FP32
                              arithmetic, FP64 reductions, FP64 reliable updates of x and r             */
    wd_prec spinor_store;  /* storage of the iterated vectors when mixed: WD_F32 or WD_F16             */
    wd_prec link_store;    /* storage of the links of the low-precision operator: WD_F32, WD_F16,
                              WD_BF16                                                                  */
    int recon;             /* link format of the low-precision operator: 12 (two rows stored, third
                              rebuilt from unitarity), 18, or 8 (WD_F16 only: u01, u02, u10 and the
                              phases of u00 and u20, the rest rebuilt from unitarity, 16 bytes per
                              link; SU(3) links with |u00| < 1 - 1e-6 on every link, caller's gauge
                              only, else WD_ERR_UNSUPPORTED)                                           */
    int eo;                /* 1: even-odd preconditioning (Sec. 6.2.3); single-mass solves only       */
    double delta_reliable; /* mixed: reliable update once |r| < delta * max|r| since the last one     */
    int use_x0;            /* 1: x holds the start vector on entry (single-mass solves only)          */
    int dagger;            /* 1: solve M^dag x = b instead, through M^dag = gamma5 M gamma5            */
    int mixed_mode;        /* mixed only. WD_MIXED_RELIABLE: one Krylov run; x and r are refreshed in
                              FP64 once |r| < delta * max|r| since the last refresh, keeping the
                              shadow vector and search direction. WD_MIXED_DEFECT: defect correction
                              (Sec. 6.2.4): each inner low-precision solve of M e = r runs until |r|
                              drops below delta times its starting value, then x += e and r = b - M x
                              are updated in FP64 and a fresh inner solve starts                       */
    int guess_order;       /* sequential multi-mass start guesses use at most this many previous
                              solutions, the most recently solved ones (0: all of them)               */
    int temporal_gauge;    /* read by wd_gauge_create only: 1 = the handle's solvers work in temporal
                              gauge (a bandwidth saving named in Sec. 4): sources are rotated by
                              g(x,t) = U_t(x,0)...U_t(x,t-1), solutions back by g^dag, and the time
                              links, then the unit matrix except on the last time slice, are neither
                              loaded nor multiplied. Only for links that are SU(3) to rounding (else
                              ignored). Solutions agree with the caller's gauge to rounding.          */
    int gamma_basis;       /* read by wd_gauge_create only: 0 = the solvers work in the chiral basis of
                              Sec. 2 (Table 1); 1 = in a non-chiral basis where gamma_4 is diagonal
                              (a bandwidth saving named in Sec. 4): sources are rotated into it by
                              psi S, S = [[1, 1], [-1, 1]] / sqrt(2) in 2x2 spin blocks, solutions
                              back by S^dag, and a time hop reads two of the neighbour's four spin
                              components. Fields crossing the ABI stay in the chiral basis; solutions
                              agree with the chiral solves to rounding.                                */
} wd_solver_params;

typedef struct {
    int iters;             /* Krylov iterations                                                    */
    int reliable_updates;  /* FP64 residual recomputations (mixed mode)                            */
    int status;            /* wd_status of this system                                             */
    double true_rel_res;   /* |b - M x| / |b| in FP64 after the solve (even-odd solves: from their last
                              FP64 even-site residual, which equals the full one up to the rounding
                              of the rebuilt odd half; NaN after WD_ERR_NAN)                          */
    double seconds;        /* wall time of this system's solve (shared wall time for joint solves) */
} wd_solver_stats;

typedef struct {
    wd_gauge* gauge;   /* lattice and links of this system          */
    double kappa;      /* mass parameter                            */
    const double* b;   /* device, [V][3][4] complex128 source       */
    double* x;         /* device, [V][3][4] complex128 solution     */
} wd_system;

enum { WD_METHOD_SEQUENTIAL = 0, WD_METHOD_MULTISHIFT = 1, WD_METHOD_BATCHED = 2 };
enum { WD_GUESS_NONE = 0, WD_GUESS_POLY = 1, WD_GUESS_MINRES = 2 };
enum { WD_MIXED_RELIABLE = 0, WD_MIXED_DEFECT = 1 };

/* Defaults: tol 1e-8, max_iter 5000, mixed 1, F32 spinors, F16 links, recon 12, eo 1,
   delta_reliable 0.1, use_x0 0, dagger 0, mixed_mode WD_MIXED_RELIABLE, guess_order 0,
   temporal_gauge 0, gamma_basis 0. */
void wd_params_default(wd_solver_params* p);

/*
 * Build a handle for one lattice and gauge field (Sec. 4, eq. 8 describes the paper's link
 * layout; the handle stores its own layout). U: device pointer, complex128 [4][V][3][3], read
 * during the call only (it may be freed afterwards). storage_hint (may be NULL): low-precision
 * link formats to build now; others are built on first use.
 * Errors: WD_ERR_ARG for odd or < 2 extents or NULL pointers, WD_ERR_OOM, WD_ERR_HIP.
 */
wd_status wd_gauge_create(wd_gauge** g, const wd_geom* geom, const double* U,
                          const wd_solver_params* storage_hint, void* stream);
wd_status wd_gauge_destroy(wd_gauge* g);

/* out = M(kappa) in  (Sec. 2, eq. 3 and 4; FP64). in, out: device [V][3][4] complex128, distinct. */
wd_status wd_apply(wd_gauge* g, double kappa, double* out, const double* in, void* stream);
/* out = M(kappa)^dag in = gamma5 M gamma5 in (FP64). */
wd_status wd_apply_dag(wd_gauge* g, double kappa, double* out, const double* in, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): out = M(kappa) in (dagger = 0) or M(kappa)^dag in
 * (dagger = 1), bitwise the result of wd_apply / wd_apply_dag, with no device or pinned
 * allocation, no host-to-device copy and no synchronisation. The packed fields and the job table
 * live in a fixed device array of 64 MiB per GPU that the library holds until the process ends;
 * it fits lattices of at most 87,296 sites per parity after rounding V/2 up to a multiple of 256
 * (16^3 x 32 fits, 24^4 does not); larger lattices give WD_ERR_ARG. Every call on one GPU uses
 * that GPU's array: calls that overlap on one GPU (other streams or threads) race, so serialise
 * them. in, out: device [V][3][4] complex128, distinct. Asynchronous on `stream`.
 */
wd_status wd_apply_noalloc(wd_gauge* g, double kappa, double* out, const double* in, int dagger, void* stream);

/*
 * Single-mass BiCGstab for M(kappa) x = b (van der Vorst's method, cited in Sec. 6; the solution
 * update x <- x - beta s + chi w of Sec. 5). With params->eo the even-odd system of Sec. 6.2.3
 * (eq. eo2-eo4) is solved and the odd half rebuilt from eq. eo3. With params->mixed the
 * iteration runs with low-precision storage and FP64 updates of x and r: reliable updates inside
 * one Krylov run, or the paper's defect correction with restarted inner solves (Sec. 6.2.4),
 * selected by params->mixed_mode.
 * x, b: device [V][3][4] complex128. stats (may be NULL): filled on return, also on NOCONV.
 * Returns WD_OK, WD_ERR_NOCONV (x holds the last iterate), WD_ERR_BREAKDOWN, WD_ERR_NAN, ...
 */
wd_status bicgstab_solve(wd_gauge* g, double kappa, double* x, const double* b,
                         const wd_solver_params* params, wd_solver_stats* stats, void* stream);

/*
 * Multi-shift BiCGstab-M (Jegerlehner, cited in Sec. 6.1) for M(kappa_i) x_i = b, i < n, FP64,
 * full lattice, zero start vectors (the paper notes even-odd preconditioning, mixed precision and
 * start guesses do not apply). The unshifted system is the most singular one (largest kappa);
 * each shifted system stops being updated once it has converged; the solve stops when the
 * unshifted residual satisfies |r| < tol |b| (Sec. 6.1). x: host array of n device pointers.
 * stats: host array of n entries (may be NULL). 1 <= n <= 32.
 */
wd_status bicgstab_m_solve(wd_gauge* g, int n, const double* kappas, double* const* x, const double* b,
                           const wd_solver_params* params, wd_solver_stats* stats, void* stream);

/*
 * Multi-mass driver (Sec. 6, eq. 6.1; Sec. 7). method WD_METHOD_SEQUENTIAL: single-mass BiCGstab
 * once per mass, heaviest mass (smallest kappa) first; with WD_GUESS_POLY each start vector is the
 * highest-order Lagrange extrapolation in m a of the solutions found so far (Sec. 6.2.1); with
 * WD_GUESS_MINRES it is the combination of those solutions that minimises |b - M(kappa) v|_2
 * (solution-space minimisation, Sec. 6.2.2: since M(kappa) psi_k = b + (1/(2 kappa) -
 * 1/(2 kappa_k)) psi_k, the normal equations need inner products of the stored solutions only, no
 * operator application). params->guess_order limits either guess to the most recent solutions.
 * method WD_METHOD_MULTISHIFT: one bicgstab_m_solve. method WD_METHOD_BATCHED: the single-mass
 * systems of all masses iterate together (one kernel launch per solver step for all of them,
 * converged masses drop out, even-odd required); no start guesses. 1 <= n <= 32.
 */
wd_status wd_multimass_solve(wd_gauge* g, int n, const double* kappas, double* const* x, const double* b,
                             int method, int guess, const wd_solver_params* params,
                             wd_solver_stats* stats, void* stream);

/*
 * Batched single-mass solves: nsys independent systems (any mix of handles, lattices, kappas and
 * sources) iterate together, one kernel launch per solver step for all of them; converged
 * systems drop out. Even-odd preconditioning is required (params->eo = 1). sys: host array.
 * stats: host array of nsys entries (may be NULL). 1 <= nsys <= 1024.
 */
wd_status wd_batch_solve(int nsys, const wd_system* sys, const wd_solver_params* params,
                         wd_solver_stats* stats, void* stream);

/*
 * Shifted normal equations on the even sites (Sec. 8 names CG and its multi-shift form CG-M as
 * the Krylov pair the paper's findings carry over to; shifted systems share one Krylov space,
 * Sec. 6.1):  (M_prec^dag M_prec + sigma_i) x_i = b_e,  i < n,
 * with M_prec = (1/(2 kappa))^2 - 1/4 D_eo D_oe the even-odd operator of eq. eo4 (Hermitian
 * positive definite for sigma_i >= 0). b: device [V][3][4] complex128, its odd sites are ignored;
 * x: host array of n device pointers [V][3][4], the odd sites are set to zero. method
 * WD_METHOD_MULTISHIFT: CG-M in FP64, zero start vectors, base = the smallest shift, each other
 * shift frozen once |zeta_i| |r| <= tol |b_e|. method WD_METHOD_SEQUENTIAL: CG once per shift,
 * largest shift first, with WD_GUESS_POLY a start vector extrapolated (Lagrange, in sigma) from
 * the solutions found so far (params->guess_order limits it), and params->mixed / mixed_mode /
 * the storage formats as for bicgstab_solve (FP64 reliable updates r = b_e - (A + sigma) x, or
 * defect correction). method WD_METHOD_BATCHED: the single-shift CG systems of all shifts
 * iterate together, no start guesses. stats: the true residual is |b_e - (A + sigma_i) x_i| /
 * |b_e| in FP64. 1 <= n <= 32, sigma_i >= 0, params->dagger = 0, guess NONE or POLY;
 * params->use_x0 is ignored (x is output only). On WD_ERR_NOCONV x holds the last iterate.
 */
wd_status wd_normal_solve(wd_gauge* g, double kappa, int n, const double* sigmas, double* const* x,
                          const double* b, int method, int guess, const wd_solver_params* params,
                          wd_solver_stats* stats, void* stream);

/*
 * Link derivative of L = Re <eta, M(kappa)^{-1} b> given x = M^{-1} b and lam = M^{-dag} eta
 * (obtained by differentiating eq. 3/4 with respect to U):
 *   G_mu(n) = 1/2 s [ lam_n (1 - gamma_mu) x_{n+mu}^dag + x_n (1 + gamma_mu) lam_{n+mu}^dag ],
 * the complex derivative dL/dRe U + i dL/dIm U. With project = 1 the output is instead the
 * su(3)-valued force F = (i/2) TA(U G^dag), TA(Y) = (Y - Y^dag)/2 - tr(Y - Y^dag)/6, for which
 * dL/de_a = 2 tr(T_a F) under U -> exp(i e_a T_a) U. x, lam: device [V][3][4]; dU: device
 * [4][V][3][3] complex128. Asynchronous.
 */
wd_status wd_gauge_grad(wd_gauge* g, const double* x, const double* lam, double* dU, int project,
                        void* stream);

/*
 * How wd_apply_prec runs its two hops: each field selects one of the hop-kernel variants the
 * solvers launch, so that every variant can be compared with the FP64 definition site by site.
 */
enum { WD_RED_NONE = 0, WD_RED_ZDOT = 1, WD_RED_OUTX = 2, WD_RED_NORM = 3 };
typedef struct {
    int red;          /* reduction fused into the second hop (the solvers' epilogues):
                         WD_RED_NONE; WD_RED_ZDOT <in_e, out_e>; WD_RED_OUTX <out_e, in_e> and
                         |out_e|^2; WD_RED_NORM |out_e|^2 (all sums in FP64)                      */
    int stage;        /* LDS staging of the x and y neighbours: -1 library default, 0 off, 1 on   */
    int nontemporal;  /* cache policy of the hops: -1 the solvers' policy, 0 ordinary, 1
                         non-temporal link loads, epilogue-field loads and output stores (the
                         first, plain hop of a low-precision operator keeps ordinary stores)     */
    int tile;         /* block order: -1 autotuned, 0 site order, tz > 0 t fastest within groups
                         of tz z-planes (site order where the lattice does not allow tz)          */
    int copies;       /* 1..64 systems in one launch; in and out then hold that many fields, one
                         after the other. Systems on one gauge field share their link loads      */
    int rhs_per_thread; /* -1: the tuned choice (as in the batched solvers); 0 or 1: one system
                           per thread (systems sharing links run in interleaved block pairs);
                           k in 2..4: the multi-RHS hop, up to k systems per thread with each
                           link loaded once for all of them (FP32 / FP16 spinors, reductions
                           other than WD_RED_NORM)                                               */
    int dagger;       /* 1: the adjoint operator (both hops with swapped projectors, M^dag =
                         gamma5 M gamma5); reductions WD_RED_NONE or WD_RED_ZDOT only            */
} wd_op_variant;

/* Defaults: red WD_RED_NONE, stage -1, nontemporal -1, tile -1, copies 1, rhs_per_thread -1,
   dagger 0. */
void wd_op_variant_default(wd_op_variant* v);

/*
 * The even-odd operator exactly as the solvers apply it in their storage formats (Sec. 6.2.3,
 * eq. eo4, built from the hopping term of Sec. 2, eq. 3 and 4, with the spin projection of
 * Table 1): `in` is packed into params->spinor_store (WD_F64 when params->mixed = 0) and the hops
 * read the handle's links in params->link_store / params->recon (the FP64 operator's format when
 * params->mixed = 0), in the handle's gauge (temporal gauge when the handle was created with it;
 * sources and results are rotated as in the solvers). Two hops run:
 *   out_o = D_oe in_e                                  (first hop, its stored low-precision value)
 *   out_e = (1/(2 kappa))^2 in_e - 1/4 D_eo out_o     (second hop with the fused epilogue),
 * so out_e = M_prec in_e and out_o is the hopping term from the even to the odd sites; with
 * v->dagger the adjoint hops give out_o = (D_eo)^dag in_e and out_e = M_prec^dag in_e. The odd
 * sites of `in` are ignored. in, out: device, v->copies consecutive [V][3][4] complex128 fields
 * (distinct, not overlapping). dots (host, may be NULL): 3 doubles per copy, the fused sums of
 * v->red in the order listed there (unused entries 0). v (may be NULL): defaults.
 * Errors: WD_ERR_ARG, WD_ERR_UNSUPPORTED (format or variant not available for these links).
 * Returns after the result is in `out` (synchronises the stream).
 */
wd_status wd_apply_prec(wd_gauge* g, double kappa, double* out, const double* in, const wd_solver_params* params,
                        const wd_op_variant* v, double* dots, void* stream);

/* Human-readable name of a status code (static string). */
const char* wd_status_str(wd_status s);
/* Copy the calling thread's last error message into buf (n bytes, NUL-terminated). */
wd_status wd_last_error(char* buf, size_t n);

/*
 * Kernel timing (measurement support, not part of the method). When enabled, each launch of the
 * named kernel classes is made with a pair of HIP events on the launch stream that take the
 * kernel's own start and end times (hipExtLaunchKernel), and their durations are accumulated;
 * reading the totals synchronises the device. Solver iterations are not replayed from graphs
 * while timing is on.
 * class: 0 = low-precision even-odd hop, 1 = FP64 hop, 2 = fused vector sweeps,
 *        3 = the small finisher kernels that complete the reductions, 4 + r = the low-precision
 *        hops with fused reduction r (WD_RED_NONE .. WD_RED_NORM; also counted in class 0).
 * bytes: the compulsory bytes of the counted launches (launches in which every system was gated
 *        off are not counted).
 */
void wd_timing_enable(int on);
void wd_timing_reset(void);
wd_status wd_timing_get(int kernel_class, double* total_ms, long* launches, double* bytes);

/*
 * Execution option: replay each chunk of solver iterations from a captured HIP graph (1) or launch
 * its kernels one by one (0, the default). A handle keeps its captured chunks and reuses them for
 * later solves with identical launches. Results are identical either way (measured no faster on
 * MI355X). Graphs are not used while kernel timing is enabled. Process-wide; not thread-safe
 * against concurrent solves.
 */
void wd_set_graphs(int on);

/* Bytes of device memory held by a handle (links and cached workspaces). */
size_t wd_gauge_device_bytes(const wd_gauge* g);

#ifdef __cplusplus
}
#endif
#endif /* WDIRAC_H */
