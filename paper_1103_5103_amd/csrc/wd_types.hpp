// Structures shared by the host driver and the kernels of libwdirac.
//
// Every kernel launch works on a list of jobs held in device memory. A job is one (system,
// parity) pair: the blocks of a launch are split over the jobs, so a single launch can advance
// many independent systems of different lattice sizes at once (batched solves), and a
// full-lattice operator is simply two jobs, one per output parity.
//
// Solver scalars live on the device (SysState), one record per system. Reductions are
// deterministic: every block of a kernel writes one partial sum, and a small follow-up kernel
// (one block per system) adds the partials in a fixed order and then updates the scalars
// ("finisher"). The kernel boundary orders the two, so no device-wide fence is needed inside
// the bandwidth-bound kernels. Kernels launched with a gate (a mask of statuses) skip the
// systems whose status is not in it: the iteration runs RUNNING systems only, so a whole chunk
// of iterations can be queued without host round trips, and the steps between chunks (reliable
// updates, restarts) run on the full job tables with the mask of the systems they concern.
#pragma once
#include "wd_device.hpp"

namespace wd {

enum SysStatus {
    ST_RUNNING = 0,
    ST_CONVERGED = 1,   // iterated residual below target: verify with an FP64 residual
    ST_RELIABLE = 2,    // reliable update due
    ST_BREAKDOWN = 3,
    ST_NAN = 4,
    ST_MAXIT = 5,
    ST_DONE = 6,        // set by the host for a finished system of a batch (no kernel runs it)
    ST_SEL1 = 7,        // set by the host to select systems for a gated step (e.g. continue
    ST_SEL2 = 8,        //   after a reliable update / restart fresh; finish by sweep / by hop)
};
// Kernel gates are masks of the statuses allowed to run (0: no gating); GATE_RUN = the iteration.
constexpr int GATE_RUN = 1 << ST_RUNNING;
constexpr int GATE_STOPPED = (1 << ST_CONVERGED) | (1 << ST_RELIABLE) | (1 << ST_BREAKDOWN) | (1 << ST_MAXIT);

// Finisher kinds (what the last block does with the reduced sums)
enum Fin {
    FIN_STORE = 0,   // keep the sums in red[] for the host
    FIN_BETA = 1,    // beta = -delta / <rhat, A s>            (+ shifted zeta, beta)
    FIN_CHI = 2,     // chi = <A w, w> / <A w, A w>          (+ shifted chi, rho)
    FIN_ALPHA = 3,   // delta' = <rhat, r>, |r|^2, alpha    (+ shifted alpha, freezing)
    FIN_END = 4,     // end of iteration: commit status     (+ rotate shifted scalars)
    FIN_RESTART = 5, // new residual: delta = <rhat, r>, |r|^2, status RUNNING
    FIN_CGA = 6,     // CG: alpha = |r|^2 / <p, A p>                (+ shifted zeta, alpha)
    FIN_CGB = 7,     // CG: beta = |r_new|^2 / |r|^2, status     (+ shifted beta, freezing)
    FIN_CGEND = 8,   // CG-M end of iteration: commit status, rotate the shifted zeta
};

struct ShiftScal {
    double sigma;
    double2 zeta_prev, zeta, zeta_next;
    double2 rho, rho_next;
    double2 beta_s, chi_s, alpha_s;
    int active;      // 1: updated this iteration, 0: frozen
    int freeze;      // freeze after this iteration
    int conv_iter;   // iteration at which the shift was frozen
    int pad;
};

struct SysState {
    int status;        // SysStatus
    int pending;       // status committed at the end of the iteration
    int iter;
    int maxit;
    int mixed;
    int rsel;          // which residual buffer holds r_n (multi-shift keeps r_n and r_{n+1})
    int nshift;
    int dc;            // defect correction: the reliable-update threshold is relative to the
                       // residual at the start of the inner solve (maxrr is not raised)
    double2 delta, beta, chi, alpha, beta_prev;
    double rr;         // |r|^2 of the iterated residual
    double maxrr;      // max |r|^2 since the last reliable update
    double target2;    // stop when rr <= target2
    double delta_rel2; // reliable update when rr < delta_rel2 * maxrr
    double shift_target2;
    double cga, cga_prev, cgb;  // CG: alpha_n, alpha_{n-1}, beta_n
    double red[NRED];  // last reduced sums
    double* partials;  // [max blocks][NRED]
    ShiftScal* sh;     // [nshift]
    SpinorRef* shv;    // [2 * nshift]: x_sigma, s_sigma (BiCGstab-M) or x_sigma, p_sigma (CG-M)
};

// one entry per system of a launch: which partial sums the finisher adds
struct FinJob {
    int sys;
    int rnblk;
};

struct HopJob {
    Geo g;
    int parity;  // output parity
    int sys;     // SysState index (reduction group and gate)
    int blk0;    // first block of this job in the launch
    int nblk;
    int rblk0;   // first block within the system's reduction group
    int rnblk;   // blocks in the reduction group
    SpinorRef in;        // input half field (the other parity)
    SpinorRef out;       // output half field
    SpinorRef x0, x1;    // epilogue terms (p == nullptr: absent)
    SpinorRef z;         // partner of <z, out>
    const void* links;   // the 8 links per site of this output parity
    long lcs;            // link chunk stride
    double c0, c1, c2;   // out = c0 x0 + c1 x1 + c2 * hop
    int tz;              // block order: 0 = site order; > 0 = t fastest within groups of tz z-planes
    int bpp;             // blocks per (z, t) plane when tz > 0
    // Jobs that read the same links (same gauge field and parity) may form an interleaved group
    // of ilv consecutive jobs with equal blk0: block blk0 + ilv * l + k runs block l of job
    // (first + k), so the systems' blocks for one range of sites run together on one XCD and the
    // links come from memory once and from L2 for the others.
    int ilv;             // jobs in the group (1: not interleaved)
    int ilv_pos;         // position of this job in its group
    int tg;              // links in temporal gauge: the time links are the unit matrix except
                         // those leaving the last time slice (not loaded, not multiplied)
    // rhs >= 2: the group is run by the multi-RHS hop instead (k_hop_mrhs): one thread per output
    // site applies the hop to all ilv (<= rhs) systems of the group, loading each link once; the
    // group then spans nblk blocks rather than ilv * nblk. Every job of a launch has the same mode.
    int rhs;
    int nc;              // spinors in the non-chiral basis (gamma_4 diagonal): time hops read and
                         // update two spin components (hop_t_nc)
};

// Roles of the fields of a sweep job
enum SweepRole { R_F0 = 0, R_F1, R_F2, R_F3, R_F4, R_F5, R_F6, R_F7, NROLE };

struct SweepJob {
    int sys;
    int n;       // sites
    int blk0;
    int nblk;
    int rblk0;
    int rnblk;
    int flags;   // op-specific
    int pad;
    double c[8]; // op-specific coefficients
    SpinorRef f[NROLE];
};

} // namespace wd
