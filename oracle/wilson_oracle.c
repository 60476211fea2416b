/*
 * Wilson-Dirac CPU oracle: TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 implementation of what the GPU path computes, used to check it.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg load this
 * library. The GPU library neither links nor calls it, and this file shares no code,
 * header, table or constant with the GPU sources.
 *
 * Paper: "Multi-mass solvers for lattice QCD on GPUs" (Alexandru, Pelissier, Gamari, Lee).
 *
 * Layout (lexicographic, x fastest, interleaved complex):
 *   site n = x + X*(y + Y*(z + Z*t)),  mu = 0,1,2,3 <-> x,y,z,t  (paper's mu = 1..4)
 *   fermion psi[n][c][s]   : a 3x4 colour-by-spin matrix per site (Sec. 2, after eq. 3)
 *   gauge   U[mu][n][a][b] : the SU(3) link from n to n+mu (Sec. 2, eq. 4)
 * Boundary: periodic in x, y, z; antiperiodic in t when `anti` is set (the paper is silent;
 * the sign is applied to the time hops that cross the t boundary).
 *
 * Normalisation: M(kappa) is the paper's M(m;U) with m*a + 4 = 1/(2 kappa):
 *   (M psi)_n = (1/(2 kappa)) psi_n - 1/2 sum_{mu=+-1..+-4} (T_mu psi)_n       (Sec. 2, eq. 3)
 *   (T_{+mu} psi)_n = U_mu(n) psi_{n+mu} (1 - gamma_mu)                         (eq. 4)
 *   (T_{-mu} psi)_n = U_mu(n-mu)^dag psi_{n-mu} (1 + gamma_mu)                  (eq. 4)
 * The spin matrices multiply the 3x4 site matrix from the right, as full 4x4 products;
 * no spin-projection shortcut is used here.
 * The adjoint M^dag (with <a,b> = sum conj(a) b) swaps (1 - gamma) and (1 + gamma).
 *
 * Parity pins (tests): Table 1 projector identities, gamma5-hermiticity, gauge covariance,
 * the free-field momentum-space closed form, dense LU on a 2^4 lattice, even-odd solution
 * equal to the full solution, shifted true residuals of BiCGstab-M, and central finite
 * differences for the link gradient.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ---------------------------------------------------------------- gamma matrices */

/* gamma_i = [[0, i sigma_i], [-i sigma_i, 0]], gamma_4 = [[0, -1], [-1, 0]] (Sec. 2). */
static cplx GAMMA[4][4][4];
static cplx PMINUS[4][4][4]; /* 1 - gamma_mu */
static cplx PPLUS[4][4][4];  /* 1 + gamma_mu */
static int gamma_ready = 0;

static void build_gammas(void)
{
    if (gamma_ready) return;
    cplx sigma[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(GAMMA, 0, sizeof(GAMMA));
    for (int i = 0; i < 3; i++)
        for (int r = 0; r < 2; r++)
            for (int c = 0; c < 2; c++) {
                GAMMA[i][r][2 + c] = I * sigma[i][r][c];
                GAMMA[i][2 + r][c] = -I * sigma[i][r][c];
            }
    for (int r = 0; r < 2; r++) {
        GAMMA[3][r][2 + r] = -1;
        GAMMA[3][2 + r][r] = -1;
    }
    for (int mu = 0; mu < 4; mu++)
        for (int r = 0; r < 4; r++)
            for (int c = 0; c < 4; c++) {
                cplx id = (r == c) ? 1.0 : 0.0;
                PMINUS[mu][r][c] = id - GAMMA[mu][r][c];
                PPLUS[mu][r][c] = id + GAMMA[mu][r][c];
            }
    gamma_ready = 1;
}

/* Export gamma_mu (mu = 0..3) as 16 interleaved complex numbers, row-major. */
void oracle_gamma(int mu, double *out)
{
    build_gammas();
    memcpy(out, GAMMA[mu], sizeof(GAMMA[mu]));
}

/* ---------------------------------------------------------------- geometry */

static long vol(const int *L) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void coords(const int *L, long n, int *x)
{
    x[0] = (int)(n % L[0]); n /= L[0];
    x[1] = (int)(n % L[1]); n /= L[1];
    x[2] = (int)(n % L[2]); n /= L[2];
    x[3] = (int)n;
}

static long index_of(const int *L, const int *x)
{
    return x[0] + (long)L[0] * (x[1] + (long)L[1] * (x[2] + (long)L[2] * x[3]));
}

/* neighbour n + dir*mu_hat with periodic wrap */
static long neighbour(const int *L, const int *x, int mu, int dir)
{
    int y[4] = {x[0], x[1], x[2], x[3]};
    y[mu] = (y[mu] + dir + L[mu]) % L[mu];
    return index_of(L, y);
}

int oracle_parity(const int *L, long n)
{
    int x[4];
    coords(L, n, x);
    return (x[0] + x[1] + x[2] + x[3]) & 1;
}

/* ---------------------------------------------------------------- hopping term */

/*
 * out_n = sum_mu [ s U_mu(n) psi_{n+mu} P_fwd + s U_mu(n-mu)^dag psi_{n-mu} P_bwd ]
 * with (P_fwd, P_bwd) = (1 - gamma, 1 + gamma) for D and swapped for D^dag (Sec. 2, eq. 4).
 * s = -1 for a time hop that crosses the t boundary when `anti` is set.
 */
void oracle_hopping(const int *L, int anti, const double *Ud, const double *ind, double *outd, int dag)
{
    build_gammas();
    const cplx *U = (const cplx *)Ud;
    const cplx *psi = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    const long V = vol(L);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < V; n++) {
        int x[4];
        coords(L, n, x);
        cplx acc[3][4];
        memset(acc, 0, sizeof(acc));
        for (int mu = 0; mu < 4; mu++) {
            for (int dir = +1; dir >= -1; dir -= 2) {
                long m = neighbour(L, x, mu, dir);
                double sgn = 1.0;
                if (anti && mu == 3) {
                    if (dir == +1 && x[3] == L[3] - 1) sgn = -1.0;
                    if (dir == -1 && x[3] == 0) sgn = -1.0;
                }
                /* colour matrix: U_mu(n) forward, U_mu(n-mu)^dag backward */
                cplx W[3][3];
                if (dir == +1) {
                    const cplx *u = U + ((long)mu * V + n) * 9;
                    for (int a = 0; a < 3; a++)
                        for (int b = 0; b < 3; b++) W[a][b] = u[a * 3 + b];
                } else {
                    const cplx *u = U + ((long)mu * V + m) * 9;
                    for (int a = 0; a < 3; a++)
                        for (int b = 0; b < 3; b++) W[a][b] = conj(u[b * 3 + a]);
                }
                /* spin matrix */
                const cplx (*P)[4];
                if ((dir == +1) != (dag != 0)) P = (const cplx(*)[4])PMINUS[mu];
                else P = (const cplx(*)[4])PPLUS[mu];
                const cplx *p = psi + m * 12;
                /* tmp = W * psi_m  (3x3 times 3x4) */
                cplx tmp[3][4];
                for (int a = 0; a < 3; a++)
                    for (int s = 0; s < 4; s++) {
                        cplx v = 0;
                        for (int b = 0; b < 3; b++) v += W[a][b] * p[b * 4 + s];
                        tmp[a][s] = v;
                    }
                /* acc += sgn * tmp * P  (3x4 times 4x4) */
                for (int a = 0; a < 3; a++)
                    for (int s = 0; s < 4; s++) {
                        cplx v = 0;
                        for (int r = 0; r < 4; r++) v += tmp[a][r] * P[r][s];
                        acc[a][s] += sgn * v;
                    }
            }
        }
        for (int a = 0; a < 3; a++)
            for (int s = 0; s < 4; s++) out[n * 12 + a * 4 + s] = acc[a][s];
    }
}

/* out = M(kappa) in, or M(kappa)^dag in when dag != 0 (Sec. 2, eq. 3) */
void oracle_apply(const int *L, int anti, const double *U, double kappa, const double *ind, double *outd, int dag)
{
    const long N = vol(L) * 12;
    cplx *hop = malloc(sizeof(cplx) * N);
    oracle_hopping(L, anti, U, ind, (double *)hop, dag);
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    const double diag = 1.0 / (2.0 * kappa);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; i++) out[i] = diag * in[i] - 0.5 * hop[i];
    free(hop);
}

/* ---------------------------------------------------------------- even-odd (Sec. 6.2.3) */

/* Zero the sites of parity `par` (0 even, 1 odd) in a full-length field. */
static void zero_parity(const int *L, cplx *f, int par)
{
    const long V = vol(L);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < V; n++)
        if (oracle_parity(L, n) == par)
            for (int k = 0; k < 12; k++) f[n * 12 + k] = 0;
}

/*
 * M_prec psi_e = (1/(2 kappa))^2 psi_e - 1/4 D_eo D_oe psi_e            (eq. eo4)
 * Fields are full length; `in` must vanish on odd sites, `out` does on return.
 */
void oracle_mprec(const int *L, int anti, const double *U, double kappa, const double *ind, double *outd, int dag)
{
    const long V = vol(L), N = V * 12;
    cplx *t1 = malloc(sizeof(cplx) * N), *t2 = malloc(sizeof(cplx) * N);
    memcpy(t1, ind, sizeof(cplx) * N);
    zero_parity(L, t1, 1);
    oracle_hopping(L, anti, U, (double *)t1, (double *)t2, dag); /* odd part = D_oe psi_e */
    zero_parity(L, t2, 0);
    oracle_hopping(L, anti, U, (double *)t2, (double *)t1, dag); /* even part = D_eo D_oe psi_e */
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    const double a = 1.0 / (2.0 * kappa);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < V; n++) {
        int even = oracle_parity(L, n) == 0;
        for (int k = 0; k < 12; k++)
            out[n * 12 + k] = even ? a * a * in[n * 12 + k] - 0.25 * t1[n * 12 + k] : 0;
    }
    free(t1);
    free(t2);
}

/* b_prec = (1/(2 kappa)) b_e + 1/2 D_eo b_o, stored on even sites (eq. eo2/eo4) */
void oracle_eo_source(const int *L, int anti, const double *U, double kappa, const double *bd, double *outd)
{
    const long V = vol(L), N = V * 12;
    cplx *bo = malloc(sizeof(cplx) * N), *h = malloc(sizeof(cplx) * N);
    memcpy(bo, bd, sizeof(cplx) * N);
    zero_parity(L, bo, 0);
    oracle_hopping(L, anti, U, (double *)bo, (double *)h, 0);
    const cplx *b = (const cplx *)bd;
    cplx *out = (cplx *)outd;
    const double a = 1.0 / (2.0 * kappa);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < V; n++) {
        int even = oracle_parity(L, n) == 0;
        for (int k = 0; k < 12; k++) out[n * 12 + k] = even ? a * b[n * 12 + k] + 0.5 * h[n * 12 + k] : 0;
    }
    free(bo);
    free(h);
}

/* Given psi_e (even sites of x), fill the odd sites: psi_o = 2 kappa (b_o + 1/2 D_oe psi_e)  (eq. eo3) */
void oracle_eo_reconstruct(const int *L, int anti, const double *U, double kappa, const double *bd, double *xd)
{
    const long V = vol(L), N = V * 12;
    cplx *xe = malloc(sizeof(cplx) * N), *h = malloc(sizeof(cplx) * N);
    memcpy(xe, xd, sizeof(cplx) * N);
    zero_parity(L, xe, 1);
    oracle_hopping(L, anti, U, (double *)xe, (double *)h, 0);
    const cplx *b = (const cplx *)bd;
    cplx *x = (cplx *)xd;
    const double a = 1.0 / (2.0 * kappa);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < V; n++)
        if (oracle_parity(L, n) == 1)
            for (int k = 0; k < 12; k++) x[n * 12 + k] = (b[n * 12 + k] + 0.5 * h[n * 12 + k]) / a;
    free(xe);
    free(h);
}

/* ---------------------------------------------------------------- BLAS-1 (plain loops) */

static cplx vdot(long n, const cplx *a, const cplx *b)
{
    double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (long i = 0; i < n; i++) {
        cplx v = conj(a[i]) * b[i];
        re += creal(v);
        im += cimag(v);
    }
    return re + I * im;
}

static double vnorm2(long n, const cplx *a)
{
    double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (long i = 0; i < n; i++) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

/* ---------------------------------------------------------------- BiCGstab */

typedef struct {
    const int *L;
    int anti;
    const double *U;
    double kappa;
    int prec; /* 0: full M, 1: even-odd M_prec */
} opctx;

static void op_apply(const opctx *c, const cplx *in, cplx *out)
{
    if (c->prec) oracle_mprec(c->L, c->anti, c->U, c->kappa, (const double *)in, (double *)out, 0);
    else oracle_apply(c->L, c->anti, c->U, c->kappa, (const double *)in, (double *)out, 0);
}

enum { OR_OK = 0, OR_NOCONV = 4, OR_BREAKDOWN = 5 };

/*
 * BiCGstab (van der Vorst, as cited in Sec. 6), in the notation that makes the solution update
 * read x <- x - beta s + chi w (Sec. 5):
 *   r = b - A x0, rhat = r, s = r, delta = <rhat, r>
 *   repeat: beta = -delta / <rhat, A s>;  w = r + beta A s;  chi = <A w, w> / <A w, A w>
 *           x <- x - beta s + chi w;  r <- w - chi A w;  delta' = <rhat, r>
 *           alpha = -beta delta' / (delta chi);  s <- r + alpha (s - chi A s)
 *   until |r| < tol |b|                                                   (Sec. 6.1)
 * `hist` (may be NULL) receives |r|/|b| after each iteration.
 */
static int bicgstab_core(const opctx *c, long N, const cplx *b, cplx *x, double tol, int maxit, int *iters,
                         double *hist)
{
    cplx *r = malloc(sizeof(cplx) * N), *rh = malloc(sizeof(cplx) * N), *s = malloc(sizeof(cplx) * N);
    cplx *As = malloc(sizeof(cplx) * N), *w = malloc(sizeof(cplx) * N), *Aw = malloc(sizeof(cplx) * N);
    op_apply(c, x, As);
    for (long i = 0; i < N; i++) r[i] = b[i] - As[i];
    memcpy(rh, r, sizeof(cplx) * N);
    memcpy(s, r, sizeof(cplx) * N);
    const double bn = sqrt(vnorm2(N, b));
    cplx delta = vdot(N, rh, r);
    int status = OR_NOCONV, it = 0;
    if (sqrt(vnorm2(N, r)) < tol * bn) status = OR_OK;
    while (status == OR_NOCONV && it < maxit) {
        op_apply(c, s, As);
        cplx rhAs = vdot(N, rh, As);
        if (cabs(rhAs) == 0.0) { status = OR_BREAKDOWN; break; }
        cplx beta = -delta / rhAs;
        for (long i = 0; i < N; i++) w[i] = r[i] + beta * As[i];
        op_apply(c, w, Aw);
        double AwAw = vnorm2(N, Aw);
        if (AwAw == 0.0) { status = OR_BREAKDOWN; break; }
        cplx chi = vdot(N, Aw, w) / AwAw;
        for (long i = 0; i < N; i++) {
            x[i] = x[i] - beta * s[i] + chi * w[i];
            r[i] = w[i] - chi * Aw[i];
        }
        cplx delta1 = vdot(N, rh, r);
        it++;
        double rn = sqrt(vnorm2(N, r));
        if (hist) hist[it - 1] = rn / bn;
        if (rn < tol * bn) { status = OR_OK; break; }
        if (cabs(delta1) == 0.0 || cabs(chi) == 0.0) { status = OR_BREAKDOWN; break; }
        cplx alpha = -beta * delta1 / (delta * chi);
        for (long i = 0; i < N; i++) s[i] = r[i] + alpha * (s[i] - chi * As[i]);
        delta = delta1;
    }
    *iters = it;
    free(r); free(rh); free(s); free(As); free(w); free(Aw);
    return status;
}

/* Full-lattice BiCGstab for M(kappa) x = b. x holds the start vector when use_x0 != 0. */
int oracle_bicgstab(const int *L, int anti, const double *U, double kappa, const double *b, double *x, double tol,
                    int maxit, int use_x0, int *iters, double *hist)
{
    opctx c = {L, anti, U, kappa, 0};
    const long N = vol(L) * 12;
    if (!use_x0) memset(x, 0, sizeof(cplx) * N);
    return bicgstab_core(&c, N, (const cplx *)b, (cplx *)x, tol, maxit, iters, hist);
}

/*
 * Even-odd preconditioned BiCGstab (Sec. 6.2.3): solve M_prec psi_e = b_prec, then rebuild
 * psi_o from eq. eo3. The stopping test |b_prec - M_prec psi_e| < tol (1/(2 kappa)) |b|
 * equals |b - M psi| < tol |b| in exact arithmetic, since the odd residual vanishes and the
 * even residual of the full system is 2 kappa times the preconditioned one.
 * With use_x0 the even sites of x hold the start vector psi_e.
 */
int oracle_bicgstab_eo(const int *L, int anti, const double *U, double kappa, const double *bd, double *xd,
                       double tol, int maxit, int use_x0, int *iters, double *hist)
{
    opctx c = {L, anti, U, kappa, 1};
    const long N = vol(L) * 12;
    cplx *bp = malloc(sizeof(cplx) * N);
    oracle_eo_source(L, anti, U, kappa, bd, (double *)bp);
    cplx *x = (cplx *)xd;
    if (!use_x0) memset(x, 0, sizeof(cplx) * N);
    zero_parity(L, x, 1);
    /* rescale the tolerance: |b_prec| differs from (1/(2 kappa))|b| */
    const double a = 1.0 / (2.0 * kappa);
    const double bn = sqrt(vnorm2(N, (const cplx *)bd)), bpn = sqrt(vnorm2(N, bp));
    double tol_prec = tol * a * bn / bpn;
    int st = bicgstab_core(&c, N, bp, x, tol_prec, maxit, iters, hist);
    if (hist)
        for (int i = 0; i < *iters; i++) hist[i] *= bpn / (a * bn);
    oracle_eo_reconstruct(L, anti, U, kappa, bd, xd);
    free(bp);
    return st;
}

/*
 * BiCGstab-M (multi-shift BiCGstab, Jegerlehner; Sec. 6.1) for M(kappa_i) x_i = b.
 * The unshifted matrix A = M(kappa_base) is the most singular one (largest kappa, smallest
 * mass); shifts sigma_i = 1/(2 kappa_i) - 1/(2 kappa_base) >= 0 give M(kappa_i) = A + sigma_i.
 * The shifted iterates follow from the collinearity of the shifted residuals,
 * r^sigma_n = zeta^sigma_n rho^sigma_n r_n, with zero start vectors:
 *   zeta_{n+1} = zeta_n zeta_{n-1} beta_{n-1} /
 *                [beta_n alpha_n (zeta_{n-1} - zeta_n) + zeta_{n-1} beta_{n-1} (1 - sigma beta_n)]
 *   beta^s_n = beta_n zeta_{n+1}/zeta_n,  chi^s = chi/(1 + chi sigma),  rho_{n+1} = rho_n/(1 + chi sigma)
 *   x^s <- x^s - beta^s s^s + chi^s rho_n zeta_{n+1} w
 *   alpha^s_{n+1} = alpha_{n+1} zeta_{n+1} beta^s_n / (zeta_n beta_n)
 *   s^s <- zeta_{n+1} rho_{n+1} r_{n+1} + alpha^s_{n+1} (s^s - (chi^s/beta^s_n) rho_n (zeta_{n+1} w - zeta_n r_n))
 * A shift stops being updated once |zeta rho| |r| < tol |b| (Sec. 6.1); the run ends when
 * the unshifted residual satisfies |r| < tol |b|.
 * xs: nk full-length fields (caller's order of kappas). conv_iter[i] receives the iteration at
 * which system i was frozen (the base system: the final iteration).
 */
int oracle_bicgstab_m(const int *L, int anti, const double *U, int nk, const double *kappas, const double *bd,
                      double *xsd, double tol, int maxit, int *iters, int *conv_iter)
{
    const long N = vol(L) * 12;
    if (nk < 1 || nk > 64) return -1;
    int base = 0;
    for (int i = 1; i < nk; i++)
        if (kappas[i] > kappas[base]) base = i;
    opctx c = {L, anti, U, kappas[base], 0};
    const cplx *b = (const cplx *)bd;
    cplx *xs = (cplx *)xsd;
    cplx *r = malloc(sizeof(cplx) * N), *rold = malloc(sizeof(cplx) * N), *s = malloc(sizeof(cplx) * N);
    cplx *As = malloc(sizeof(cplx) * N), *w = malloc(sizeof(cplx) * N), *Aw = malloc(sizeof(cplx) * N);
    cplx *ss = malloc(sizeof(cplx) * N * nk);
    double *sigma = malloc(sizeof(double) * nk);
    cplx *zeta = malloc(sizeof(cplx) * nk), *zeta_prev = malloc(sizeof(cplx) * nk), *rho = malloc(sizeof(cplx) * nk);
    int *active = malloc(sizeof(int) * nk);
    for (int i = 0; i < nk; i++) {
        sigma[i] = 1.0 / (2.0 * kappas[i]) - 1.0 / (2.0 * kappas[base]);
        zeta[i] = zeta_prev[i] = rho[i] = 1.0;
        active[i] = (i != base);
        conv_iter[i] = 0;
        memset(xs + i * N, 0, sizeof(cplx) * N);
        memcpy(ss + i * N, b, sizeof(cplx) * N);
    }
    cplx *x = xs + base * N;
    memcpy(r, b, sizeof(cplx) * N);
    memcpy(s, b, sizeof(cplx) * N);
    const cplx *rh = b;
    const double bn = sqrt(vnorm2(N, b));
    cplx delta = vdot(N, rh, r);
    cplx beta_prev = 1.0, alpha = 0.0;
    int status = OR_NOCONV, it = 0;
    while (it < maxit) {
        op_apply(&c, s, As);
        cplx rhAs = vdot(N, rh, As);
        if (cabs(rhAs) == 0.0) { status = OR_BREAKDOWN; break; }
        cplx beta = -delta / rhAs;
        cplx zn[64], bs[64];
        for (int i = 0; i < nk; i++) {
            if (!active[i]) continue;
            cplx den = beta * alpha * (zeta_prev[i] - zeta[i]) + zeta_prev[i] * beta_prev * (1.0 - sigma[i] * beta);
            zn[i] = zeta[i] * zeta_prev[i] * beta_prev / den;
            bs[i] = beta * zn[i] / zeta[i];
        }
        for (long k = 0; k < N; k++) w[k] = r[k] + beta * As[k];
        op_apply(&c, w, Aw);
        double AwAw = vnorm2(N, Aw);
        if (AwAw == 0.0) { status = OR_BREAKDOWN; break; }
        cplx chi = vdot(N, Aw, w) / AwAw;
        memcpy(rold, r, sizeof(cplx) * N);
        for (long k = 0; k < N; k++) {
            x[k] = x[k] - beta * s[k] + chi * w[k];
            r[k] = w[k] - chi * Aw[k];
        }
        cplx delta1 = vdot(N, rh, r);
        cplx alpha1 = -beta * delta1 / (delta * chi);
        it++;
        double rn = sqrt(vnorm2(N, r));
        for (int i = 0; i < nk; i++) {
            if (!active[i]) continue;
            cplx cs = chi / (1.0 + chi * sigma[i]);
            cplx rho1 = rho[i] / (1.0 + chi * sigma[i]);
            cplx as = alpha1 * zn[i] * bs[i] / (zeta[i] * beta);
            cplx *xi = xs + i * N, *si = ss + i * N;
            for (long k = 0; k < N; k++) {
                xi[k] = xi[k] - bs[i] * si[k] + cs * rho[i] * zn[i] * w[k];
                si[k] = zn[i] * rho1 * r[k] + as * (si[k] - (cs / bs[i]) * rho[i] * (zn[i] * w[k] - zeta[i] * rold[k]));
            }
            zeta_prev[i] = zeta[i];
            zeta[i] = zn[i];
            rho[i] = rho1;
            if (cabs(zeta[i] * rho[i]) * rn < tol * bn) {
                active[i] = 0;
                conv_iter[i] = it;
            }
        }
        if (rn < tol * bn) { status = OR_OK; break; }
        if (cabs(delta1) == 0.0 || cabs(chi) == 0.0) { status = OR_BREAKDOWN; break; }
        for (long k = 0; k < N; k++) s[k] = r[k] + alpha1 * (s[k] - chi * As[k]);
        beta_prev = beta;
        alpha = alpha1;
        delta = delta1;
    }
    conv_iter[base] = it;
    for (int i = 0; i < nk; i++)
        if (active[i]) conv_iter[i] = it;
    *iters = it;
    free(r); free(rold); free(s); free(As); free(w); free(Aw); free(ss);
    free(sigma); free(zeta); free(zeta_prev); free(rho); free(active);
    return status;
}

/* ---------------------------------------------------------------- link gradient */

/*
 * For L = Re <eta, M^{-1} b> with x = M^{-1} b and lam = M^{-dag} eta, the derivative with
 * respect to the complex link U_mu(n) (d/dRe + i d/dIm) is
 *   G_mu(n) = 1/2 s [ lam_n (1 - gamma_mu) x_{n+mu}^dag + x_n (1 + gamma_mu) lam_{n+mu}^dag ]
 * (3x3, summed over spin), obtained by differentiating eq. 3/4 in U. s is the boundary sign.
 * G[mu][n][a][b], interleaved complex.
 */
void oracle_gauge_grad(const int *L, int anti, const double *xd, const double *lamd, double *Gd)
{
    build_gammas();
    const cplx *x = (const cplx *)xd, *lam = (const cplx *)lamd;
    cplx *G = (cplx *)Gd;
    const long V = vol(L);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < V; n++) {
        int c[4];
        coords(L, n, c);
        for (int mu = 0; mu < 4; mu++) {
            long m = neighbour(L, c, mu, +1);
            double sgn = (anti && mu == 3 && c[3] == L[3] - 1) ? -1.0 : 1.0;
            /* A = lam_n (1 - gamma), B = x_n (1 + gamma)  (3x4 each) */
            cplx A[3][4], B[3][4];
            for (int a = 0; a < 3; a++)
                for (int s = 0; s < 4; s++) {
                    cplx va = 0, vb = 0;
                    for (int r = 0; r < 4; r++) {
                        va += lam[n * 12 + a * 4 + r] * PMINUS[mu][r][s];
                        vb += x[n * 12 + a * 4 + r] * PPLUS[mu][r][s];
                    }
                    A[a][s] = va;
                    B[a][s] = vb;
                }
            for (int a = 0; a < 3; a++)
                for (int bb = 0; bb < 3; bb++) {
                    cplx g = 0;
                    for (int s = 0; s < 4; s++)
                        g += A[a][s] * conj(x[m * 12 + bb * 4 + s]) + B[a][s] * conj(lam[m * 12 + bb * 4 + s]);
                    G[((long)mu * V + n) * 9 + a * 3 + bb] = 0.5 * sgn * g;
                }
        }
    }
}

/* ---------------------------------------------------------------- misc */

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
