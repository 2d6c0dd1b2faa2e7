/*
 * ferro_oracle.c -- plain FP64 CPU oracle of the TDGL + Poisson time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the HIP library.
 *
 * What it computes (FerroX, arXiv 2210.15668, Methods):
 *   - the polarisation update of eq. (TDGL2) with the Landau energy of
 *     eq. (free), the gradient energy of eq. (grad), the boundary conditions
 *     of eqs. (Pbc), (PbcFree), (PbcDir) and the forward-Euler Step 1a of the
 *     numerical scheme;
 *   - the potential from eq. (Poisson) with spatially varying permittivity,
 *     Dirichlet contacts on the z-ends and periodic x/y (section "Electrical
 *     boundary conditions"), and the semiconductor charge of eq. (rho) with
 *     the Maxwell-Boltzmann carrier densities of eq. (MaxBolt_ne_np);
 *   - Step 0 (phi initialised to zero) and Step 1b (warm start from phi^n),
 *     each solved to the unique root of the discrete nonlinear system.
 *
 * The paper's own solver is a lagged-charge fixed point with an AMReX
 * multigrid inner solve.  Both that and this code converge to the same root
 * of the same discrete equations; here the root is found by damped Newton
 * with a Jacobi-preconditioned conjugate-gradient inner solve, which is slow
 * but easy to check by eye.
 *
 * Discrete definition (cell-centred, spacing h, cell (i,j,k) centred at
 * ((i+1/2)h, (j+1/2)h, (k+1/2)h), index (k*ny + j)*nx + i):
 *
 *  Planes.  Each z-plane k has a material (metal, ferroelectric,
 *  dielectric, semiconductor) and a relative permittivity.  Metal planes
 *  are contiguous runs at the two ends; the remaining planes [kb, kt) are
 *  the device.  phi = v_bottom on the device's bottom face and v_top on its
 *  top face; metal cells hold their contact value.
 *
 *  Poisson, finite-volume form of div(eps grad phi - P z) = -rho:
 *    z-face between planes L (below) and R (above):
 *      eps_f = 2 eps_L eps_R / (eps_L + eps_R),
 *      P_f   = (eps_R P_L + eps_L P_R) / (eps_L + eps_R),
 *    both from continuity of D_z = -eps dphi/dz + P across two half-cells of
 *    constant eps and P.  A contact face uses the cell's own eps at distance
 *    h/2 and P_f = P of the cell.  x/y faces use the plane's eps.
 *    With L phi = sum_faces eps_f (phi - phi_nb)/dist/h (Dirichlet
 *    neighbours contribute through the right-hand side), the cell equation is
 *      N(phi) = L phi - rho_c(phi) = f,
 *      f = [contact terms 2 eps V / h^2] - (P_{k+1/2} - P_{k-1/2}) / h,
 *    rho_c = e [p0 expm1(-phi/VT) - n0 expm1(phi/VT)] on semiconductor
 *    planes, p0 and n0 the neutral-bulk densities of the plane's doping
 *    (p0 - n0 + Nd - Na = 0, p0 n0 = ni^2), so phi = 0 is charge neutral.
 *    The Newton Jacobian is L + diag(sigma), sigma = e (p + n) / VT > 0.
 *
 *  TDGL, eq. (TDGL2), Step 1a:
 *    P' = P - dt Gamma [alpha P + beta P^3 + gamma P^5
 *                       - g44 (Dxx + Dyy) P - g11 Dzz P + Dz phi]
 *    Dxx, Dyy: periodic 3-point.  Dzz: 3-point inside the ferroelectric; on
 *    its two boundary planes the one-sided three-point stencil through the
 *    surface value P_s (at distance h/2 outside), the boundary cell P_0 and
 *    the next cell inward P_1:  Dzz = 4 (2 P_s - 3 P_0 + P_1) / (3 h^2), with
 *    P_s from the surface condition lambda dP/dn + P = 0 (outward normal n)
 *    applied to the same quadratic:
 *      free   (lambda -> inf): P_s = (9 P_0 - P_1) / 8
 *      zero   (lambda = 0)   : P_s = 0
 *      lambda               : P_s = lambda (9 P_0 - P_1) / (8 lambda + 3 h).
 *    Dz phi: central difference inside the ferroelectric; on its boundary
 *    planes the one-sided three-point stencil over ferroelectric cells only.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>

#define Q_E   1.602176634e-19
#define K_B   1.380649e-23
#define EPS0  8.8541878128e-12
#define HBAR  1.054571817e-34
#define M_E0  9.1093837015e-31
#define PI    3.14159265358979323846

enum { MAT_METAL = 0, MAT_FE = 1, MAT_DE = 2, MAT_SC = 3 };
enum { BC_FREE = 0, BC_ZERO = 1, BC_LAMBDA = 2 };
enum { CARRIERS_BOLTZMANN = 0, CARRIERS_FD = 1 };

typedef struct {
    int nx, ny, nz;
    double h;
    const int *mat;
    const double *eps_r, *Na, *Nd;
    double alpha, beta, gamma, g11, g44, Gamma;
    int pbc;
    double lambda;
    double ni, T;
    double v_bottom, v_top;
    int carriers;        /* CARRIERS_BOLTZMANN (densities from ni) or CARRIERS_FD */
    double me, mp;       /* effective masses / free-electron mass (Fermi-Dirac only) */
    double Eg;           /* band gap [eV] (Fermi-Dirac only) */
} orc_desc;

typedef struct {
    int newton_iters;
    int cg_iters;
    double res_norm;
    double rhs_norm;
    int status;          /* 0 ok, 1 not converged, 2 invalid */
} orc_info;

/* ---------------------------------------------------------------- layout */

static int find_layout(const orc_desc *d, int *kb, int *kt, int *f0, int *f1)
{
    int k;
    *kb = -1; *kt = -1; *f0 = -1; *f1 = -1;
    for (k = 0; k < d->nz; k++)
        if (d->mat[k] != MAT_METAL) { if (*kb < 0) *kb = k; *kt = k + 1; }
    if (*kb < 0) return -1;
    for (k = *kb; k < *kt; k++) if (d->mat[k] == MAT_METAL) return -1;
    for (k = 0; k < d->nz; k++)
        if (d->mat[k] == MAT_FE) { if (*f0 < 0) *f0 = k; *f1 = k + 1; }
    if (*f0 >= 0) {
        for (k = *f0; k < *f1; k++) if (d->mat[k] != MAT_FE) return -1;
        if (*f1 - *f0 < 3) return -1;
    }
    return 0;
}

#define IDX(d, i, j, k) (((size_t)(k) * (d)->ny + (j)) * (d)->nx + (i))
#define XP(d, i) ((i) + 1 == (d)->nx ? 0 : (i) + 1)
#define XM(d, i) ((i) == 0 ? (d)->nx - 1 : (i) - 1)
#define YP(d, j) ((j) + 1 == (d)->ny ? 0 : (j) + 1)
#define YM(d, j) ((j) == 0 ? (d)->ny - 1 : (j) - 1)

/* ---------------------------------------------------------------- TDGL */

static double surface_value(const orc_desc *d, double P0, double P1)
{
    if (d->pbc == BC_FREE) return (9.0 * P0 - P1) / 8.0;
    if (d->pbc == BC_ZERO) return 0.0;
    return d->lambda * (9.0 * P0 - P1) / (8.0 * d->lambda + 3.0 * d->h);
}

/* f(P, phi) of eq. (TDGL_simp) on ferroelectric cells, zero elsewhere. */
int orc_tdgl_rhs(const orc_desc *d, const double *P, const double *phi, double *out)
{
    int kb, kt, f0, f1;
    if (find_layout(d, &kb, &kt, &f0, &f1)) return 2;
    const double h = d->h, h2 = h * h;
    memset(out, 0, sizeof(double) * (size_t)d->nx * d->ny * d->nz);
    if (f0 < 0) return 0;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = f0; k < f1; k++)
        for (int j = 0; j < d->ny; j++)
            for (int i = 0; i < d->nx; i++) {
                const double p = P[IDX(d, i, j, k)];
                const double dxx = (P[IDX(d, XP(d, i), j, k)] - 2.0 * p + P[IDX(d, XM(d, i), j, k)]) / h2;
                const double dyy = (P[IDX(d, i, YP(d, j), k)] - 2.0 * p + P[IDX(d, i, YM(d, j), k)]) / h2;
                double dzz, dzphi;
                if (k == f0) {
                    const double p1 = P[IDX(d, i, j, k + 1)];
                    dzz = 4.0 * (2.0 * surface_value(d, p, p1) - 3.0 * p + p1) / (3.0 * h2);
                    dzphi = (-3.0 * phi[IDX(d, i, j, k)] + 4.0 * phi[IDX(d, i, j, k + 1)]
                             - phi[IDX(d, i, j, k + 2)]) / (2.0 * h);
                } else if (k == f1 - 1) {
                    const double p1 = P[IDX(d, i, j, k - 1)];
                    dzz = 4.0 * (2.0 * surface_value(d, p, p1) - 3.0 * p + p1) / (3.0 * h2);
                    dzphi = (3.0 * phi[IDX(d, i, j, k)] - 4.0 * phi[IDX(d, i, j, k - 1)]
                             + phi[IDX(d, i, j, k - 2)]) / (2.0 * h);
                } else {
                    dzz = (P[IDX(d, i, j, k + 1)] - 2.0 * p + P[IDX(d, i, j, k - 1)]) / h2;
                    dzphi = (phi[IDX(d, i, j, k + 1)] - phi[IDX(d, i, j, k - 1)]) / (2.0 * h);
                }
                const double p2 = p * p;
                const double landau = d->alpha * p + d->beta * p2 * p + d->gamma * p2 * p2 * p;
                const double dF = landau - d->g44 * (dxx + dyy) - d->g11 * dzz + dzphi;
                out[IDX(d, i, j, k)] = -d->Gamma * dF;
            }
    return 0;
}

/* Step 1a: P_out = P + dt f(P, phi).  P_out must not alias P. */
int orc_tdgl_step(const orc_desc *d, const double *P, const double *phi, double dt, double *Pout)
{
    size_t n = (size_t)d->nx * d->ny * d->nz;
    int s = orc_tdgl_rhs(d, P, phi, Pout);
    if (s) return s;
    for (size_t c = 0; c < n; c++) Pout[c] = P[c] + dt * Pout[c];
    return 0;
}

/* ---------------------------------------------------------------- Poisson */

typedef struct {
    int kb, kt;
    double *eps;      /* nz, absolute permittivity */
    double *cxy;      /* per plane: eps_k / h^2 */
    double *czm, *czp;/* per plane: face coefficient / h^2 (contact faces 2 eps / h^2) */
    double *p0, *n0;  /* per plane neutral-bulk densities (semiconductor planes) */
    double *etn, *etp;/* Fermi-Dirac: (E_F - E_c)/kT and (E_v - E_F)/kT at phi = 0 */
    double Nc, Nv;    /* Fermi-Dirac: effective densities of states */
    double VT;
} orc_tables;

/*
 * Fermi-Dirac integral of order 1/2 in the normalisation that tends to e^eta
 * for eta -> -inf: F(eta) = (2/sqrt(pi)) int_0^inf sqrt(x) / (1 + e^(x - eta)) dx.
 * Then eq. (ne) reads n_e = Nc F((E_F - E_c)/kT) with Nc = 2 (m kT / (2 pi hbar^2))^(3/2),
 * and eq. (np) likewise for holes.  As the paper does (Methods, Poisson solve),
 * F is taken from the closed-form approximation of Bednarczyk and Bednarczyk
 * (1978):  F(eta) = 1 / (e^-eta + xi),  xi = (3 sqrt(pi) / 4) nu^(-3/8),
 * nu = eta^4 + 50 + 33.6 eta (1 - 0.68 exp(-0.17 (eta + 1)^2)).
 * dF is the derivative of that expression, so that the Newton Jacobian is the
 * derivative of the charge actually used.
 */
void orc_fd_half(double eta, double *F, double *dF)
{
    const double a = eta + 1.0;
    const double g = exp(-0.17 * a * a);
    const double s = 1.0 - 0.68 * g;
    const double nu = pow(eta, 4.0) + 50.0 + 33.6 * eta * s;
    const double dnu = 4.0 * pow(eta, 3.0) + 33.6 * s + 33.6 * eta * 0.68 * 0.34 * a * g;
    const double xi = 0.75 * sqrt(PI) * pow(nu, -0.375);
    const double dxi = -0.375 * xi * dnu / nu;
    const double em = exp(-eta);
    const double D = em + xi;
    *F = 1.0 / D;
    *dF = (em - dxi) / (D * D);
}

static double fd_F(double eta)
{
    double F, dF;
    orc_fd_half(eta, &F, &dF);
    return F;
}

/* Fermi-Dirac neutrality at phi = 0: the x = (E_F - E_c)/kT with
 * Nv F(-x - Eg/kT) - Nc F(x) + Nd - Na = 0 (eq. rho with no field), by
 * bisection (the left side falls monotonically in x). */
static double fd_neutral_eta(double Nc, double Nv, double egkt, double Na, double Nd)
{
    double lo = -egkt - 100.0, hi = 100.0;
    for (int it = 0; it < 400; it++) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        const double g = Nv * fd_F(-mid - egkt) - Nc * fd_F(mid) + Nd - Na;
        if (g > 0.0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

static void neutral_densities(double Na, double Nd, double ni, double *p0, double *n0)
{
    const double net = Nd - Na;
    if (net >= 0.0) {
        *n0 = 0.5 * net + sqrt(0.25 * net * net + ni * ni);
        *p0 = ni * ni / *n0;
    } else {
        *p0 = -0.5 * net + sqrt(0.25 * net * net + ni * ni);
        *n0 = ni * ni / *p0;
    }
}

static int build_tables(const orc_desc *d, orc_tables *t)
{
    int f0, f1;
    if (find_layout(d, &t->kb, &t->kt, &f0, &f1)) return 2;
    int nz = d->nz;
    t->eps = calloc(nz, sizeof(double)); t->cxy = calloc(nz, sizeof(double));
    t->czm = calloc(nz, sizeof(double)); t->czp = calloc(nz, sizeof(double));
    t->p0 = calloc(nz, sizeof(double));  t->n0 = calloc(nz, sizeof(double));
    t->etn = calloc(nz, sizeof(double)); t->etp = calloc(nz, sizeof(double));
    const double h2 = d->h * d->h;
    t->VT = K_B * d->T / Q_E;
    const double kT = K_B * d->T;
    t->Nc = 2.0 * pow(d->me * M_E0 * kT / (2.0 * PI * HBAR * HBAR), 1.5);
    t->Nv = 2.0 * pow(d->mp * M_E0 * kT / (2.0 * PI * HBAR * HBAR), 1.5);
    for (int k = 0; k < nz; k++) t->eps[k] = EPS0 * d->eps_r[k];
    for (int k = t->kb; k < t->kt; k++) {
        t->cxy[k] = t->eps[k] / h2;
        if (k == t->kb) t->czm[k] = 2.0 * t->eps[k] / h2;
        else t->czm[k] = 2.0 * t->eps[k - 1] * t->eps[k] / (t->eps[k - 1] + t->eps[k]) / h2;
        if (k == t->kt - 1) t->czp[k] = 2.0 * t->eps[k] / h2;
        else t->czp[k] = 2.0 * t->eps[k] * t->eps[k + 1] / (t->eps[k] + t->eps[k + 1]) / h2;
        if (d->mat[k] == MAT_SC && d->carriers == CARRIERS_FD) {
            const double egkt = d->Eg / t->VT;
            t->etn[k] = fd_neutral_eta(t->Nc, t->Nv, egkt, d->Na[k], d->Nd[k]);
            t->etp[k] = -t->etn[k] - egkt;
        } else if (d->mat[k] == MAT_SC) {
            neutral_densities(d->Na[k], d->Nd[k], d->ni, &t->p0[k], &t->n0[k]);
        }
    }
    return 0;
}

static void free_tables(orc_tables *t)
{
    free(t->eps); free(t->cxy); free(t->czm); free(t->czp); free(t->p0); free(t->n0);
    free(t->etn); free(t->etp);
}

/* Face value of P between planes k (below) and k+1 (above) at (i,j). */
static double face_P_up(const orc_desc *d, const orc_tables *t, const double *P, int i, int j, int k)
{
    if (k == t->kt - 1) return P[IDX(d, i, j, k)];
    const double eL = t->eps[k], eR = t->eps[k + 1];
    return (eR * P[IDX(d, i, j, k)] + eL * P[IDX(d, i, j, k + 1)]) / (eL + eR);
}

static double face_P_down(const orc_desc *d, const orc_tables *t, const double *P, int i, int j, int k)
{
    if (k == t->kb) return P[IDX(d, i, j, k)];
    return face_P_up(d, t, P, i, j, k - 1);
}

static void compute_f(const orc_desc *d, const orc_tables *t, const double *P, double *f)
{
    memset(f, 0, sizeof(double) * (size_t)d->nx * d->ny * d->nz);
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = t->kb; k < t->kt; k++)
        for (int j = 0; j < d->ny; j++)
            for (int i = 0; i < d->nx; i++) {
                double v = 0.0;
                if (k == t->kb) v += t->czm[k] * d->v_bottom;
                if (k == t->kt - 1) v += t->czp[k] * d->v_top;
                v -= (face_P_up(d, t, P, i, j, k) - face_P_down(d, t, P, i, j, k)) / d->h;
                f[IDX(d, i, j, k)] = v;
            }
}

/* rho_c(phi) and sigma = -d rho_c / d phi at one cell of plane k. */
static void carriers(const orc_desc *d, const orc_tables *t, int k, double phi, double *rho, double *sig)
{
    if (d->mat[k] != MAT_SC) { *rho = 0.0; *sig = 0.0; return; }
    const double u = phi / t->VT;
    if (d->carriers == CARRIERS_FD) {
        /* eq. (rho) with n_e = Nc F(eta_n), n_p = Nv F(eta_p); the potential
         * lowers the conduction band by e phi: eta_n = eta_n0 + u, eta_p = eta_p0 - u */
        double Fn, dFn, Fp, dFp;
        orc_fd_half(t->etn[k] + u, &Fn, &dFn);
        orc_fd_half(t->etp[k] - u, &Fp, &dFp);
        *rho = Q_E * (t->Nv * Fp - t->Nc * Fn + d->Nd[k] - d->Na[k]);
        *sig = Q_E * (t->Nv * dFp + t->Nc * dFn) / t->VT;
        return;
    }
    *rho = Q_E * (t->p0[k] * expm1(-u) - t->n0[k] * expm1(u));
    *sig = Q_E * (t->p0[k] * exp(-u) + t->n0[k] * exp(u)) / t->VT;
}

/* Neutral-bulk carrier densities of plane k as the oracle uses them (for tests). */
int orc_plane_densities(const orc_desc *d, int k, double *p0, double *n0)
{
    orc_tables t;
    if (build_tables(d, &t)) return 2;
    if (k < 0 || k >= d->nz || d->mat[k] != MAT_SC) { free_tables(&t); return 2; }
    if (d->carriers == CARRIERS_FD) {
        *p0 = t.Nv * fd_F(t.etp[k]);
        *n0 = t.Nc * fd_F(t.etn[k]);
    } else {
        *p0 = t.p0[k];
        *n0 = t.n0[k];
    }
    free_tables(&t);
    return 0;
}

/* out = N(phi) = L phi - rho_c(phi) on device cells (Dirichlet neighbours zero). */
static void apply_N(const orc_desc *d, const orc_tables *t, const double *phi, double *out)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = t->kb; k < t->kt; k++)
        for (int j = 0; j < d->ny; j++)
            for (int i = 0; i < d->nx; i++) {
                const double c = phi[IDX(d, i, j, k)];
                double v = t->cxy[k] * (4.0 * c - phi[IDX(d, XP(d, i), j, k)] - phi[IDX(d, XM(d, i), j, k)]
                                        - phi[IDX(d, i, YP(d, j), k)] - phi[IDX(d, i, YM(d, j), k)]);
                v += t->czm[k] * (c - (k > t->kb ? phi[IDX(d, i, j, k - 1)] : 0.0));
                v += t->czp[k] * (c - (k < t->kt - 1 ? phi[IDX(d, i, j, k + 1)] : 0.0));
                double rho, sig;
                carriers(d, t, k, c, &rho, &sig);
                out[IDX(d, i, j, k)] = v - rho;
            }
}

/* y = (L + diag sigma) x on device cells. */
static void apply_J(const orc_desc *d, const orc_tables *t, const double *sig, const double *x, double *y)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = t->kb; k < t->kt; k++)
        for (int j = 0; j < d->ny; j++)
            for (int i = 0; i < d->nx; i++) {
                const double c = x[IDX(d, i, j, k)];
                double v = t->cxy[k] * (4.0 * c - x[IDX(d, XP(d, i), j, k)] - x[IDX(d, XM(d, i), j, k)]
                                        - x[IDX(d, i, YP(d, j), k)] - x[IDX(d, i, YM(d, j), k)]);
                v += t->czm[k] * (c - (k > t->kb ? x[IDX(d, i, j, k - 1)] : 0.0));
                v += t->czp[k] * (c - (k < t->kt - 1 ? x[IDX(d, i, j, k + 1)] : 0.0));
                y[IDX(d, i, j, k)] = v + sig[IDX(d, i, j, k)] * c;
            }
}

static double dot_dev(const orc_desc *d, const orc_tables *t, const double *a, const double *b)
{
    double s = 0.0;
    size_t lo = IDX(d, 0, 0, t->kb), hi = IDX(d, 0, 0, t->kt);
#pragma omp parallel for reduction(+:s) schedule(static)
    for (size_t c = lo; c < hi; c++) s += a[c] * b[c];
    return s;
}

/* r = f - N(phi) over device cells; returns ||r||_2. */
static double residual(const orc_desc *d, const orc_tables *t, const double *f, const double *phi, double *r)
{
    size_t lo = IDX(d, 0, 0, t->kb), hi = IDX(d, 0, 0, t->kt);
    apply_N(d, t, phi, r);
#pragma omp parallel for schedule(static)
    for (size_t c = lo; c < hi; c++) r[c] = f[c] - r[c];
    return sqrt(dot_dev(d, t, r, r));
}

/* Jacobi-preconditioned CG for (L + sigma) x = b to ||b - A x|| <= rtol ||b||. */
static int pcg(const orc_desc *d, const orc_tables *t, const double *sig, const double *b, double *x,
               double rtol, int maxit, int *iters)
{
    size_t n = (size_t)d->nx * d->ny * d->nz;
    size_t lo = IDX(d, 0, 0, t->kb), hi = IDX(d, 0, 0, t->kt);
    double *r = calloc(n, sizeof(double)), *z = calloc(n, sizeof(double));
    double *p = calloc(n, sizeof(double)), *q = calloc(n, sizeof(double));
    double *dinv = calloc(n, sizeof(double));
    for (int k = t->kb; k < t->kt; k++)
        for (size_t c = IDX(d, 0, 0, k); c < IDX(d, 0, 0, k + 1); c++)
            dinv[c] = 1.0 / (4.0 * t->cxy[k] + t->czm[k] + t->czp[k] + sig[c]);
    for (size_t c = lo; c < hi; c++) { x[c] = 0.0; r[c] = b[c]; z[c] = dinv[c] * r[c]; p[c] = z[c]; }
    const double bn = sqrt(dot_dev(d, t, b, b));
    double rz = dot_dev(d, t, r, z);
    int it = 0, ok = (bn == 0.0);
    while (!ok && it < maxit) {
        apply_J(d, t, sig, p, q);
        const double a = rz / dot_dev(d, t, p, q);
#pragma omp parallel for schedule(static)
        for (size_t c = lo; c < hi; c++) { x[c] += a * p[c]; r[c] -= a * q[c]; }
        it++;
        if (sqrt(dot_dev(d, t, r, r)) <= rtol * bn) { ok = 1; break; }
#pragma omp parallel for schedule(static)
        for (size_t c = lo; c < hi; c++) z[c] = dinv[c] * r[c];
        const double rz2 = dot_dev(d, t, r, z);
        const double beta = rz2 / rz;
        rz = rz2;
#pragma omp parallel for schedule(static)
        for (size_t c = lo; c < hi; c++) p[c] = z[c] + beta * p[c];
    }
    free(r); free(z); free(p); free(q); free(dinv);
    *iters += it;
    return ok ? 0 : 1;
}

static void set_contacts(const orc_desc *d, const orc_tables *t, double *phi)
{
    for (int k = 0; k < d->nz; k++) {
        if (k >= t->kb && k < t->kt) continue;
        const double v = k < t->kb ? d->v_bottom : d->v_top;
        for (size_t c = IDX(d, 0, 0, k); c < IDX(d, 0, 0, k + 1); c++) phi[c] = v;
    }
}

/*
 * Solve N(phi) = f(P) for phi (in/out, full grid) to ||f - N(phi)|| <= tol ||f||.
 * phi on entry is the starting guess (zero for Step 0, phi^n for Step 1b).
 */
int orc_solve(const orc_desc *d, const double *P, double *phi, double tol, int max_newton, orc_info *info)
{
    orc_tables t;
    memset(info, 0, sizeof(*info));
    if (build_tables(d, &t)) { info->status = 2; return 2; }
    size_t n = (size_t)d->nx * d->ny * d->nz;
    size_t lo = IDX(d, 0, 0, t.kb), hi = IDX(d, 0, 0, t.kt);
    double *f = calloc(n, sizeof(double)), *r = calloc(n, sizeof(double));
    double *sig = calloc(n, sizeof(double)), *dx = calloc(n, sizeof(double));
    double *trial = calloc(n, sizeof(double)), *rt = calloc(n, sizeof(double));
    compute_f(d, &t, P, f);
    set_contacts(d, &t, phi);
    const double fn = sqrt(dot_dev(d, &t, f, f));
    if (fn == 0.0)      /* N(0) = 0 exactly, so the unique root of N(phi) = 0 is phi = 0 */
        for (size_t c = lo; c < hi; c++) phi[c] = 0.0;
    double rn = residual(d, &t, f, phi, r);
    int it = 0, status = 1;
    for (;;) {
        if (rn <= tol * fn || rn == 0.0) { status = 0; break; }
        if (it >= max_newton) break;
        for (int k = t.kb; k < t.kt; k++)
            for (size_t c = IDX(d, 0, 0, k); c < IDX(d, 0, 0, k + 1); c++) {
                double rho;
                carriers(d, &t, k, phi[c], &rho, &sig[c]);
            }
        /* inner solve to a relative tolerance well below the outer target */
        double rtol = 1e-6;
        if (tol * fn / rn * 0.1 > rtol) rtol = tol * fn / rn * 0.1;
        if (rtol > 1e-2) rtol = 1e-2;
        pcg(d, &t, sig, r, dx, rtol, 200000, &info->cg_iters);
        /* backtracking on ||G|| keeps the exponentials in range far from the root */
        double step = 1.0, rnt = 0.0;
        for (int ls = 0; ls < 60; ls++) {
            for (size_t c = 0; c < n; c++) trial[c] = phi[c];
            for (size_t c = lo; c < hi; c++) trial[c] = phi[c] + step * dx[c];
            rnt = residual(d, &t, f, trial, rt);
            if (isfinite(rnt) && rnt < rn) break;
            step *= 0.5;
        }
        if (!(isfinite(rnt) && rnt < rn)) break;
        memcpy(phi, trial, n * sizeof(double));
        memcpy(r, rt, n * sizeof(double));
        rn = rnt;
        it++;
    }
    info->newton_iters = it;
    info->res_norm = rn;
    info->rhs_norm = fn;
    info->status = status;
    free(f); free(r); free(sig); free(dx); free(trial); free(rt);
    free_tables(&t);
    return status;
}

/* Diagnostics used by the tests: the right-hand side f, N(phi), rho_c and sigma. */
int orc_poisson_parts(const orc_desc *d, const double *P, const double *phi,
                      double *f, double *Nphi, double *rho, double *sig)
{
    orc_tables t;
    if (build_tables(d, &t)) return 2;
    size_t n = (size_t)d->nx * d->ny * d->nz;
    if (f) compute_f(d, &t, P, f);
    if (Nphi) { memset(Nphi, 0, n * sizeof(double)); apply_N(d, &t, phi, Nphi); }
    if (rho || sig) {
        for (int k = 0; k < d->nz; k++)
            for (size_t c = IDX(d, 0, 0, k); c < IDX(d, 0, 0, k + 1); c++) {
                double a = 0.0, b = 0.0;
                if (k >= t.kb && k < t.kt) carriers(d, &t, k, phi[c], &a, &b);
                if (rho) rho[c] = a;
                if (sig) sig[c] = b;
            }
    }
    free_tables(&t);
    return 0;
}

/* Relative residual ||f - N(phi)|| / ||f|| of a given phi (norms returned separately). */
int orc_residual_norms(const orc_desc *d, const double *P, const double *phi, double *rnorm, double *fnorm)
{
    orc_tables t;
    if (build_tables(d, &t)) return 2;
    size_t n = (size_t)d->nx * d->ny * d->nz;
    double *f = calloc(n, sizeof(double)), *r = calloc(n, sizeof(double));
    compute_f(d, &t, P, f);
    *rnorm = residual(d, &t, f, phi, r);
    *fnorm = sqrt(dot_dev(d, &t, f, f));
    free(f); free(r);
    free_tables(&t);
    return 0;
}

/*
 * Q and V_fe^avg of the Q-V characteristics (Results, MFIM).
 *
 * z_int is the face between the ferroelectric run and a dielectric plane next
 * to it: the ferroelectric's bottom face if the plane below is dielectric, else
 * its top face if the plane above is.  Across that face, take the lower cell L
 * and the upper cell R, each half cell with constant eps and P (z upward,
 * D_z = -eps dphi/dz + P).  The face potential phi_int and the flux D are the
 * solution of the two half-cell relations
 *     D = -eps_L (phi_int - phi_L) / (h/2) + P_L
 *     D = -eps_R (phi_R - phi_int) / (h/2) + P_R.
 * In the dielectric half cell P = 0, so D = eps0 eps_DE E_z there, the paper's
 * integrand.  Q is the lateral mean of -D: the charge density counted from the
 * gate (top) into the stack, positive for a positive gate over a
 * series capacitor.  V_fe = v_top - (lateral mean of phi_int).
 * Returns 2 if the layout is invalid or the ferroelectric has no dielectric
 * neighbour.
 */
int orc_qv(const orc_desc *d, const double *P, const double *phi, double *Q, double *V_fe)
{
    int kb, kt, f0, f1, kl, kr;
    if (find_layout(d, &kb, &kt, &f0, &f1) || f0 < 0) return 2;
    if (f0 - 1 >= kb && d->mat[f0 - 1] == MAT_DE) { kl = f0 - 1; kr = f0; }
    else if (f1 < kt && d->mat[f1] == MAT_DE) { kl = f1 - 1; kr = f1; }
    else return 2;
    const double eL = EPS0 * d->eps_r[kl], eR = EPS0 * d->eps_r[kr], hh = 0.5 * d->h;
    double sumD = 0.0, sumphi = 0.0;
    for (int j = 0; j < d->ny; j++)
        for (int i = 0; i < d->nx; i++) {
            const double pL = d->mat[kl] == MAT_FE ? P[IDX(d, i, j, kl)] : 0.0;
            const double pR = d->mat[kr] == MAT_FE ? P[IDX(d, i, j, kr)] : 0.0;
            const double phiL = phi[IDX(d, i, j, kl)], phiR = phi[IDX(d, i, j, kr)];
            /* eliminate D: eps_L (phi_int - phi_L) + eps_R (phi_int - phi_R) = (P_L - P_R) h/2 */
            const double phi_int = (eL * phiL + eR * phiR + (pL - pR) * hh) / (eL + eR);
            const double D = -eL * (phi_int - phiL) / hh + pL;
            sumD += D;
            sumphi += phi_int;
        }
    const double area = (double)d->nx * d->ny;
    *Q = -sumD / area;
    *V_fe = d->v_top - sumphi / area;
    return 0;
}

/*
 * Time loop: for n = 0..nsteps-1:  P^{n+1} = P^n + dt f(P^n, phi^n) (Step 1a);
 * phi^{n+1} solved for P^{n+1} with gate v_sched[n] (or d->v_top when NULL),
 * warm-started from phi^n (Step 1b).  P and phi are in/out.
 */
int orc_run(const orc_desc *d_in, double *P, double *phi, int nsteps, double dt,
            const double *v_sched, double tol, int max_newton, orc_info *last)
{
    orc_desc d = *d_in;
    size_t n = (size_t)d.nx * d.ny * d.nz;
    double *Pn = calloc(n, sizeof(double));
    int s = 0;
    for (int step = 0; step < nsteps; step++) {
        s = orc_tdgl_step(&d, P, phi, dt, Pn);
        if (s) break;
        memcpy(P, Pn, n * sizeof(double));
        if (v_sched) d.v_top = v_sched[step];
        s = orc_solve(&d, P, phi, tol, max_newton, last);
        if (s) break;
    }
    free(Pn);
    return s;
}

/*
 * Second-order time loop, the predictor-corrector of the Numerical Approach:
 *   predictor  P* = P^n + dt f(P^n, phi^n)                         (Step 1a)
 *              phi* solved for P*, warm-started from phi^n          (Step 1b)
 *   corrector  P^{n+1} = P^n + dt/2 f(P^n, phi^n) + dt/2 f(P*, phi*) (Step 2a)
 *              phi^{n+1} solved for P^{n+1}, warm-started from phi* (Step 2b)
 * with the gate v_sched[n] (or d->v_top) for both solves of step n.
 */
int orc_run_pc(const orc_desc *d_in, double *P, double *phi, int nsteps, double dt,
               const double *v_sched, double tol, int max_newton, orc_info *last)
{
    orc_desc d = *d_in;
    size_t n = (size_t)d.nx * d.ny * d.nz;
    double *f0 = calloc(n, sizeof(double)), *f1 = calloc(n, sizeof(double));
    double *Ps = calloc(n, sizeof(double));
    int s = 0;
    for (int step = 0; step < nsteps && !s; step++) {
        if (v_sched) d.v_top = v_sched[step];
        s = orc_tdgl_rhs(&d, P, phi, f0);
        if (s) break;
        for (size_t c = 0; c < n; c++) Ps[c] = P[c] + dt * f0[c];
        s = orc_solve(&d, Ps, phi, tol, max_newton, last);          /* phi := phi* */
        if (s) break;
        s = orc_tdgl_rhs(&d, Ps, phi, f1);
        if (s) break;
        for (size_t c = 0; c < n; c++) P[c] = P[c] + 0.5 * dt * f0[c] + 0.5 * dt * f1[c];
        s = orc_solve(&d, P, phi, tol, max_newton, last);           /* phi := phi^{n+1} */
    }
    free(f0);
    free(f1);
    free(Ps);
    return s;
}
