/*
 * lbm_oracle.c -- plain, slow, FP64 CPU reference of the one-domain porous-media lattice
 * Boltzmann method of Gusev & Karlin, "Monolithic kinetic algorithm for heterogeneous porous
 * media systems using a continuous one-domain approach" (arXiv 2606.29619).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the oracle the GPU library is checked against.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may load it; the product
 * path never does.  It shares no code, header, table or constant generator with the GPU library.
 *
 * Every routine follows the paper's algorithm in the paper's order and notation:
 *   populations f-bar_i, porosity eps, intrinsic density rho, superficial velocity v,
 *   acceleration a, corrections Phi^ext and Phi^eta, relaxation parameter beta, lambda = dt = 1.
 * Citations name the paper's sections and equation labels.
 *
 * Storage is two plain arrays A/B (push streaming), FP64 everywhere, loops over cells in
 * index order n = x + nx*(y + ny*z).  Every axis wraps periodically; solid cells (mask != 0)
 * hold no populations and reflect populations by halfway (link-wise) bounce-back, so a wall is a
 * layer of solid cells.  The porosity eps is read on every cell (solid cells included) and its
 * derivatives are plain central differences; moment fields exist on fluid cells only and their
 * derivatives become one-sided next to solids (Sec. 3.5, last paragraph).
 *
 * Build with -ffp-contract=off: the expressions below are evaluated exactly as written.
 *
 * Threads (OpenMP): the per-cell passes split the cells among threads.  Every iteration writes
 * only its own cell's results (streaming writes each destination slot exactly once) and reads
 * fields that the pass does not write, and the global sums stay sequential, so the result is
 * bit for bit the same for any number of threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXQ 27

typedef struct {
    int D;              /* 2 (D2Q9) or 3 (D3Q27) */
    int nx, ny, nz;     /* nz must be 1 when D == 2 */
    double RT;          /* lattice temperature; RT = 1/3 is the lattice reference */
    double nu_f;        /* molecular viscosity in the Darcy coefficient mu_D */
    double nu_eff_ref;  /* effective shear viscosity nu_eff(eps) = nu_eff_ref * eps^nu_eff_pow */
    int nu_eff_pow;     /* -1, 0 or 1 */
    double eta_eff;     /* effective bulk viscosity; NaN switches the Phi^eta correction off */
    double b[3];        /* body acceleration */
    double rho0;        /* uniform initial intrinsic density when rho_init is NULL */
    int visc_corr;      /* 1: full Delta_nu; 0: omit Delta_nu (the paper's diagnostic variant) */
    int ext_corr;       /* 1: Phi^ext on; 0: off (the paper's diagnostic variant) */
    int lagged;         /* 0: faithful; 1: neighbour moments taken from the previous step */
    const double *eps;  /* [N] porosity, every cell */
    const double *kappa;/* [N] permeability, +inf allowed (free fluid) */
    const double *cf;   /* [N] Forchheimer coefficient C_F = F_eps / sqrt(kappa) */
    const uint8_t *mask;/* [N] 1 = solid, NULL = no solids */
    const double *rho_init; /* [N] or NULL */
    const double *v_init;   /* [D][N] superficial velocity or NULL (zero) */
    /* Wet-node boundaries (Sec. 3.4); bc_type NULL = none.  A boundary node is a fluid cell
     * whose outward neighbour along each of its normals is solid.  A node with one normal (a
     * face) has a bulk fluid cell as inward neighbour; a velocity node may have two or three
     * (an edge or corner, Sec. 3.4.1), and then the two cells x_b + d and x_b + 2d along the
     * inward diagonal d = -(sum of its normals) are bulk fluid cells. */
    const uint8_t *bc_type;   /* [N] 0 bulk, 1 velocity node, 2 pressure node, 3 outflow node */
    const uint8_t *bc_normal; /* [N] one outward normal: 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z; or
                                 several: 64 + sx + 4 sy + 16 sz with s = 0 none, 1 minus,
                                 2 plus along that axis */
    const double *bc_vel;     /* [D][N] prescribed superficial velocity (velocity nodes), or NULL */
    const double *bc_rho;     /* [N] prescribed intrinsic density (pressure nodes), or NULL */
    int bc_scheme;            /* 0 equilibrium (eq_bc_f_bar), 1 NEEM (NEEM_bc_f_bar), 2 TMS */
    int bc_density;           /* velocity nodes: 0 mass continuity (bc_density_impermWall) on
                                 faces and extrapolation from the bulk on edges and corners,
                                 1 bounce-back (bc_density_BounceBack) everywhere */
    /* Second-order velocity evaluation (App. F): Picard iterations after the one-shot
     * correction (0 = one-shot only) and the under-relaxation factor omega in (0, 1]. */
    int picard_iters;
    double picard_omega;
    /* Analytic porosity derivatives (Sec. 3.5), both NULL for central differences:
     * grad_eps [D][N], hess_eps [D(D+1)/2][N] holding the Hessian's upper triangle row by row
     * (xx, xy, yy in 2D; xx, xy, xz, yy, yz, zz in 3D). */
    const double *grad_eps;
    const double *hess_eps;
} orc_params;

typedef struct {
    orc_params p;
    int D, Q;
    long N;
    int c[ORC_MAXQ][3];
    int opp[ORC_MAXQ];
    double *F, *G;          /* populations [Q][N], current and scratch */
    double *eps, *muD, *muF, *nu, *dnu, *beta;
    double *ge;             /* [D][N] grad eps */
    double *H;              /* [D*D][N] Hessian of eps */
    uint8_t *solid;         /* [N] */
    double *rho, *v1, *v;   /* moments: rho [N], v^(1) [D][N], corrected v [D][N] */
    double *v0;             /* base predictor v_0 [D][N] (v_(0)) */
    double *m;              /* scratch vector field [D][N] */
    double *g;              /* scratch scalar field [N] */
    double *prho, *pv1, *pv;/* previous-step rho, v^(1) and v (lagged mode) */
    double *vw;             /* scratch velocity field [D][N] */
    int have_prev;
    double *vsnap;          /* residual snapshot [D][N] */
    long *nbr;              /* [3][2][N] index of the periodic neighbour n -/+ e_a */
    long *bnodes;           /* boundary node indices, nb of them */
    long nb;
    long t;
} orc_solver;

/* ------------------------------------------------------------------------------------------ */
/* Lattices D2Q9 and D3Q27 (Sec. 3.1): c_ia in {-1,0,1}, Q = 3^D.                             */
/* D2Q9 numbering is the one the paper's wall example uses (Sec. 3.4.1): tangential {0,1,3},   */
/* outgoing set {4,7,8} on the bottom wall and {2,5,6} on the top wall.                        */
/* D3Q27 numbering: rest, six faces, twelve edges, eight corners, opposite pairs adjacent.     */
/* ------------------------------------------------------------------------------------------ */
static const int C2[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};

static const int C3[27][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
    {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};

int orc_lattice(int D, int *c_out, int *opp_out)
{
    int Q, i, j, a;
    const int (*C)[3];
    if (D == 2) { Q = 9; C = C2; }
    else if (D == 3) { Q = 27; C = C3; }
    else return -1;
    for (i = 0; i < Q; ++i) {
        for (a = 0; a < 3; ++a) c_out[3 * i + a] = C[i][a];
        for (j = 0; j < Q; ++j)
            if (C[j][0] == -C[i][0] && C[j][1] == -C[i][1] && C[j][2] == -C[i][2]) opp_out[i] = j;
    }
    return Q;
}

/* One-dimensional factor of the product-form equilibrium, eq. (1d_scaled_eq):
 * Psi(c; xi, P) = 1 - c^2 + ((3c^2 - 2) P + c xi) / 2. */
static double psi(int c, double xi, double P)
{
    double cc = (double)(c * c);
    return (1.0 - cc) + ((3.0 * cc - 2.0) * P + (double)c * xi) / 2.0;
}

/* Lattice weights, eq. (eq_weights): w_i = prod_a Psi(c_ia; 0, RT). */
int orc_weights(int D, double RT, double *w_out)
{
    int c[ORC_MAXQ * 3], opp[ORC_MAXQ], Q, i, a;
    Q = orc_lattice(D, c, opp);
    if (Q < 0) return -1;
    for (i = 0; i < Q; ++i) {
        double w = 1.0;
        for (a = 0; a < D; ++a) w = w * psi(c[3 * i + a], 0.0, RT);
        w_out[i] = w;
    }
    return Q;
}

/* Product-form populations, eq. (prod_form): f_i = eps rho prod_a Psi(c_ia; xi_a, P_aa).
 * The product is taken in axis order x, y, z starting from eps*rho. */
static void product_form(int D, int Q, const int (*c)[3], double eps, double rho,
                         const double *xi, const double *P, double *f)
{
    int i, a;
    for (i = 0; i < Q; ++i) {
        double val = eps * rho;
        for (a = 0; a < D; ++a) val = val * psi(c[i][a], xi[a], P[a]);
        f[i] = val;
    }
}

void orc_product_form(int D, double eps, double rho, const double *xi, const double *P, double *f)
{
    int c[ORC_MAXQ][3], opp[ORC_MAXQ], Q;
    Q = orc_lattice(D, &c[0][0], opp);
    if (Q < 0) return;
    product_form(D, Q, (const int (*)[3])c, eps, rho, xi, P, f);
}

/* Closed-form implicit drag solve, eqs. (v_(1)) and (velocity_coefficients) with dt = 1:
 * c1 = 1 + mu_D/2, c2 = mu_F/2, v1 = 2 v0 / (c1 + sqrt(c1^2 + 4 c2 |v0|)). */
static void drag_solve(int D, const double *v0, double muD, double muF, double *v1)
{
    int a;
    double c1 = 1.0 + 0.5 * muD;
    double c2 = 0.5 * muF;
    double s = 0.0, vm, den;
    for (a = 0; a < D; ++a) s = s + v0[a] * v0[a];
    vm = sqrt(s);
    den = c1 + sqrt(c1 * c1 + (4.0 * c2) * vm);
    for (a = 0; a < D; ++a) v1[a] = (2.0 * v0[a]) / den;
}

void orc_drag_solve(int D, const double *v0, double muD, double muF, double *v1)
{
    drag_solve(D, v0, muD, muF, v1);
}

/* ------------------------------------------------------------------------------------------ */
/* Grid helpers                                                                               */
/* ------------------------------------------------------------------------------------------ */
/* Periodic neighbour n + k e_a (|k| <= 2) through the neighbour table built at creation. */
static long shift(const orc_solver *S, long n, int a, int k)
{
    long N = S->N;
    while (k > 0) { n = S->nbr[(a * 2 + 1) * N + n]; --k; }
    while (k < 0) { n = S->nbr[(a * 2 + 0) * N + n]; ++k; }
    return n;
}

static long shift3(const orc_solver *S, long n, const int *c)
{
    int a;
    for (a = 0; a < 3; ++a) n = shift(S, n, a, c[a]);
    return n;
}

static void build_neighbours(orc_solver *S)
{
    long nx = S->p.nx, ny = S->p.ny, nz = S->p.nz, N = S->N, n;
    for (n = 0; n < N; ++n) {
        long x = n % nx, y = (n / nx) % ny, z = n / (nx * ny);
        S->nbr[0 * N + n] = ((x + nx - 1) % nx) + nx * (y + ny * z);
        S->nbr[1 * N + n] = ((x + 1) % nx) + nx * (y + ny * z);
        S->nbr[2 * N + n] = x + nx * (((y + ny - 1) % ny) + ny * z);
        S->nbr[3 * N + n] = x + nx * (((y + 1) % ny) + ny * z);
        S->nbr[4 * N + n] = x + nx * (y + ny * ((z + nz - 1) % nz));
        S->nbr[5 * N + n] = x + nx * (y + ny * ((z + 1) % nz));
    }
}

/* Derivative of a moment field g along axis a at fluid cell n (Sec. 3.5, last paragraph):
 * second-order central difference when both axis neighbours are fluid, second-order one-sided
 * difference into the fluid next to a solid, first order when only one fluid cell is available
 * on that side, and zero for a cell with no fluid neighbour along the axis.  g0 is the cell's own
 * value: g[n] itself, or the current value where the lagged scheme takes the neighbour values
 * from the previous step. */
static double deriv_own(const orc_solver *S, const double *g, long n, int a, double g0)
{
    long p1 = shift(S, n, a, 1), m1 = shift(S, n, a, -1);
    int fp1 = !S->solid[p1], fm1 = !S->solid[m1];
    if (fp1 && fm1) return (g[p1] - g[m1]) * 0.5;
    if (fp1) {
        long p2 = shift(S, n, a, 2);
        if (!S->solid[p2]) return ((-3.0 * g0 + 4.0 * g[p1]) - g[p2]) * 0.5;
        return g[p1] - g0;
    }
    if (fm1) {
        long m2 = shift(S, n, a, -2);
        if (!S->solid[m2]) return ((3.0 * g0 - 4.0 * g[m1]) + g[m2]) * 0.5;
        return g0 - g[m1];
    }
    return 0.0;
}


/* Porosity gradient and Hessian.  Sec. 3.5 prefers analytic derivatives of eps where eps(x) is
 * given in closed form: then they are the caller's.  Otherwise central differences on the
 * (everywhere defined) eps field. */
static void porosity_derivatives(orc_solver *S)
{
    int D = S->D, a, b;
    long n, N = S->N;
    const double *e = S->eps;
    if (S->p.grad_eps) {
        for (n = 0; n < N; ++n) {
            int k = 0;
            for (a = 0; a < D; ++a) S->ge[a * N + n] = S->p.grad_eps[a * N + n];
            for (a = 0; a < D; ++a)
                for (b = a; b < D; ++b) {
                    double h = S->p.hess_eps[(long)k * N + n];
                    S->H[(a * D + b) * N + n] = h;
                    S->H[(b * D + a) * N + n] = h;
                    k = k + 1;
                }
        }
        return;
    }
#pragma omp parallel for private(a, b) schedule(static)
    for (n = 0; n < N; ++n) {
        for (a = 0; a < D; ++a) {
            long p = shift(S, n, a, 1), q = shift(S, n, a, -1);
            S->ge[a * N + n] = (e[p] - e[q]) * 0.5;
        }
        /* pure second derivatives e(+1) - 2 e(0) + e(-1); mixed ones by the four diagonal
         * neighbours, computed once for a < b so that the Hessian is exactly symmetric */
        for (a = 0; a < D; ++a)
            for (b = a; b < D; ++b) {
                double h;
                if (a == b) {
                    long p = shift(S, n, a, 1), q = shift(S, n, a, -1);
                    h = (e[p] - 2.0 * e[n]) + e[q];
                } else {
                    long pa = shift(S, n, a, 1), ma = shift(S, n, a, -1);
                    long pp = shift(S, pa, b, 1), pm = shift(S, pa, b, -1);
                    long mp = shift(S, ma, b, 1), mm = shift(S, ma, b, -1);
                    h = (((e[pp] - e[pm]) - e[mp]) + e[mm]) * 0.25;
                }
                S->H[(a * D + b) * N + n] = h;
                S->H[(b * D + a) * N + n] = h;
            }
    }
}

/* Variable-porosity viscous correction Delta_nu(m) at cell n, expanded form
 * (porosity_correction_expanded), which follows from the divergence form (porosity_correction):
 *   nu {[H + tr(H) I] m + (div m) grad eps + (grad m) grad eps}
 *     + nu' [|grad eps|^2 m + (m . grad eps) grad eps],
 * with [(grad m) grad eps]_a = sum_b (d_b m_a)(d_b eps).  J[a][b] = d_b m_a. */
static void delta_nu(const orc_solver *S, long n, const double *mv, const double (*J)[3],
                     double *out)
{
    int D = S->D, a, b;
    long N = S->N;
    double ge[3], trH = 0.0, div = 0.0, g2 = 0.0, mg = 0.0;
    double nu = S->nu[n], dnu = S->dnu[n];
    for (a = 0; a < D; ++a) ge[a] = S->ge[a * N + n];
    for (a = 0; a < D; ++a) trH = trH + S->H[(a * D + a) * N + n];
    for (a = 0; a < D; ++a) div = div + J[a][a];
    for (a = 0; a < D; ++a) g2 = g2 + ge[a] * ge[a];
    for (a = 0; a < D; ++a) mg = mg + mv[a] * ge[a];
    for (a = 0; a < D; ++a) {
        double Hm = 0.0, Jg = 0.0, t1, t2, t3, t4, t5;
        for (b = 0; b < D; ++b) Hm = Hm + S->H[(a * D + b) * N + n] * mv[b];
        for (b = 0; b < D; ++b) Jg = Jg + J[a][b] * ge[b];
        t1 = Hm + trH * mv[a];
        t2 = div * ge[a];
        t3 = Jg;
        t4 = g2 * mv[a];
        t5 = mg * ge[a];
        out[a] = nu * ((t1 + t2) + t3) + dnu * (t4 + t5);
    }
}

/* Delta_nu of the vector field m (stored [D][N]) at fluid cell n whose own value is mv (m at n
 * itself, or the current value where the neighbours are the previous step's). */
static void delta_nu_own(const orc_solver *S, const double *m, long n, const double *mv,
                         double *out)
{
    int D = S->D, a, b;
    long N = S->N;
    double J[3][3];
    for (a = 0; a < D; ++a)
        for (b = 0; b < D; ++b) J[a][b] = deriv_own(S, m + a * N, n, b, mv[a]);
    delta_nu(S, n, mv, (const double (*)[3])J, out);
}

/* Delta_nu of the vector field m (stored [D][N]) at fluid cell n. */
static void delta_nu_field(const orc_solver *S, const double *m, long n, double *out)
{
    int D = S->D, a;
    long N = S->N;
    double mv[3];
    for (a = 0; a < D; ++a) mv[a] = m[a * N + n];
    delta_nu_own(S, m, n, mv, out);
}

/* ------------------------------------------------------------------------------------------ */
/* Creation: drag coefficients (mu_D_Ergun_perm, mu_F_Ergun_perm), nu_eff(eps), nu_eff'(eps)  */
/* and beta from (nu_eff_def) with dt = 1, porosity derivatives, then the initial populations */
/* (eq_bc_f_bar applied to every cell, as the flowchart's initialisation step prescribes).    */
/* ------------------------------------------------------------------------------------------ */
static void *xcalloc(long n, long sz)
{
    void *p = calloc((size_t)(n > 0 ? n : 1), (size_t)sz);
    return p;
}

static void init_populations(orc_solver *S);
static int bc_normal_vec(const orc_solver *S, long b, int *nv);
static long bc_inner(const orc_solver *S, long b, const int *nv);

void orc_destroy(orc_solver *S)
{
    if (!S) return;
    free(S->F); free(S->G); free(S->eps); free(S->muD); free(S->muF); free(S->nu);
    free(S->dnu); free(S->beta); free(S->ge); free(S->H); free(S->solid); free(S->rho);
    free(S->v1); free(S->v); free(S->m); free(S->g); free(S->prho); free(S->pv1); free(S->pv);
    free(S->bnodes); free(S->v0);
    free(S->vw);
    free(S->vsnap);
    free(S->nbr);
    free(S);
}

orc_solver *orc_create(const orc_params *p, char *err, int errlen)
{
    orc_solver *S;
    int Q, i, D = p->D;
    long n, N;
    if (!(D == 2 || D == 3) || p->nx < 1 || p->ny < 1 || p->nz < 1 || (D == 2 && p->nz != 1)) {
        snprintf(err, (size_t)errlen, "bad lattice or dimensions");
        return NULL;
    }
    if (!(p->nu_eff_pow == -1 || p->nu_eff_pow == 0 || p->nu_eff_pow == 1)) {
        snprintf(err, (size_t)errlen, "nu_eff_pow must be -1, 0 or 1");
        return NULL;
    }
    if (!(p->RT > 0.0) || !(p->nu_eff_ref > 0.0) || !p->eps || !p->kappa || !p->cf) {
        snprintf(err, (size_t)errlen, "bad physical parameters or missing fields");
        return NULL;
    }
    if ((p->grad_eps == NULL) != (p->hess_eps == NULL)) {
        snprintf(err, (size_t)errlen, "grad_eps and hess_eps go together");
        return NULL;
    }
    S = (orc_solver *)xcalloc(1, sizeof(orc_solver));
    S->p = *p;
    S->D = D;
    N = (long)p->nx * p->ny * p->nz;
    S->N = N;
    {
        int cflat[ORC_MAXQ * 3];
        Q = orc_lattice(D, cflat, S->opp);
        for (i = 0; i < Q; ++i) {
            S->c[i][0] = cflat[3 * i]; S->c[i][1] = cflat[3 * i + 1]; S->c[i][2] = cflat[3 * i + 2];
        }
    }
    S->Q = Q;
    S->F = (double *)xcalloc(Q * N, sizeof(double));
    S->G = (double *)xcalloc(Q * N, sizeof(double));
    S->eps = (double *)xcalloc(N, sizeof(double));
    S->muD = (double *)xcalloc(N, sizeof(double));
    S->muF = (double *)xcalloc(N, sizeof(double));
    S->nu = (double *)xcalloc(N, sizeof(double));
    S->dnu = (double *)xcalloc(N, sizeof(double));
    S->beta = (double *)xcalloc(N, sizeof(double));
    S->ge = (double *)xcalloc(D * N, sizeof(double));
    S->H = (double *)xcalloc(D * D * N, sizeof(double));
    S->solid = (uint8_t *)xcalloc(N, 1);
    S->rho = (double *)xcalloc(N, sizeof(double));
    S->v1 = (double *)xcalloc(D * N, sizeof(double));
    S->v = (double *)xcalloc(D * N, sizeof(double));
    S->m = (double *)xcalloc(D * N, sizeof(double));
    S->g = (double *)xcalloc(N, sizeof(double));
    S->prho = (double *)xcalloc(N, sizeof(double));
    S->pv1 = (double *)xcalloc(D * N, sizeof(double));
    S->pv = (double *)xcalloc(D * N, sizeof(double));
    S->vw = (double *)xcalloc(D * N, sizeof(double));
    S->v0 = (double *)xcalloc(D * N, sizeof(double));
    S->vsnap = (double *)xcalloc(D * N, sizeof(double));
    S->nbr = (long *)xcalloc(6 * N, sizeof(long));
    if (!S->F || !S->G || !S->eps || !S->muD || !S->muF || !S->nu || !S->dnu || !S->beta ||
        !S->ge || !S->H || !S->solid || !S->rho || !S->v1 || !S->v || !S->m || !S->g ||
        !S->prho || !S->pv1 || !S->pv || !S->vw || !S->vsnap || !S->nbr || !S->v0) {
        snprintf(err, (size_t)errlen, "out of host memory");
        orc_destroy(S);
        return NULL;
    }
    for (n = 0; n < N; ++n) {
        double e = p->eps[n], k = p->kappa[n], nu;
        S->solid[n] = p->mask ? (p->mask[n] ? 1 : 0) : 0;
        if (!(e > 0.0 && e <= 1.0)) {
            snprintf(err, (size_t)errlen, "porosity outside (0,1] at cell %ld", n);
            orc_destroy(S);
            return NULL;
        }
        if (!S->solid[n] && !(k > 0.0)) {
            snprintf(err, (size_t)errlen, "permeability must be positive at cell %ld", n);
            orc_destroy(S);
            return NULL;
        }
        S->eps[n] = e;
        /* (mu_D_Ergun_perm): mu_D = eps nu_f / kappa, zero for kappa = +inf. */
        S->muD[n] = e * p->nu_f / k;
        /* (mu_F_Ergun_perm) with C_F = F_eps / sqrt(kappa): mu_F = eps C_F. */
        S->muF[n] = e * p->cf[n];
        if (p->nu_eff_pow == -1) { nu = p->nu_eff_ref / e; S->dnu[n] = -p->nu_eff_ref / (e * e); }
        else if (p->nu_eff_pow == 1) { nu = p->nu_eff_ref * e; S->dnu[n] = p->nu_eff_ref; }
        else { nu = p->nu_eff_ref; S->dnu[n] = 0.0; }
        S->nu[n] = nu;
        /* (nu_eff_def) solved for beta with dt = 1: beta = 1 / (1 + 2 nu_eff / RT). */
        S->beta[n] = 1.0 / (1.0 + (2.0 * nu) / p->RT);
    }
    build_neighbours(S);
    if (p->bc_type) {
        long k = 0;
        for (n = 0; n < N; ++n) k += p->bc_type[n] ? 1 : 0;
        S->bnodes = (long *)xcalloc(k > 0 ? k : 1, sizeof(long));
        S->nb = k;
        k = 0;
        for (n = 0; n < N; ++n)
            if (p->bc_type[n]) S->bnodes[k++] = n;
        /* edge and corner nodes: velocity nodes whose two inward-diagonal cells are bulk fluid
         * (their density may be extrapolated from them) */
        for (k = 0; k < S->nb; ++k) {
            int nv[3];
            long b = S->bnodes[k], f1, f2;
            if (bc_normal_vec(S, b, nv) < 2) continue;
            f1 = bc_inner(S, b, nv);
            f2 = bc_inner(S, f1, nv);
            if (p->bc_type[b] != 1 || S->solid[f1] || S->solid[f2] || p->bc_type[f1] ||
                p->bc_type[f2]) {
                snprintf(err, (size_t)errlen, "edge or corner node %ld: velocity nodes only, with "
                         "bulk fluid along the inward diagonal", b);
                orc_destroy(S);
                return NULL;
            }
        }
    }
    porosity_derivatives(S);
    S->p.grad_eps = NULL;   /* the caller's arrays are read only here */
    S->p.hess_eps = NULL;
    init_populations(S);
    return S;
}

/* ------------------------------------------------------------------------------------------ */
/* Moments (pass one): density (transformed_density_moment), momentum                         */
/* (transformed_momentum_moment), v^(0) (v_(0)) and the drag solve v^(1) (v_(1)).              */
/* ------------------------------------------------------------------------------------------ */
static void moments_v1(orc_solver *S)
{
    int D = S->D, Q = S->Q, i, a;
    long n, N = S->N;
#pragma omp parallel for private(i, a) schedule(static)
    for (n = 0; n < N; ++n) {
        double sum = 0.0, Pi[3] = {0.0, 0.0, 0.0}, v0[3], v1[3], rho, e;
        if (S->solid[n]) {
            S->rho[n] = 0.0;
            for (a = 0; a < D; ++a) S->v1[a * N + n] = 0.0;
            continue;
        }
        for (i = 0; i < Q; ++i) {
            double f = S->F[(long)i * N + n];
            sum = sum + f;
            for (a = 0; a < D; ++a) Pi[a] = Pi[a] + (double)S->c[i][a] * f;
        }
        e = S->eps[n];
        rho = sum / e;
        for (a = 0; a < D; ++a)
            v0[a] = Pi[a] / rho + 0.5 * (e * S->p.b[a] + S->p.RT * S->ge[a * N + n]);
        drag_solve(D, v0, S->muD[n], S->muF[n], v1);
        for (a = 0; a < D; ++a) S->v0[a * N + n] = v0[a];
        S->rho[n] = rho;
        for (a = 0; a < D; ++a) S->v1[a * N + n] = v1[a];
    }
}

/* Field m = rho * w / eps on fluid cells, from densities r and a velocity field w. */
static void momentum_over_eps(orc_solver *S, const double *r, const double *w)
{
    int D = S->D, a;
    long n, N = S->N;
#pragma omp parallel for private(a) schedule(static)
    for (n = 0; n < N; ++n)
        for (a = 0; a < D; ++a)
            S->m[a * N + n] = S->solid[n] ? 0.0 : (r[n] * w[a * N + n]) / S->eps[n];
}

/* Velocity correction (v_final): v = v^(1) + Delta_nu(rho v^(1) / eps) / (2 rho).
 * In lagged mode the neighbour values of rho v^(1)/eps come from the previous step's rho and
 * v^(1) while the cell's own value is current, so a steady state is the faithful one. */
static void correct_velocity(orc_solver *S)
{
    int D = S->D, a;
    long n, N = S->N;
    if (!S->p.visc_corr) {
        memcpy(S->v, S->v1, sizeof(double) * (size_t)(D * N));
        return;
    }
    if (S->p.lagged && S->have_prev) momentum_over_eps(S, S->prho, S->pv1);
    else momentum_over_eps(S, S->rho, S->v1);
#pragma omp parallel for private(a) schedule(static)
    for (n = 0; n < N; ++n) {
        double dn[3];
        if (S->solid[n]) {
            for (a = 0; a < D; ++a) S->v[a * N + n] = 0.0;
            continue;
        }
        if (S->p.lagged && S->have_prev) {
            /* own value current, neighbour values lagged */
            double own[3];
            for (a = 0; a < D; ++a) own[a] = (S->rho[n] * S->v1[a * N + n]) / S->eps[n];
            delta_nu_own(S, S->m, n, own, dn);
        } else {
            delta_nu_field(S, S->m, n, dn);
        }
        for (a = 0; a < D; ++a) S->v[a * N + n] = S->v1[a * N + n] + dn[a] / (2.0 * S->rho[n]);
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Wet-node boundaries (Sec. 3.4).  For a boundary node with outward unit normal n, the        */
/* post-advection populations split into P- (c_i . n < 0: incoming from outside, unknown),     */
/* P0 (c_i . n = 0) and P+ (c_i . n > 0), eq. (bc_rho_components_def).                         */
/* ------------------------------------------------------------------------------------------ */
/* Outward normal(s) of boundary node b as a vector with one entry per axis in {-1, 0, 1};
 * returns how many axes carry a normal (1 on a face, 2 on an edge, 3 on a corner). */
static int bc_normal_vec(const orc_solver *S, long b, int *nv)
{
    int code = S->p.bc_normal[b], a, k = 0;
    nv[0] = nv[1] = nv[2] = 0;
    if (code >= 64) {
        for (a = 0; a < 3; ++a) {
            int sa = (code - 64) >> (2 * a) & 3;
            nv[a] = sa == 1 ? -1 : (sa == 2 ? 1 : 0);
            if (nv[a] != 0) k = k + 1;
        }
        return k;
    }
    nv[code / 2] = (code % 2) ? 1 : -1;
    return 1;
}

static int c_dot(const orc_solver *S, int i, const int *nv)
{
    return S->c[i][0] * nv[0] + S->c[i][1] * nv[1] + S->c[i][2] * nv[2];
}

/* Is population i one of the unknown incoming ones (P-)?  It arrives from outside through one
 * of the node's faces: c_i points inwards along some normal axis. */
static int in_pminus(const orc_solver *S, int i, const int *nv)
{
    int a;
    for (a = 0; a < 3; ++a)
        if (nv[a] != 0 && S->c[i][a] == -nv[a]) return 1;
    return 0;
}

/* The bulk node next to boundary node b along its inward normal (the inward diagonal on edges
 * and corners). */
static long bc_inner(const orc_solver *S, long b, const int *nv)
{
    int m[3] = {-nv[0], -nv[1], -nv[2]};
    return shift3(S, b, m);
}

/* Zero-gradient outflow, eq. (f_bar_outflow_BC): the unknown incoming populations copy those
 * of the inner node. */
static void apply_outflow(orc_solver *S)
{
    long k, N = S->N;
    int i, nv[3];
    for (k = 0; k < S->nb; ++k) {
        long b = S->bnodes[k], f;
        if (S->p.bc_type[b] != 3) continue;
        bc_normal_vec(S, b, nv);
        f = bc_inner(S, b, nv);
        for (i = 0; i < S->Q; ++i)
            if (in_pminus(S, i, nv)) S->F[(long)i * N + b] = S->F[(long)i * N + f];
    }
}

/* Viscous term of eq. (accel_approx_boundary) at face node b with outward normal nv: the
 * normal component of Delta_nu(rho v / eps) / rho with the density taken outside the
 * divergence of eq. (porosity_correction),
 *   div W,  W(x) = nu_eff(x) [ (v(x) / eps(x)) (n . grad eps)(x) + grad eps(x) (n . v(x)) / eps(x) ],
 * n fixed to the node's normal, v the velocities of the records at this point of the step
 * (v^(1) on bulk cells, the boundary velocity on boundary nodes), grad eps as everywhere else
 * (R6), and each d/dx_beta by the derivative rule of moment fields (one-sided next to solids).
 * The W_beta values of the stencil go through the scratch field g. */
static double bc_flux(const orc_solver *S, long c, const int *nv, int beta)
{
    int D = S->D, a;
    long N = S->N;
    double e = S->eps[c], gn = 0.0, vn = 0.0;
    for (a = 0; a < D; ++a) {
        gn = gn + (double)nv[a] * S->ge[a * N + c];
        vn = vn + (double)nv[a] * S->v1[a * N + c];
    }
    return S->nu[c] * ((S->v1[beta * N + c] / e) * gn + S->ge[beta * N + c] * (vn / e));
}

static double bc_viscous_term(orc_solver *S, long b, const int *nv)
{
    int beta, k;
    double div = 0.0;
    for (beta = 0; beta < S->D; ++beta) {
        for (k = -2; k <= 2; ++k) {
            long c = shift(S, b, beta, k);
            if (k != 0 && !S->solid[c]) S->g[c] = bc_flux(S, c, nv, beta);
        }
        div = div + deriv_own(S, S->g, b, beta, bc_flux(S, b, nv, beta));
    }
    return div;
}

/* Density and velocity of the velocity and pressure nodes, written over the bulk moments, in
 * two stages.
 * Stage 1, every node:
 *   velocity node, v_b prescribed, density rho_b:
 *     bounce-back rule: eq. (bc_density_BounceBack), which with halfway bounce-back in the
 *       streaming is the sum of all post-advection populations over eps_b;
 *     continuity rule, face node (one normal): mass continuity, eq. (bc_density_impermWall),
 *       rho_b = (S0 + 2 S+) / (eps_b + v_b,perp - a_b,perp / 2), S0 and S+ the sums of the known
 *       populations in P0 and P+, a_b,perp from eq. (accel_approx_boundary) without its viscous
 *       term in this stage: eps_b b_perp - mu_D v_perp - mu_F |v_b| v_perp + RT (d eps / dn);
 *     continuity rule, edge or corner node: the relation does not apply there (Sec. 3.4.1), and
 *       the density is extrapolated from the bulk along the inward diagonal d:
 *       rho_b = 2 rho(x_b + d) - rho(x_b + 2 d);
 *   pressure node (one normal): rho_b prescribed, tangential velocity zero, and the same
 *     continuity relation solved for v_perp: v_perp (1 + mu_D / 2) + (mu_F / 2) |v_perp| v_perp = R
 *     with R = (S0 + 2 S+) / rho_b - eps_b + (eps_b b_perp + RT d eps / dn) / 2, in closed form as
 *     in eq. (v_(1)).
 * Stage 2, face velocity nodes under the continuity rule, with the viscous correction on: the
 *   density again, now with the viscous term of eq. (accel_approx_boundary) in a_b,perp, from
 *   the velocities stage 1 left in the records. */
static void boundary_records(orc_solver *S)
{
    int D = S->D, a, i, nv[3], stage;
    long k, N = S->N;
    for (stage = 1; stage <= 2; ++stage) {
        if (stage == 2 && !(S->p.visc_corr && S->p.bc_density == 0)) break;
        for (k = 0; k < S->nb; ++k) {
            long b = S->bnodes[k];
            int type = S->p.bc_type[b], nn;
            double e = S->eps[b], s0 = 0.0, sp = 0.0, gperp = 0.0, bperp = 0.0;
            double vb[3] = {0.0, 0.0, 0.0};
            if (type != 1 && type != 2) continue;
            nn = bc_normal_vec(S, b, nv);
            if (stage == 2 && (type != 1 || nn != 1)) continue;
            for (i = 0; i < S->Q; ++i) {
                int cn = c_dot(S, i, nv);
                double f = S->F[(long)i * N + b];
                if (cn == 0) s0 = s0 + f;
                else if (cn > 0) sp = sp + f;
            }
            for (a = 0; a < D; ++a) {
                gperp = gperp + (double)nv[a] * S->ge[a * N + b];
                bperp = bperp + (double)nv[a] * S->p.b[a];
            }
            if (type == 1) {
                double vperp = 0.0, vm = 0.0, aperp, rho;
                for (a = 0; a < D; ++a) vb[a] = S->p.bc_vel ? S->p.bc_vel[a * N + b] : 0.0;
                for (a = 0; a < D; ++a) vperp = vperp + (double)nv[a] * vb[a];
                for (a = 0; a < D; ++a) vm = vm + vb[a] * vb[a];
                vm = sqrt(vm);
                if (S->p.bc_density == 1) {
                    double sum = 0.0;
                    for (i = 0; i < S->Q; ++i) sum = sum + S->F[(long)i * N + b];
                    rho = sum / e;
                } else if (nn > 1) {
                    long f1 = bc_inner(S, b, nv), f2 = bc_inner(S, f1, nv);
                    rho = 2.0 * S->rho[f1] - S->rho[f2];
                } else {
                    aperp = ((e * bperp - S->muD[b] * vperp) - (S->muF[b] * vm) * vperp) +
                            S->p.RT * gperp;
                    if (stage == 2) aperp = aperp + bc_viscous_term(S, b, nv);
                    rho = (s0 + 2.0 * sp) / ((e + vperp) - 0.5 * aperp);
                }
                S->rho[b] = rho;
            } else {
                double rho = S->p.bc_rho[b];
                double R = ((s0 + 2.0 * sp) / rho - e) + 0.5 * (e * bperp + S->p.RT * gperp);
                double c1 = 1.0 + 0.5 * S->muD[b], c2 = 0.5 * S->muF[b];
                double vperp = (2.0 * R) / (c1 + sqrt(c1 * c1 + (4.0 * c2) * fabs(R)));
                for (a = 0; a < D; ++a) vb[a] = (double)nv[a] * vperp;
                S->rho[b] = rho;
            }
            for (a = 0; a < D; ++a) S->v1[a * N + b] = vb[a];
        }
    }
}

/* The corrected velocity of velocity and pressure nodes is their boundary velocity. */
static void boundary_velocity(orc_solver *S)
{
    int D = S->D, a;
    long k, N = S->N;
    for (k = 0; k < S->nb; ++k) {
        long b = S->bnodes[k];
        if (S->p.bc_type[b] != 1 && S->p.bc_type[b] != 2) continue;
        for (a = 0; a < D; ++a) S->v[a * N + b] = S->v1[a * N + b];
    }
}

/* Equilibrium f^eq(eps, rho, w) of eqs. (1d_scaled_eq)-(P_alpha_alpha_eq) at velocity w. */
static void equilibrium_at(const orc_solver *S, double e, double rho, const double *w, double *f)
{
    double xi[3], P[3];
    int a;
    for (a = 0; a < S->D; ++a) {
        xi[a] = w[a] / e;
        P[a] = xi[a] * xi[a] + S->p.RT;
    }
    product_form(S->D, S->Q, (const int (*)[3])S->c, e, rho, xi, P, f);
}

/* Forcing quantities at every fluid cell from the moment fields (rho, v):
 * acceleration a (accel) with m = rho v / eps, Phi^ext (ex_corr) and Phi^eta (eta_corr), then
 * xi, P (xi_alpha_eq, P_alpha_alpha_eq) and xi*, P* (xi_alpha_*, P_aa_*) with lambda = 1.
 * The results are written to xi[D][N], P[D][N], xs[D][N], Ps[D][N] and optionally the
 * acceleration and corrections for diagnostics. */
typedef struct {
    double *xi, *P, *xs, *Ps, *acc, *phx, *pheta;
} forcing_out;

static void forcing(orc_solver *S, const double *rho, const double *v, const double *nrho,
                    const double *nv, forcing_out *o)
{
    int D = S->D, a;
    long n, N = S->N;
    double RT = S->p.RT;
    double omr = 1.0 - 3.0 * RT;
    int eta_on = !isnan(S->p.eta_eff);
    double *gext = (double *)xcalloc(D * N, sizeof(double));
    double *vw = S->vw;
    /* neighbour fields: m = rho v / eps, g_a = rho v_a (1 - 3RT) - rho v_a^3 / eps^2 and v */
#pragma omp parallel for private(a) schedule(static)
    for (n = 0; n < N; ++n)
        for (a = 0; a < D; ++a) {
            double r = nrho[n], va = nv[a * N + n], e = S->eps[n];
            if (S->solid[n]) {
                S->m[a * N + n] = 0.0; gext[a * N + n] = 0.0; vw[a * N + n] = 0.0;
                continue;
            }
            S->m[a * N + n] = (r * va) / e;
            gext[a * N + n] = (r * va) * omr - (r * ((va * va) * va)) / (e * e);
            vw[a * N + n] = va;
        }
#pragma omp parallel for private(a) schedule(static)
    for (n = 0; n < N; ++n) {
        double vv[3], dm[3] = {0.0, 0.0, 0.0}, acc[3], phx[3], pheta = 0.0, s = 0.0, vm;
        double e, r, own_m[3], own_g[3];
        if (S->solid[n]) continue;
        e = S->eps[n];
        r = rho[n];
        for (a = 0; a < D; ++a) vv[a] = v[a * N + n];
        /* the cell's own values are always current (they differ from the neighbour fields
         * only in lagged mode) */
        for (a = 0; a < D; ++a) {
            own_m[a] = (r * vv[a]) / e;
            own_g[a] = (r * vv[a]) * omr - (r * ((vv[a] * vv[a]) * vv[a])) / (e * e);
        }
        /* acceleration, eq. (accel), with Delta_nu(rho u) = Delta_nu(rho v / eps) */
        if (S->p.visc_corr) delta_nu_own(S, S->m, n, own_m, dm);
        for (a = 0; a < D; ++a) s = s + vv[a] * vv[a];
        vm = sqrt(s);
        for (a = 0; a < D; ++a)
            acc[a] = (((e * S->p.b[a] - S->muD[n] * vv[a]) - (S->muF[n] * vm) * vv[a]) +
                      RT * S->ge[a * N + n]) + dm[a] / r;
        /* extended-equilibrium correction, eq. (ex_corr): one axis at a time, no summation */
        for (a = 0; a < D; ++a)
            phx[a] = S->p.ext_corr ? deriv_own(S, gext + a * N, n, a, own_g[a]) : 0.0;
        /* bulk-viscosity correction, eq. (eta_corr) */
        if (eta_on) {
            double divv = 0.0;
            for (a = 0; a < D; ++a) divv = divv + deriv_own(S, vw + a * N, n, a, vv[a]);
            pheta = ((r * RT) * (2.0 / (double)D - S->p.eta_eff / S->nu[n])) * divv;
        }
        /* equilibrium and shifted-equilibrium arguments, eqs. (xi_alpha_eq),
         * (P_alpha_alpha_eq), (xi_alpha_*), (P_aa_*) with lambda = 1 */
        for (a = 0; a < D; ++a) {
            double xi = vv[a] / e;
            double xs = (vv[a] + acc[a]) / e;
            o->xi[a * N + n] = xi;
            o->P[a * N + n] = xi * xi + RT;
            o->xs[a * N + n] = xs;
            o->Ps[a * N + n] = (xs * xs + RT) + (1.0 / (e * r)) * (phx[a] + pheta);
            if (o->acc) o->acc[a * N + n] = acc[a];
            if (o->phx) o->phx[a * N + n] = phx[a];
        }
        if (o->pheta) o->pheta[n] = pheta;
    }
    free(gext);
}

static void alloc_forcing(long DN, forcing_out *o)
{
    o->xi = (double *)xcalloc(DN, sizeof(double));
    o->P = (double *)xcalloc(DN, sizeof(double));
    o->xs = (double *)xcalloc(DN, sizeof(double));
    o->Ps = (double *)xcalloc(DN, sizeof(double));
    o->acc = NULL; o->phx = NULL; o->pheta = NULL;
}

static void free_forcing(forcing_out *o)
{
    free(o->xi); free(o->P); free(o->xs); free(o->Ps);
}

/* Initial populations (eq_bc_f_bar) on every fluid cell, lambda = dt = 1:
 * f-bar_i = (1 + 1/2) f^eq_i(eps, rho_0, v_0) - (1/2) f^*_i(eps, rho_0, v_0 + a_0),
 * with a_0, Phi^ext_0, Phi^eta_0 from the initial fields as the flowchart prescribes. */
static void init_populations(orc_solver *S)
{
    int D = S->D, Q = S->Q, i, a;
    long n, N = S->N;
    forcing_out o;
    for (n = 0; n < N; ++n) {
        S->rho[n] = S->solid[n] ? 0.0 : (S->p.rho_init ? S->p.rho_init[n] : S->p.rho0);
        for (a = 0; a < D; ++a)
            S->v[a * N + n] = S->solid[n] ? 0.0 : (S->p.v_init ? S->p.v_init[a * N + n] : 0.0);
    }
    alloc_forcing(D * N, &o);
    forcing(S, S->rho, S->v, S->rho, S->v, &o);
    for (n = 0; n < N; ++n) {
        double xi[3], P[3], xs[3], Ps[3], feq[ORC_MAXQ], fs[ORC_MAXQ];
        if (S->solid[n]) {
            for (i = 0; i < Q; ++i) S->F[(long)i * N + n] = 0.0;
            continue;
        }
        for (a = 0; a < D; ++a) {
            xi[a] = o.xi[a * N + n]; P[a] = o.P[a * N + n];
            xs[a] = o.xs[a * N + n]; Ps[a] = o.Ps[a * N + n];
        }
        product_form(D, Q, (const int (*)[3])S->c, S->eps[n], S->rho[n], xi, P, feq);
        product_form(D, Q, (const int (*)[3])S->c, S->eps[n], S->rho[n], xs, Ps, fs);
        for (i = 0; i < Q; ++i) S->F[(long)i * N + n] = 1.5 * feq[i] - 0.5 * fs[i];
    }
    free_forcing(&o);
    memcpy(S->prho, S->rho, sizeof(double) * (size_t)N);
    memcpy(S->pv1, S->v, sizeof(double) * (size_t)(D * N));
    memcpy(S->pv, S->v, sizeof(double) * (size_t)(D * N));
    S->have_prev = 1;
    S->t = 0;
}

/* Reconstruction of all post-advection populations of the velocity and pressure nodes from
 * the boundary state (rho_b, v_b) and acceleration a_b, with lambda = dt = 1 and
 * f^tgt = f^eq(eps_b, rho_b, v_b), f^* = f^eq(eps_b, rho_b, v_b + a_b):
 *   equilibrium, eq. (eq_bc_f_bar):  f-bar_i = (3/2) f^tgt_i - (1/2) f^*_i;
 *   NEEM, eqs. (NEEM_bc_f_bar), (zeta_beta_NEEM), with the inner node x_f:
 *     f-bar_i = zeta f-bar_i(x_f) + (3/2)[f^tgt_i - zeta f^eq_i(x_f)] + (1/2)[zeta f^*_i(x_f) - f^*_i];
 *   TMS, steps 1-3 of Sec. 3.4.4: local (rho_loc, v_loc) from the known populations, then
 *     f-bar_i = (f^tgt_i - f^loc_i)/(1 - beta_b) + (3/2) f^tgt_i - (1/2) f^*_i for i in P-,
 *     f-bar_i = (f^tgt_i - f^loc_i)/(1 - beta_b) + f-bar_i for the others. */
static void reconstruct_boundaries(orc_solver *S, const double *acc)
{
    int D = S->D, Q = S->Q, a, i, nv[3];
    long k, N = S->N;
    for (k = 0; k < S->nb; ++k) {
        long b = S->bnodes[k];
        double e = S->eps[b], rho = S->rho[b], vb[3], vs[3];
        double ftgt[ORC_MAXQ], fst[ORC_MAXQ];
        if (S->p.bc_type[b] != 1 && S->p.bc_type[b] != 2) continue;
        bc_normal_vec(S, b, nv);
        for (a = 0; a < D; ++a) {
            vb[a] = S->v[a * N + b];
            vs[a] = vb[a] + acc[a * N + b];
        }
        equilibrium_at(S, e, rho, vb, ftgt);
        equilibrium_at(S, e, rho, vs, fst);
        if (S->p.bc_scheme == 0) {
            for (i = 0; i < Q; ++i) S->F[(long)i * N + b] = 1.5 * ftgt[i] - 0.5 * fst[i];
        } else if (S->p.bc_scheme == 1) {
            long f = bc_inner(S, b, nv);
            double ef = S->eps[f], rf = S->rho[f], vf[3], vfs[3];
            double feqf[ORC_MAXQ], fstf[ORC_MAXQ];
            double zeta = (1.0 - S->beta[f]) / (1.0 - S->beta[b]);
            for (a = 0; a < D; ++a) {
                vf[a] = S->v[a * N + f];
                vfs[a] = vf[a] + acc[a * N + f];
            }
            equilibrium_at(S, ef, rf, vf, feqf);
            equilibrium_at(S, ef, rf, vfs, fstf);
            for (i = 0; i < Q; ++i)
                S->F[(long)i * N + b] = (zeta * S->F[(long)i * N + f] +
                                         1.5 * (ftgt[i] - zeta * feqf[i])) +
                                        0.5 * (zeta * fstf[i] - fst[i]);
        } else {
            double omb = 1.0 - S->beta[b], s0 = 0.0, s1[3] = {0.0, 0.0, 0.0}, rloc, vloc[3];
            double floc[ORC_MAXQ];
            for (i = 0; i < Q; ++i) {
                double d;
                if (in_pminus(S, i, nv)) continue;
                d = (S->F[(long)i * N + b] - 1.5 * ftgt[i]) + 0.5 * fst[i];
                s0 = s0 + d;
                for (a = 0; a < D; ++a) s1[a] = s1[a] + (double)S->c[i][a] * d;
            }
            rloc = (e * rho + omb * s0) / e;
            for (a = 0; a < D; ++a) vloc[a] = (rho * vb[a] + omb * s1[a]) / rloc;
            equilibrium_at(S, e, rloc, vloc, floc);
            for (i = 0; i < Q; ++i) {
                double neq = (ftgt[i] - floc[i]) / omb;
                if (in_pminus(S, i, nv)) S->F[(long)i * N + b] = neq + (1.5 * ftgt[i] - 0.5 * fst[i]);
                else S->F[(long)i * N + b] = neq + S->F[(long)i * N + b];
            }
        }
    }
}

/* Second-order velocity evaluation (App. F): starting from the one-shot velocity, Picard
 * iterations of the implicit relation c_1 v + c_2 |v| v = v_0 + Delta_nu(rho v / eps) / (2 rho):
 *   s^(k) = v_0 + Delta_nu(rho v^(k) / eps) / (2 rho),  v^(k+1) = 2 s^(k) / (c_1 + sqrt(c_1^2 +
 *   4 c_2 |s^(k)|)), optionally under-relaxed, v^(k+1) <- (1 - omega) v^(k) + omega v^(k+1);
 * a fixed number of iterations, every cell from the previous iterate (Jacobi order).  Boundary
 * velocity and pressure nodes keep their boundary velocity. */
static void picard_velocity(orc_solver *S)
{
    int D = S->D, a, it;
    long n, N = S->N;
    double omega = S->p.picard_omega;
    double *vn = S->vw;
    for (it = 0; it < S->p.picard_iters; ++it) {
        momentum_over_eps(S, S->rho, S->v);
#pragma omp parallel for private(a) schedule(static)
        for (n = 0; n < N; ++n) {
            double dn[3], sv[3], vk[3];
            int bnode = S->p.bc_type && (S->p.bc_type[n] == 1 || S->p.bc_type[n] == 2);
            if (S->solid[n] || bnode) {
                for (a = 0; a < D; ++a) vn[a * N + n] = S->v[a * N + n];
                continue;
            }
            delta_nu_field(S, S->m, n, dn);
            for (a = 0; a < D; ++a) sv[a] = S->v0[a * N + n] + dn[a] / (2.0 * S->rho[n]);
            drag_solve(D, sv, S->muD[n], S->muF[n], vk);
            for (a = 0; a < D; ++a)
                vn[a * N + n] = omega == 1.0 ? vk[a]
                                             : (1.0 - omega) * S->v[a * N + n] + omega * vk[a];
        }
        memcpy(S->v, vn, sizeof(double) * (size_t)(D * N));
    }
}

/* Moments of the current state: outflow copies, bulk moments and drag solve, boundary
 * records, velocity correction. */
static void compute_moments(orc_solver *S)
{
    apply_outflow(S);
    moments_v1(S);
    boundary_records(S);
    correct_velocity(S);
    boundary_velocity(S);
    if (S->p.picard_iters > 0) picard_velocity(S);
}

/* Post-collision populations (dicrete_scheme, momentum_rate) with lambda = dt = 1:
 * f-bar^pc_i = f-bar_i + 2 beta (f^eq_i - f-bar_i) + (1 - beta)(f^*_i - f^eq_i). */
static void collide_cell(const orc_solver *S, long n, const forcing_out *o, double *fpc)
{
    int D = S->D, Q = S->Q, i, a;
    long N = S->N;
    double xi[3], P[3], xs[3], Ps[3], feq[ORC_MAXQ], fs[ORC_MAXQ];
    double beta = S->beta[n];
    for (a = 0; a < D; ++a) {
        xi[a] = o->xi[a * N + n]; P[a] = o->P[a * N + n];
        xs[a] = o->xs[a * N + n]; Ps[a] = o->Ps[a * N + n];
    }
    product_form(D, Q, (const int (*)[3])S->c, S->eps[n], S->rho[n], xi, P, feq);
    product_form(D, Q, (const int (*)[3])S->c, S->eps[n], S->rho[n], xs, Ps, fs);
    for (i = 0; i < Q; ++i) {
        double f = S->F[(long)i * N + n];
        fpc[i] = (f + (2.0 * beta) * (feq[i] - f)) + (1.0 - beta) * (fs[i] - feq[i]);
    }
}

/* One full step: moments, velocity correction, forcing, collision, then streaming with halfway
 * bounce-back at solid cells and periodic wrap (the paper's collide-and-stream, dicrete_scheme). */
static void step_once(orc_solver *S)
{
    int D = S->D, Q = S->Q, i;
    long n, N = S->N;
    forcing_out o;
    double *tmp;
    compute_moments(S);
    alloc_forcing(D * N, &o);
    if (S->nb) o.acc = (double *)xcalloc(D * N, sizeof(double));
    if (S->p.lagged && S->have_prev) forcing(S, S->rho, S->v, S->prho, S->pv, &o);
    else forcing(S, S->rho, S->v, S->rho, S->v, &o);
    if (S->nb) reconstruct_boundaries(S, o.acc);
    /* every destination slot is written by exactly one cell: the loop needs no ordering */
#pragma omp parallel for private(i) schedule(static)
    for (n = 0; n < N; ++n) {
        double fpc[ORC_MAXQ];
        if (S->solid[n]) continue;
        collide_cell(S, n, &o, fpc);
        for (i = 0; i < Q; ++i) {
            long y = shift3(S, n, S->c[i]);
            if (S->solid[y]) S->G[(long)S->opp[i] * N + n] = fpc[i];
            else S->G[(long)i * N + y] = fpc[i];
        }
    }
    free_forcing(&o);
    memcpy(S->prho, S->rho, sizeof(double) * (size_t)N);
    memcpy(S->pv1, S->v1, sizeof(double) * (size_t)(D * N));
    memcpy(S->pv, S->v, sizeof(double) * (size_t)(D * N));
    S->have_prev = 1;
    tmp = S->F; S->F = S->G; S->G = tmp;
    S->t += 1;
}

int orc_step(orc_solver *S, long nsteps)
{
    long k;
    for (k = 0; k < nsteps; ++k) step_once(S);
    return 0;
}

long orc_time(const orc_solver *S) { return S->t; }

/* Threads of the per-cell passes (n <= 0: the OpenMP default); returns the count now in use. */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Macroscopic output of the current state: intrinsic density rho and corrected superficial
 * velocity v (steps v_(0), v_(1), v_final on the current populations).  Solid cells give 0.
 * v1_out (optional) receives the drag-solve velocity v^(1). */
void orc_moments(orc_solver *S, double *rho_out, double *v_out, double *v1_out)
{
    long N = S->N;
    int D = S->D;
    compute_moments(S);
    if (rho_out) memcpy(rho_out, S->rho, sizeof(double) * (size_t)N);
    if (v_out) memcpy(v_out, S->v, sizeof(double) * (size_t)(D * N));
    if (v1_out) memcpy(v1_out, S->v1, sizeof(double) * (size_t)(D * N));
}

/* The current populations; the unknown incoming populations of outflow nodes are the ones the
 * next step uses (the outflow copy is applied first). */
void orc_get_state(orc_solver *S, double *f_out)
{
    apply_outflow(S);
    memcpy(f_out, S->F, sizeof(double) * (size_t)(S->Q * S->N));
}

/* Replace the populations (natural layout [Q][N]); the lagged-mode history restarts. */
void orc_set_state(orc_solver *S, const double *f_in, long t)
{
    memcpy(S->F, f_in, sizeof(double) * (size_t)(S->Q * S->N));
    S->have_prev = 0;
    S->t = t;
}

/* Forcing diagnostics of the current state: acceleration a [D][N], Phi^ext [D][N],
 * Phi^eta [N] and the equilibrium arguments xi, P, xi*, P* [D][N] each (any may be NULL). */
void orc_forcing_fields(orc_solver *S, double *acc, double *phx, double *pheta, double *xi,
                        double *P, double *xs, double *Ps)
{
    int D = S->D;
    long N = S->N;
    forcing_out o;
    compute_moments(S);
    alloc_forcing(D * N, &o);
    o.acc = acc; o.phx = phx; o.pheta = pheta;
    forcing(S, S->rho, S->v, S->rho, S->v, &o);
    if (xi) memcpy(xi, o.xi, sizeof(double) * (size_t)(D * N));
    if (P) memcpy(P, o.P, sizeof(double) * (size_t)(D * N));
    if (xs) memcpy(xs, o.xs, sizeof(double) * (size_t)(D * N));
    if (Ps) memcpy(Ps, o.Ps, sizeof(double) * (size_t)(D * N));
    free_forcing(&o);
}

/* Delta_nu applied to an arbitrary vector field m [D][N] (diagnostic of the expanded form). */
void orc_delta_nu_field(orc_solver *S, const double *m_in, double *out)
{
    int D = S->D, a;
    long n, N = S->N;
    for (n = 0; n < N; ++n) {
        double dn[3] = {0.0, 0.0, 0.0};
        if (!S->solid[n]) delta_nu_field(S, m_in, n, dn);
        for (a = 0; a < D; ++a) out[a * N + n] = dn[a];
    }
}

/* The viscous term of eq. (accel_approx_boundary) at each face node of `nodes` (boundary
 * nodes with one normal), evaluated as in the boundary records from the velocity field v_in
 * [D][N] in place of the records' velocities.  Test diagnostic: the solver's v^(1) records are
 * overwritten (the next step recomputes them). */
void orc_boundary_viscous_term(orc_solver *S, const double *v_in, long nnodes, const long *nodes,
                               double *out)
{
    long k;
    int nv[3];
    memcpy(S->v1, v_in, sizeof(double) * (size_t)(S->D * S->N));
    for (k = 0; k < nnodes; ++k) {
        if (!S->p.bc_type || bc_normal_vec(S, nodes[k], nv) != 1) { out[k] = NAN; continue; }
        out[k] = bc_viscous_term(S, nodes[k], nv);
    }
}

/* Porosity derivatives as the oracle uses them: grad eps [D][N], Hessian [D*D][N]. */
void orc_porosity_derivatives(const orc_solver *S, double *ge, double *H)
{
    int D = S->D;
    long N = S->N;
    if (ge) memcpy(ge, S->ge, sizeof(double) * (size_t)(D * N));
    if (H) memcpy(H, S->H, sizeof(double) * (size_t)(D * D * N));
}

/* Post-collision populations of selected fluid cells of the current state, without advancing
 * (used to check one step at sampled cells of a large domain).  fpc_out is [ncells][Q]. */
void orc_post_collision(orc_solver *S, long ncells, const long *cells, double *fpc_out)
{
    int D = S->D, Q = S->Q;
    long k, N = S->N;
    forcing_out o;
    compute_moments(S);
    alloc_forcing(D * N, &o);
    forcing(S, S->rho, S->v, S->rho, S->v, &o);
    for (k = 0; k < ncells; ++k) {
        long n = cells[k];
        if (n < 0 || n >= N || S->solid[n]) {
            int i;
            for (i = 0; i < Q; ++i) fpc_out[k * Q + i] = 0.0;
            continue;
        }
        collide_cell(S, n, &o, fpc_out + k * Q);
    }
    free_forcing(&o);
}

/* Global statistics of the current state (Sec. 4.2's steady-state measure and the
 * conservation sums), in FP64:
 *   out[0] total mass sum_x sum_i f-bar_i;  out[1..3] sum_x rho v;  out[4] max |v|;
 *   out[5] sum |v - v_snap|^2;  out[6] sum |v_snap|^2;  out[7] number of fluid cells whose
 *   populations or velocity are not finite.
 * The snapshot then takes the current v. */
void orc_stats(orc_solver *S, double *out)
{
    int D = S->D, Q = S->Q, i, a;
    long n, N = S->N;
    double mass = 0.0, mom[3] = {0.0, 0.0, 0.0}, vmax = 0.0, d2 = 0.0, s2 = 0.0, bad = 0.0;
    compute_moments(S);
    for (n = 0; n < N; ++n) {
        double cell = 0.0, vv = 0.0;
        if (S->solid[n]) continue;
        for (i = 0; i < Q; ++i) cell = cell + S->F[(long)i * N + n];
        mass = mass + cell;
        for (a = 0; a < D; ++a) {
            double va = S->v[a * N + n], sa = S->vsnap[a * N + n];
            mom[a] = mom[a] + S->rho[n] * va;
            vv = vv + va * va;
            d2 = d2 + (va - sa) * (va - sa);
            s2 = s2 + sa * sa;
        }
        if (!isfinite(cell) || !isfinite(vv)) bad = bad + 1.0;   /* each cell counts once */
        if (isfinite(vv) && sqrt(vv) > vmax) vmax = sqrt(vv);
    }
    out[0] = mass;
    out[1] = mom[0]; out[2] = mom[1]; out[3] = mom[2];
    out[4] = vmax; out[5] = d2; out[6] = s2; out[7] = bad;
    memcpy(S->vsnap, S->v, sizeof(double) * (size_t)(D * N));
}
