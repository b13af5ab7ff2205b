/*
 * lbem_oracle.c -- plain, slow, FP64 reference implementation of the
 * pseudo-vector lattice-BGK scheme for Maxwell's equations in heterogeneous
 * media (Hanasoge, Succi & Orszag, "Lattice Boltzmann Method for
 * Electromagnetic Wave Propagation", arXiv:1108.2651).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code with the HIP path.
 *
 * Each population carries the FULL D x D tensor g_{i,alpha,beta} (diagonal
 * and both triangles), exactly as the paper writes it (Section "Lattice BGK
 * formulation"), with no reduction to pseudo-vector components, no fusion
 * and no blocking.  One time step is: moments -> equilibrium -> source ->
 * BGK collision (eq. COLLI) -> streaming (eq. STREAM) into a second buffer.
 *
 * Readings of the paper taken here (listed with reasons in the design notes):
 *  - c^2 in the equilibrium is the per-axis second moment of the weights,
 *    c_L^2 = sum_i w_i c_{i,gamma}^2 = (1-w0)/D (the 6+1 example of the
 *    lattice section fixes the per-axis meaning).
 *  - The magnetic field entering the equilibrium is Bbar = K/(D-1), with
 *    K_beta = sum_alpha sum_i c_{i,alpha} g_{i,alpha,beta}: eq. relate.2
 *    puts each B_beta into (D-1) first moments; Bbar is their symmetric
 *    mean.  The physical field reported is B = K and the Maxwell speed is
 *    c_M^2 = c_L^2/(D-1) (identical readings in 2D, where D-1 = 1).
 *  - The medium: c_L^2(x) = (1 - w0_vac)/(D eps_r mu_r), i.e. the rest
 *    weight w0(x) = 1 - D c_L^2(x) realises the local light speed
 *    (weights of the lattice section); w0 must lie in [0,1).
 *  - Source S_gamma = c_M^2 eps_{gamma,beta,kappa} B_beta d_kappa ln mu
 *    - j_gamma/eps_abs (Maxwell section; the polarisation convolution is
 *    omitted as the paper itself does), eps_abs = eps_r/c_vac^2, the
 *    gradient by periodic central differences.
 *  - Macroscopic variables come from the plain pre-collision sums; the
 *    source of step t uses B(t) and j(x,t); initial populations are the
 *    equilibrium of the initial fields.
 *  - 3D velocity order 0,+x,+y,+z,-x,-y,-z; 2D order of the paper
 *    (0,(1,0),(0,1),(-1,0),(0,-1)).
 *  - Non-periodic faces (the paper treats periodic boxes only and leaves
 *    other boundaries open): a wall sits half a cell outside the first and
 *    last cell of an axis.  A perfectly conducting (PEC) wall is the mirror
 *    image of the box: the population that would leave through the face
 *    re-enters the same cell along the opposite velocity, with each tensor
 *    component transformed as a tensor under the reflection of that axis
 *    (sign -1 where alpha or beta is the normal axis), so tangential E is odd
 *    and normal E even about the wall.  A PMC wall takes the opposite sign.
 *    Beside a wall the medium is mirrored too (the ln mu gradient uses the
 *    cell itself for the missing neighbour).
 *  - Absorbing layer: after collision every population of a cell is
 *    multiplied by 1 - sigma(x); E and B decay at the same rate, so the
 *    layer's electric and magnetic losses stay in the ratio eps : mu (an
 *    impedance-matched absorber).
 *  - Anisotropic media (the lattice section notes that different weights
 *    for particles moving along different axes model them): per-axis
 *    moving weights w_a, per-axis second moments s_a = 2 w_a, rest weight
 *    w0 = 1 - sum_a s_a, and c^2 in the equilibrium their mean (1/D) sum_a
 *    s_a.  The equilibrium keeps its form (w_i/c^2)[Lambda + c_ia Bbar_b -
 *    c_ib Bbar_a] with these weights; Bbar generalises K/(D-1) so that the
 *    equilibrium carries the cell's K: Bbar_b = K_b / sum_{a != b} r_a with
 *    r_a = 2 w_a / c^2 (all r_a = 1 when isotropic).  The equilibrium is
 *    then the orthogonal projection onto the conserved moments in the 1/w_i
 *    inner product, so at tau = 1/2 the collision is an isometry and Q_c is
 *    conserved wherever the ratios r_a are uniform.  A wave along axis a
 *    polarised along b travels at c^2 = s_a^2/(s_a + s_b) in 3D and at s_a
 *    in 2D (isotropic: s/(D-1)).  Per cell the user gives factors f_a > 0 on
 *    the isotropic c_L^2: s_a = f_a c_L^2; eps_abs becomes (D-1)/(mu c^2).
 *    Equal factors give the isotropic scheme.
 *  - Frequency-dispersive permittivity (the convolution term of the source,
 *    which the paper defers to auxiliary differential equations): one
 *    Lorentz pole per cell, chi(w) = wp2 / (w02 - w^2 - i gamma w), relative
 *    to the cell's permittivity, in lattice units.  Auxiliary fields P (the
 *    polarisation in units of E) at integer times and J = dP/dt at half
 *    times: J(t+1/2) = [(1 - gamma/2) J(t-1/2) + wp2 E(t) - w02 P(t)] /
 *    (1 + gamma/2), P(t+1) = P(t) + J(t+1/2).  The polarisation source of
 *    step t, which the scheme integrates over [t, t+1], is -J(t+1/2)
 *    (leapfrog: E at integer, J at half-integer times).  It enters the rest
 *    particle only, T_{0,a,b} = -(1/c^2) eps_{g a b} S_g: the same change of
 *    E and no first moment, but unlike the w_i-weighted injection (which adds
 *    (c^2/2) times the lattice Laplacian of S(t) alone to the three-level form
 *    of the update) it enters as S(t) - S(t-1), so the coupled update is the
 *    centred leapfrog of E'' = c^2 lap E - P'' and stays stable; the
 *    w_i-weighted form pumps one polariton branch.  P and J start at zero.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EUNSTABLE (-3)
#define ORC_ESTATE (-6)

typedef struct {
    int D, Q;
    long nx, ny, nz, n;
    double tau, w0_vac;
    int c[7][3];          /* lattice velocities c_{i,alpha} */
    double *cL2;          /* per-axis lattice c^2 (the paper's c^2) */
    double *w0;           /* rest weight */
    double *eps_abs;      /* absolute permittivity (vacuum mu = 1) */
    double *mu_r;         /* relative permeability */
    double *dlnmu;        /* [3][n] central-difference gradient of ln mu */
    double *g, *gs;       /* [n][Q][D][D] populations, streamed copy */
    double *jd;           /* [3][n] current-density footprint (weights) */
    double *keep;         /* [n] 1 - sigma of the absorbing layer, or NULL */
    double *wax;          /* [3][n] per-axis moving weights (anisotropic), or NULL */
    double *ade;          /* [3][n] wp2, w02, gamma of the Lorentz pole, or NULL */
    double *pol, *pcur;   /* [3][n] P and J (per field component) */
    int bc[3];            /* per axis: 0 periodic, 1 PEC wall, 2 PMC wall */
    long t;
    int have_medium, have_fields, has_mu;
} orc_t;

/* Levi-Civita symbol over three indices. */
static int levi(int a, int b, int c)
{
    if (a == b || b == c || a == c) return 0;
    if ((a == 0 && b == 1 && c == 2) || (a == 1 && b == 2 && c == 0) ||
        (a == 2 && b == 0 && c == 1))
        return 1;
    return -1;
}

static void velocities(int D, int c[7][3])
{
    memset(c, 0, sizeof(int) * 21);
    if (D == 2) {
        /* counter-clockwise order of the lattice section */
        c[1][0] = 1; c[2][1] = 1; c[3][0] = -1; c[4][1] = -1;
    } else {
        c[1][0] = 1; c[2][1] = 1; c[3][2] = 1;
        c[4][0] = -1; c[5][1] = -1; c[6][2] = -1;
    }
}

static double weight(int i, double w0, int D)
{
    /* rest particle w0, moving particles (1-w0)/(2D) */
    return i == 0 ? w0 : (1.0 - w0) / (2.0 * D);
}

/* isotropic weights of all velocities from the rest weight */
static void iso_weights(int D, double w0, double* w)
{
    for (int i = 0; i < 2 * D + 1; ++i) w[i] = weight(i, w0, D);
}

static long wrap(long v, long n) { v %= n; return v < 0 ? v + n : v; }

static long neighbour(const orc_t* o, long x, const int* d, int sign)
{
    long ix = x % o->nx, iy = (x / o->nx) % o->ny, iz = x / (o->nx * o->ny);
    ix = wrap(ix + sign * d[0], o->nx);
    iy = wrap(iy + sign * d[1], o->ny);
    iz = wrap(iz + sign * d[2], o->nz);
    return ix + o->nx * (iy + o->ny * iz);
}

/* Neighbour for the ln mu gradient: beyond a wall the mirror image of the
 * missing cell is the cell itself. */
static long medium_neighbour(const orc_t* o, long x, int k, int sign)
{
    long ix = x % o->nx, iy = (x / o->nx) % o->ny, iz = x / (o->nx * o->ny);
    long v[3] = {ix, iy, iz}, nn[3] = {o->nx, o->ny, o->nz};
    long w = v[k] + sign;
    if (o->bc[k] != 0 && (w < 0 || w >= nn[k])) w = v[k];
    v[k] = wrap(w, nn[k]);
    return v[0] + o->nx * (v[1] + o->ny * v[2]);
}

#define GI(o, x, i, a, b) ((((size_t)(x) * (o)->Q + (i)) * (o)->D + (a)) * (o)->D + (b))

/* Bbar from K: Bbar_b = K_b / sum_{a != b} 2 w_a / c^2 (K/(D-1) when isotropic);
 * w holds the weights of all velocities, velocity 1+a moving along +a. */
static void bbar_of(int D, const double* w, double cl2, const double* K, double* Bbar)
{
    for (int b = 0; b < D; ++b) {
        double rs = 0.0;
        for (int a = 0; a < D; ++a)
            if (a != b) rs += 2.0 * w[1 + a] / cl2;
        Bbar[b] = K[b] / rs;
    }
}

/* weights of all velocities at cell x (per-axis when the medium is anisotropic) */
static void cell_weights(const orc_t* o, long x, double* w)
{
    iso_weights(o->D, o->w0[x], w);
    if (o->wax)
        for (int i = 1; i < o->Q; ++i)
            for (int a = 0; a < o->D; ++a)
                if (o->c[i][a] != 0) w[i] = o->wax[a * o->n + x];
}

/* ------------------------------------------------------------------------
 * Equilibrium of eq. distrib.func:
 *   g0_{i,a,b} = (w_i/c^2) [ Lambda_{a,b} + c_{i,a} Bbar_b - c_{i,b} Bbar_a ]
 * The wedge term is evaluated as one difference so that the result is
 * exactly antisymmetric in (a,b) under IEEE arithmetic.
 * ------------------------------------------------------------------------ */
static void equilibrium(int D, const int c[7][3], const double* w, double cl2,
                        const double* Lam, const double* Bbar, double* out)
{
    int Q = 2 * D + 1;
    for (int i = 0; i < Q; ++i) {
        double wc = w[i] / cl2;
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) {
                double wedge = c[i][a] * Bbar[b] - c[i][b] * Bbar[a];
                out[(i * D + a) * D + b] = wc * (Lam[a * D + b] + wedge);
            }
    }
}

/* Moments of one cell: rho_{ab} = sum_i g_iab (relate.1 before scaling),
 * K_b = sum_a sum_i c_ia g_iab (contracted first moment, relate.2). */
static void moments(int D, const int c[7][3], const double* gc, double* rho, double* K)
{
    int Q = 2 * D + 1;
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
            double s = 0.0;
            for (int i = 0; i < Q; ++i) s += gc[(i * D + a) * D + b];
            rho[a * D + b] = s;
        }
    for (int b = 0; b < D; ++b) {
        double s = 0.0;
        for (int a = 0; a < D; ++a)
            for (int i = 0; i < Q; ++i) s += c[i][a] * gc[(i * D + a) * D + b];
        K[b] = s;
    }
}

/* E_gamma = -1/2 eps_{gamma a b} Lambda_{ab} (Levi-Civita recovery). */
static void efield(int D, const double* Lam, double* E)
{
    for (int gm = 0; gm < 3; ++gm) {
        double s = 0.0;
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) s += levi(gm, a, b) * Lam[a * D + b];
        E[gm] = -0.5 * s;
    }
}

/* One cell's collision (eq. COLLI) with tensor source
 * T_{i,a,b} = -(w_i/c^2) eps_{gamma a b} S_gamma. */
static void collide_cell(int D, const int c[7][3], const double* w, double cl2, double tau,
                         const double* gc, const double* S, double* out)
{
    int Q = 2 * D + 1;
    double rho[9], K[3], Lam[9], Bbar[3], geq[63];
    moments(D, c, gc, rho, K);
    for (int k = 0; k < D * D; ++k) Lam[k] = cl2 * rho[k];
    bbar_of(D, w, cl2, K, Bbar);
    equilibrium(D, c, w, cl2, Lam, Bbar, geq);
    double om = 1.0 / tau;
    for (int i = 0; i < Q; ++i) {
        double wc = w[i] / cl2;
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) {
                double es = 0.0;
                for (int gm = 0; gm < 3; ++gm) es += levi(gm, a, b) * S[gm];
                double T = -wc * es;
                int k = (i * D + a) * D + b;
                out[k] = (1.0 - om) * gc[k] + om * geq[k] + T;
            }
    }
}

/* ------------------------------------------------------------------------ */

orc_t* orc_create(int D, long nx, long ny, long nz, double tau, double w0_vac)
{
    if ((D != 2 && D != 3) || nx < 1 || ny < 1 || nz < 1 || (D == 2 && nz != 1))
        return NULL;
    if (!(tau > 0.0) || !(w0_vac >= 0.0 && w0_vac < 1.0)) return NULL;
    orc_t* o = (orc_t*)calloc(1, sizeof(orc_t));
    if (!o) return NULL;
    o->D = D; o->Q = 2 * D + 1;
    o->nx = nx; o->ny = ny; o->nz = nz; o->n = nx * ny * nz;
    o->tau = tau; o->w0_vac = w0_vac;
    velocities(D, o->c);
    size_t n = (size_t)o->n, pop = n * o->Q * D * D;
    o->cL2 = (double*)calloc(n, sizeof(double));
    o->w0 = (double*)calloc(n, sizeof(double));
    o->eps_abs = (double*)calloc(n, sizeof(double));
    o->mu_r = (double*)calloc(n, sizeof(double));
    o->dlnmu = (double*)calloc(3 * n, sizeof(double));
    o->g = (double*)calloc(pop, sizeof(double));
    o->gs = (double*)calloc(pop, sizeof(double));
    o->jd = (double*)calloc(3 * n, sizeof(double));
    if (!o->cL2 || !o->w0 || !o->eps_abs || !o->mu_r || !o->dlnmu || !o->g || !o->gs ||
        !o->jd) {
        free(o->cL2); free(o->w0); free(o->eps_abs); free(o->mu_r); free(o->dlnmu);
        free(o->g); free(o->gs); free(o->jd); free(o);
        return NULL;
    }
    return o;
}

void orc_destroy(orc_t* o)
{
    if (o) {
        free(o->keep);
        free(o->wax);
        free(o->ade);
        free(o->pol);
        free(o->pcur);
    }
    if (!o) return;
    free(o->cL2); free(o->w0); free(o->eps_abs); free(o->mu_r); free(o->dlnmu);
    free(o->g); free(o->gs); free(o->jd); free(o);
}

int orc_set_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
    return omp_get_max_threads();
#else
    (void)k;
    return 1;
#endif
}

/* Medium: c_L^2 = (1-w0_vac)/(D eps_r mu_r); w0 = 1 - D c_L^2 in [0,1). */
int orc_set_medium(orc_t* o, const double* eps_r, const double* mu_r)
{
    int D = o->D;
    double cvac2 = (1.0 - o->w0_vac) / (double)(D * (D - 1));
    o->has_mu = 0;
    free(o->wax);
    o->wax = NULL;
    for (long x = 0; x < o->n; ++x) {
        double e = eps_r[x], m = mu_r ? mu_r[x] : 1.0;
        if (!(e > 0.0) || !(m > 0.0) || !isfinite(e) || !isfinite(m)) return ORC_EINVAL;
        double cl2 = (1.0 - o->w0_vac) / ((double)D * e * m);
        double w0 = 1.0 - D * cl2;
        if (!(w0 >= 0.0 && w0 < 1.0)) return ORC_EUNSTABLE;
        o->cL2[x] = cl2;
        o->w0[x] = w0;
        o->eps_abs[x] = e / cvac2;
        o->mu_r[x] = m;
        if (m != 1.0) o->has_mu = 1;
    }
    for (long x = 0; x < o->n; ++x)
        for (int k = 0; k < 3; ++k) {
            if (k >= D) { o->dlnmu[k * o->n + x] = 0.0; continue; }
            long xp = medium_neighbour(o, x, k, +1), xm = medium_neighbour(o, x, k, -1);
            o->dlnmu[k * o->n + x] = 0.5 * (log(o->mu_r[xp]) - log(o->mu_r[xm]));
        }
    o->have_medium = 1;
    return ORC_OK;
}

/* Initial populations: equilibrium of E0, B0 with Lambda_ab = -eps_{gab} E_g. */
int orc_init_fields(orc_t* o, const double* E, const double* B)
{
    if (!o->have_medium) return ORC_ESTATE;
    int D = o->D;
    long n = o->n;
    for (long x = 0; x < n; ++x) {
        double Lam[9], Bbar[3];
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) {
                double s = 0.0;
                for (int gm = 0; gm < 3; ++gm) s += levi(gm, a, b) * E[gm * n + x];
                Lam[a * D + b] = -s;
            }
        double w[7], Bp[3] = {B[x], B[n + x], B[2 * n + x]};
        cell_weights(o, x, w);
        bbar_of(D, w, o->cL2[x], Bp, Bbar);
        equilibrium(D, o->c, w, o->cL2[x], Lam, Bbar, &o->g[GI(o, x, 0, 0, 0)]);
    }
    o->t = 0;
    o->have_fields = 1;
    if (o->ade) {
        memset(o->pol, 0, sizeof(double) * 3 * n);
        memset(o->pcur, 0, sizeof(double) * 3 * n);
    }
    return ORC_OK;
}

/* Current footprint: j_comp(cell) += weight (amplitude series given per step). */
int orc_set_source(orc_t* o, long m, const int* comp, const long* cell, const double* weight)
{
    memset(o->jd, 0, sizeof(double) * 3 * o->n);
    for (long k = 0; k < m; ++k) {
        if (comp[k] < 0 || comp[k] > 2 || cell[k] < 0 || cell[k] >= o->n) return ORC_EINVAL;
        if (o->D == 2 && comp[k] != 2) return ORC_EINVAL;
        o->jd[comp[k] * o->n + cell[k]] += weight[k];
    }
    return ORC_OK;
}

/* Pre-collision macroscopic fields of one cell (E, B = K). */
static void cell_fields(const orc_t* o, long x, double* E, double* B)
{
    int D = o->D;
    double rho[9], K[3], Lam[9];
    moments(D, o->c, &o->g[GI(o, x, 0, 0, 0)], rho, K);
    for (int k = 0; k < D * D; ++k) Lam[k] = o->cL2[x] * rho[k];
    efield(D, Lam, E);
    B[0] = B[1] = B[2] = 0.0;
    for (int b = 0; b < D; ++b) B[b] = K[b];
}

int orc_step(orc_t* o, long nsteps, const double* amp)
{
    if (!o->have_medium || !o->have_fields) return ORC_ESTATE;
    int D = o->D, Q = o->Q;
    long n = o->n;
    for (long s = 0; s < nsteps; ++s) {
        double a = amp ? amp[s] : 0.0;
#pragma omp parallel for schedule(static)
        for (long x = 0; x < n; ++x) {
            double E[3], B[3], S[3], Sp[3] = {0.0, 0.0, 0.0}, out[63];
            cell_fields(o, x, E, B);
            double cM2 = o->cL2[x] / (double)(D - 1);
            for (int gm = 0; gm < 3; ++gm) {
                double mu_term = 0.0;
                if (o->has_mu)
                    for (int b = 0; b < 3; ++b)
                        for (int k = 0; k < 3; ++k)
                            mu_term += levi(gm, b, k) * B[b] * o->dlnmu[k * n + x];
                S[gm] = cM2 * mu_term - a * o->jd[gm * n + x] / o->eps_abs[x];
            }
            if (o->ade) {
                double wp2 = o->ade[x], w02 = o->ade[n + x], gam = o->ade[2 * n + x];
                for (int gm = 0; gm < 3; ++gm) {
                    double Jo = o->pcur[gm * n + x], Po = o->pol[gm * n + x];
                    double Jn = ((1.0 - 0.5 * gam) * Jo + wp2 * E[gm] - w02 * Po) / (1.0 + 0.5 * gam);
                    Sp[gm] = -Jn;
                    o->pcur[gm * n + x] = Jn;
                    o->pol[gm * n + x] = Po + Jn;
                }
            }
            double wv[7];
            cell_weights(o, x, wv);
            collide_cell(D, o->c, wv, o->cL2[x], o->tau, &o->g[GI(o, x, 0, 0, 0)], S, out);
            if (o->ade)   /* polarisation source: rest particle only */
                for (int a2 = 0; a2 < D; ++a2)
                    for (int b2 = 0; b2 < D; ++b2) {
                        double es = 0.0;
                        for (int gm = 0; gm < 3; ++gm) es += levi(gm, a2, b2) * Sp[gm];
                        out[a2 * D + b2] += -es / o->cL2[x];
                    }
            if (o->keep)
                for (int k = 0; k < Q * D * D; ++k) out[k] *= o->keep[x];
            /* streaming, eq. STREAM: g(x + c_i, t+1) = g'(x, t); through a wall
             * face: back into x along the opposite velocity, reflected */
            long v[3] = {x % o->nx, (x / o->nx) % o->ny, x / (o->nx * o->ny)};
            long nn[3] = {o->nx, o->ny, o->nz};
            for (int i = 0; i < Q; ++i) {
                int wall = -1;
                for (int a = 0; a < D; ++a)
                    if (o->c[i][a] != 0 && o->bc[a] != 0 && (v[a] + o->c[i][a] < 0 || v[a] + o->c[i][a] >= nn[a]))
                        wall = a;
                if (wall < 0) {
                    long xd = neighbour(o, x, o->c[i], +1);
                    for (int k = 0; k < D * D; ++k) o->gs[GI(o, xd, i, 0, 0) + k] = out[i * D * D + k];
                } else {
                    int io = 0;
                    for (int j = 1; j < Q; ++j)
                        if (o->c[j][wall] == -o->c[i][wall]) io = j;
                    double flip = o->bc[wall] == 1 ? -1.0 : 1.0;
                    for (int a = 0; a < D; ++a)
                        for (int b = 0; b < D; ++b) {
                            double sg = (a == wall || b == wall) ? flip : -flip;
                            o->gs[GI(o, x, io, a, b)] = sg * out[(i * D + a) * D + b];
                        }
                }
            }
        }
        double* tmp = o->g; o->g = o->gs; o->gs = tmp;
        o->t += 1;
    }
    return ORC_OK;
}

/* Boundary kind of one axis (0 periodic, 1 PEC wall, 2 PMC wall); before the
 * medium is set, since the ln mu gradient beside a wall depends on it. */
int orc_set_boundary(orc_t* o, int axis, int kind)
{
    if (axis < 0 || axis >= o->D || kind < 0 || kind > 2) return ORC_EINVAL;
    if (o->have_medium) return ORC_ESTATE;
    o->bc[axis] = kind;
    return ORC_OK;
}

/* One Lorentz pole per cell (wp2, w02, gamma >= 0; wp2 == NULL removes the
 * dispersion); the auxiliary fields restart from zero. */
int orc_set_dispersion(orc_t* o, const double* wp2, const double* w02, const double* gamma)
{
    long n = o->n;
    if (!wp2) {
        free(o->ade); free(o->pol); free(o->pcur);
        o->ade = o->pol = o->pcur = NULL;
        return ORC_OK;
    }
    for (long x = 0; x < n; ++x) {
        double a = wp2[x], b = w02 ? w02[x] : 0.0, g = gamma ? gamma[x] : 0.0;
        if (!(a >= 0.0) || !(b >= 0.0) || !(g >= 0.0) || !isfinite(a) || !isfinite(b) || !isfinite(g))
            return ORC_EINVAL;
    }
    if (!o->ade) {
        o->ade = (double*)malloc(sizeof(double) * 3 * n);
        o->pol = (double*)calloc(3 * n, sizeof(double));
        o->pcur = (double*)calloc(3 * n, sizeof(double));
        if (!o->ade || !o->pol || !o->pcur) return ORC_ENOMEM;
    }
    for (long x = 0; x < n; ++x) {
        o->ade[x] = wp2[x];
        o->ade[n + x] = w02 ? w02[x] : 0.0;
        o->ade[2 * n + x] = gamma ? gamma[x] : 0.0;
    }
    memset(o->pol, 0, sizeof(double) * 3 * n);
    memset(o->pcur, 0, sizeof(double) * 3 * n);
    return ORC_OK;
}

/* Auxiliary fields P and J of the dispersion, component-major [3][n]. */
int orc_polarisation(const orc_t* o, double* P, double* J)
{
    if (!o->ade) return ORC_ESTATE;
    memcpy(P, o->pol, sizeof(double) * 3 * o->n);
    memcpy(J, o->pcur, sizeof(double) * 3 * o->n);
    return ORC_OK;
}

/* Anisotropy factors a[axis][x] > 0 on the isotropic c_L^2 of the medium just
 * set (set_medium again restores isotropy). */
int orc_set_anisotropy(orc_t* o, const double* fac)
{
    if (!o->have_medium) return ORC_ESTATE;
    int D = o->D;
    long n = o->n;
    for (long x = 0; x < n * D; ++x)
        if (!(fac[x] > 0.0) || !isfinite(fac[x])) return ORC_EINVAL;
    double* wax = (double*)calloc(3 * (size_t)n, sizeof(double));
    if (!wax) return ORC_ENOMEM;
    for (long x = 0; x < n; ++x) {
        double sum = 0.0;
        for (int a = 0; a < D; ++a) sum += fac[a * n + x] * o->cL2[x];
        double w0 = 1.0 - sum;
        if (!(w0 >= 0.0 && w0 < 1.0)) { free(wax); return ORC_EUNSTABLE; }
    }
    for (long x = 0; x < n; ++x) {
        double sum = 0.0;
        for (int a = 0; a < D; ++a) {
            double sa = fac[a * n + x] * o->cL2[x];
            wax[a * n + x] = 0.5 * sa;
            sum += sa;
        }
        o->w0[x] = 1.0 - sum;
        o->cL2[x] = sum / (double)D;
        o->eps_abs[x] = (double)(D - 1) / (o->mu_r[x] * o->cL2[x]);
    }
    free(o->wax);
    o->wax = wax;
    return ORC_OK;
}

/* Absorbing layer: per-cell sigma in [0,1) (NULL removes it). */
int orc_set_absorber(orc_t* o, const double* sigma)
{
    if (!sigma) {
        free(o->keep);
        o->keep = NULL;
        return ORC_OK;
    }
    for (long x = 0; x < o->n; ++x)
        if (!(sigma[x] >= 0.0 && sigma[x] < 1.0)) return ORC_EINVAL;
    if (!o->keep) o->keep = (double*)malloc(sizeof(double) * o->n);
    if (!o->keep) return ORC_ENOMEM;
    for (long x = 0; x < o->n; ++x) o->keep[x] = 1.0 - sigma[x];
    return ORC_OK;
}

/* E, B at the current time, component-major [3][n]. */
int orc_fields(const orc_t* o, double* E, double* B)
{
    if (!o->have_fields) return ORC_ESTATE;
    long n = o->n;
    for (long x = 0; x < n; ++x) {
        double e[3], b[3];
        cell_fields(o, x, e, b);
        for (int k = 0; k < 3; ++k) { E[k * n + x] = e[k]; B[k * n + x] = b[k]; }
    }
    return ORC_OK;
}

/* Diagnostics, sequential FP64 sums in cell order:
 *  out[0] EM energy sum(eps_abs |E|^2 + |B|^2/mu_r)  (energy of the
 *         heterogeneous-media subsection, with c the Maxwell speed)
 *  out[1] Q_c = sum_x c_L^2 sum_i sum_{a<b} g_iab^2 / w_i (rest skipped if w0=0)
 *  out[2] sum (div_h B)^2, central differences
 *  out[3] sum |B|^2 */
int orc_diag(const orc_t* o, double* out)
{
    if (!o->have_fields) return ORC_ESTATE;
    int D = o->D, Q = o->Q;
    long n = o->n;
    double* Bf = (double*)malloc(sizeof(double) * 3 * n);
    if (!Bf) return ORC_ENOMEM;
    double en = 0.0, qc = 0.0, dv = 0.0, bb = 0.0;
    for (long x = 0; x < n; ++x) {
        double e[3], b[3];
        cell_fields(o, x, e, b);
        for (int k = 0; k < 3; ++k) Bf[k * n + x] = b[k];
        double e2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
        double b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
        en += o->eps_abs[x] * e2 + b2 / o->mu_r[x];
        bb += b2;
        double q = 0.0, wv[7];
        cell_weights(o, x, wv);
        for (int i = 0; i < Q; ++i) {
            double w = wv[i];
            if (w == 0.0) continue;
            double s = 0.0;
            for (int a = 0; a < D; ++a)
                for (int bq = a + 1; bq < D; ++bq) {
                    double v = o->g[GI(o, x, i, a, bq)];
                    s += v * v;
                }
            q += s / w;
        }
        qc += o->cL2[x] * q;
    }
    for (long x = 0; x < n; ++x) {
        double d = 0.0;
        for (int k = 0; k < D; ++k) {
            int dd[3] = {0, 0, 0};
            dd[k] = 1;
            d += 0.5 * (Bf[k * n + neighbour(o, x, dd, +1)] - Bf[k * n + neighbour(o, x, dd, -1)]);
        }
        dv += d * d;
    }
    free(Bf);
    out[0] = en; out[1] = qc; out[2] = dv; out[3] = bb;
    return ORC_OK;
}

long orc_time(const orc_t* o) { return o->t; }
long orc_state_size(const orc_t* o) { return o->n * o->Q * o->D * o->D; }

int orc_get_state(const orc_t* o, double* out)
{
    memcpy(out, o->g, sizeof(double) * (size_t)orc_state_size(o));
    return ORC_OK;
}

int orc_set_state(orc_t* o, const double* in)
{
    memcpy(o->g, in, sizeof(double) * (size_t)orc_state_size(o));
    o->have_fields = 1;
    return ORC_OK;
}

/* Medium as prepared (for tests): c_L^2, w0, eps_abs, mu_r, dlnmu[3][n]. */
int orc_get_medium(const orc_t* o, double* cl2, double* w0, double* eps_abs, double* dlnmu)
{
    memcpy(cl2, o->cL2, sizeof(double) * o->n);
    memcpy(w0, o->w0, sizeof(double) * o->n);
    memcpy(eps_abs, o->eps_abs, sizeof(double) * o->n);
    memcpy(dlnmu, o->dlnmu, sizeof(double) * 3 * o->n);
    return ORC_OK;
}

/* Stand-alone single-cell pieces for the identity tests. */
int orc_equilibrium(int D, double w0, const double* Lam, const double* Bbar, double* out)
{
    int c[7][3];
    if (D != 2 && D != 3) return ORC_EINVAL;
    velocities(D, c);
    double w[7];
    iso_weights(D, w0, w);
    equilibrium(D, c, w, (1.0 - w0) / D, Lam, Bbar, out);
    return ORC_OK;
}

int orc_collide(int D, double w0, double tau, const double* g, const double* S, double* out)
{
    int c[7][3];
    if (D != 2 && D != 3) return ORC_EINVAL;
    velocities(D, c);
    double w[7];
    iso_weights(D, w0, w);
    collide_cell(D, c, w, (1.0 - w0) / D, tau, g, S, out);
    return ORC_OK;
}

int orc_velocities(int D, int* out)
{
    int c[7][3];
    if (D != 2 && D != 3) return ORC_EINVAL;
    velocities(D, c);
    for (int i = 0; i < 2 * D + 1; ++i)
        for (int a = 0; a < 3; ++a) out[i * 3 + a] = c[i][a];
    return ORC_OK;
}
