/*
 * FP64 CPU oracle of one multiphase lattice-Boltzmann time step.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header, table or helper with
 * the GPU library: lattice tables, the MRT matrix and its inverse are built
 * here from their definitions.
 *
 * One time step t -> t+1, in the order the paper states the method
 * (Sec. 2.1 Eq. 1-6, Sec. 2.2 Eq. 9-13, Sec. 2.4 Eq. 17):
 *   1. rho^k = sum_i f_i^k,  j^k = sum_i f_i^k e_i             (Eq. 4, Eq. 10)
 *   2. improved virtual density at solid nodes that touch fluid (Eq. 17)
 *   3. pseudopotential psi^k and U^k from the EOS               (Eq. 12)
 *   4. Shan-Chen / Zhang-Chen interaction force + body force     (Eq. 13)
 *   5. equilibrium velocity (bare j/rho; common velocity for two components)
 *   6. BGK or MRT collision, then exact-difference forcing      (Eq. 3, Eq. 5);
 *      D2Q9 MRT optionally with the surface-tension source C    (Eq. 14-16);
 *      or the central-moment (cascaded) collision with the
 *      consistent forcing term of the same moments               (Eq. 3, Eq. 7-8)
 *   7. streaming with halfway bounce-back at solid nodes        (Eq. 2);
 *      open boundaries: reservoir nodes at fixed density emit
 *      their rest equilibrium (the constant-pressure inlet and
 *      outlet of Sec. 3.4.3)
 * Macroscopic velocity output uses the half-force correction   (Eq. 6).
 *
 * State layout: f[(k*q + i)*N + n], n = (z*ny + y)*nx + x, x fastest; the
 * stored state is the post-streaming (pre-collision) population f(x, t).
 * Solid and reservoir nodes carry no populations (their entries are kept at
 * zero).  Mask values: 0 fluid, 1 solid, 2 and 3 reservoirs 0 and 1.
 *
 * The same source is compiled twice: with real_t = double (symbols oref_*)
 * and with real_t = double _Complex (symbols orefc_*).  The complex build
 * gives complex-step derivatives: an imaginary perturbation of a wetting
 * parameter or of the temperature propagates through the step, and every
 * branch (clamp, square-root argument test) is taken on the real part.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORACLE_CSTEP
#include <complex.h>
typedef double _Complex real_t;
#define RE(v) creal(v)
#define SQRT_R(v) csqrt(v)
#define API(name) orefc_##name
#else
typedef double real_t;
#define RE(v) (v)
#define SQRT_R(v) sqrt(v)
#define API(name) oref_##name
#endif

#define MAXQ 19
#define MAXC 2

/* Physical and numerical parameters of a run (plain data, host only). */
typedef struct {
    int lattice;          /* 0 = D2Q9, 1 = D3Q19                              */
    int nx, ny, nz;       /* domain; nz = 1 for D2Q9                         */
    int nc;               /* number of fluid components (1 or 2)             */
    int collision;        /* 0 = BGK, 1 = MRT, 2 = central moments (CLBM)   */
    int psi_kind[MAXC];   /* 0 = Carnahan-Starling EOS, 1 = psi = rho        */
    int wet_mode[MAXC];   /* 0 = phi * rho_ave, 1 = rho_ave - drho           */
    int common_velocity;  /* two components: 1 = common velocity u'         */
    double tau[MAXC];
    double mrt_s[MAXC][MAXQ];          /* relaxation rate of each moment row  */
    double eos_a[MAXC], eos_b[MAXC], eos_R[MAXC];
    double eos_T[MAXC], eos_T_im[MAXC]; /* temperature (imag part: cstep only) */
    double alpha[MAXC];
    double A[MAXC];                    /* Zhang-Chen weight A_kk              */
    double g[MAXC][MAXC];              /* interaction strengths g_kk'         */
    double body[3];                    /* body acceleration                   */
    double rho_min[MAXC], rho_max[MAXC]; /* virtual-density limiter bounds    */
    double kappa[MAXC];                /* surface-tension adjustment (D2Q9 MRT) */
    double res_rho[2][MAXC];           /* densities of reservoirs 0 and 1      */
} oref_params;

/* Node kinds of the mask: fluid, solid (bounce-back wall or grain), two
 * reservoirs and a convective outlet.  A reservoir node is an open boundary
 * held at fixed component densities res_rho[r][k]: a population that streams
 * in from it is 2 w_i res_rho - f*_opp(i)(x) (anti-bounce-back), and it enters
 * its neighbours' force gather and the virtual densities of solids with
 * psi(res_rho), like fluid.  A convective outlet node (one plane of the
 * slowest axis, fluid on its lower side) passes the flow out: a population
 * that streams in from it obeys the convective equation d f/dt + U d f/dn = 0
 * with U the mean outward velocity of the plane below (Sec. 3.4.2), and its
 * density is that of the fluid node below it (zero gradient).  Neither kind
 * is itself updated. */
#define NODE_FLUID 0
#define NODE_SOLID 1
#define NODE_CONV 4
#define IS_RES(v) ((v) == 2 || (v) == 3)

/* ------------------------------------------------------------------------ */
/* Lattice tables built from the definition of the velocity sets.           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int q, dim;
    int e[MAXQ][3];
    double w[MAXQ];
    int opp[MAXQ];
} lattice_t;

static void build_lattice(int lat, lattice_t *L)
{
    memset(L, 0, sizeof(*L));
    int n = 0;
    if (lat == 0) {
        /* D2Q9: rest, then all (ex, ey) in {-1,0,1}^2 with |e|^2 in {1, 2} */
        static const int order[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                                        {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
        L->dim = 2;
        for (n = 0; n < 9; ++n) {
            L->e[n][0] = order[n][0];
            L->e[n][1] = order[n][1];
            L->e[n][2] = 0;
            int e2 = order[n][0] * order[n][0] + order[n][1] * order[n][1];
            L->w[n] = e2 == 0 ? 4.0 / 9.0 : (e2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
        }
        L->q = 9;
    } else {
        /* D3Q19: rest, then every e in {-1,0,1}^3 with |e|^2 = 1 or 2 */
        L->dim = 3;
        L->e[0][0] = L->e[0][1] = L->e[0][2] = 0;
        L->w[0] = 1.0 / 3.0;
        n = 1;
        for (int pass = 1; pass <= 2; ++pass)
            for (int ez = -1; ez <= 1; ++ez)
                for (int ey = -1; ey <= 1; ++ey)
                    for (int ex = -1; ex <= 1; ++ex) {
                        int e2 = ex * ex + ey * ey + ez * ez;
                        if (e2 != pass) continue;
                        L->e[n][0] = ex;
                        L->e[n][1] = ey;
                        L->e[n][2] = ez;
                        L->w[n] = pass == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
                        ++n;
                    }
        L->q = n; /* 19 */
    }
    for (int i = 0; i < L->q; ++i)
        for (int j = 0; j < L->q; ++j)
            if (L->e[j][0] == -L->e[i][0] && L->e[j][1] == -L->e[i][1] &&
                L->e[j][2] == -L->e[i][2])
                L->opp[i] = j;
}

/* MRT transform: rows are the polynomial moments of the Lallemand-Luo (D2Q9)
 * and d'Humieres (D3Q19) bases, evaluated at each lattice velocity. */
static void build_mrt(const lattice_t *L, double M[MAXQ][MAXQ])
{
    memset(M, 0, sizeof(double) * MAXQ * MAXQ);
    for (int i = 0; i < L->q; ++i) {
        double ex = L->e[i][0], ey = L->e[i][1], ez = L->e[i][2];
        double e2 = ex * ex + ey * ey + ez * ez;
        if (L->q == 9) {
            double r[9] = {1.0,
                           -4.0 + 3.0 * e2,
                           4.0 - 10.5 * e2 + 4.5 * e2 * e2,
                           ex,
                           (3.0 * e2 - 5.0) * ex,
                           ey,
                           (3.0 * e2 - 5.0) * ey,
                           ex * ex - ey * ey,
                           ex * ey};
            for (int m = 0; m < 9; ++m) M[m][i] = r[m];
        } else {
            double r[19] = {1.0,
                            19.0 * e2 - 30.0,
                            (21.0 * e2 * e2 - 53.0 * e2 + 24.0) / 2.0,
                            ex,
                            (5.0 * e2 - 9.0) * ex,
                            ey,
                            (5.0 * e2 - 9.0) * ey,
                            ez,
                            (5.0 * e2 - 9.0) * ez,
                            3.0 * ex * ex - e2,
                            (3.0 * e2 - 5.0) * (3.0 * ex * ex - e2),
                            ey * ey - ez * ez,
                            (3.0 * e2 - 5.0) * (ey * ey - ez * ez),
                            ex * ey,
                            ey * ez,
                            ex * ez,
                            (ey * ey - ez * ez) * ex,
                            (ez * ez - ex * ex) * ey,
                            (ex * ex - ey * ey) * ez};
            for (int m = 0; m < 19; ++m) M[m][i] = r[m];
        }
    }
}

#ifndef ORACLE_CSTEP
/* Central-moment transform: the rows of build_mrt evaluated at the peculiar
 * velocities e_i - u instead of e_i (CLBM, Eq. 3: N M with N the shift from
 * raw to central moments, so that N M = T(u) with rows P_a(e_i - u)). */
static void build_central(const lattice_t *L, const double u[3], double T[MAXQ][MAXQ])
{
    memset(T, 0, sizeof(double) * MAXQ * MAXQ);
    for (int i = 0; i < L->q; ++i) {
        double ex = L->e[i][0] - u[0], ey = L->e[i][1] - u[1], ez = L->e[i][2] - u[2];
        double e2 = ex * ex + ey * ey + ez * ez;
        if (L->q == 9) {
            double r[9] = {1.0, -4.0 + 3.0 * e2, 4.0 - 10.5 * e2 + 4.5 * e2 * e2, ex, (3.0 * e2 - 5.0) * ex,
                           ey, (3.0 * e2 - 5.0) * ey, ex * ex - ey * ey, ex * ey};
            for (int m = 0; m < 9; ++m) T[m][i] = r[m];
        } else {
            double r[19] = {1.0, 19.0 * e2 - 30.0, (21.0 * e2 * e2 - 53.0 * e2 + 24.0) / 2.0, ex,
                            (5.0 * e2 - 9.0) * ex, ey, (5.0 * e2 - 9.0) * ey, ez, (5.0 * e2 - 9.0) * ez,
                            3.0 * ex * ex - e2, (3.0 * e2 - 5.0) * (3.0 * ex * ex - e2), ey * ey - ez * ez,
                            (3.0 * e2 - 5.0) * (ey * ey - ez * ez), ex * ey, ey * ez, ex * ez,
                            (ey * ey - ez * ez) * ex, (ez * ez - ex * ex) * ey, (ex * ex - ey * ey) * ez};
            for (int m = 0; m < 19; ++m) T[m][i] = r[m];
        }
    }
}
#endif

/* General inverse by Gauss-Jordan elimination with partial pivoting. */
static int invert(int n, double A[MAXQ][MAXQ], double Ainv[MAXQ][MAXQ])
{
    double a[MAXQ][2 * MAXQ];
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < 2 * n; ++c)
            a[r][c] = c < n ? A[r][c] : (c - n == r ? 1.0 : 0.0);
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (fabs(a[piv][col]) < 1e-300) return -1;
        if (piv != col)
            for (int c = 0; c < 2 * n; ++c) {
                double t = a[col][c];
                a[col][c] = a[piv][c];
                a[piv][c] = t;
            }
        double d = a[col][col];
        for (int c = 0; c < 2 * n; ++c) a[col][c] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double fct = a[r][col];
            if (fct == 0.0) continue;
            for (int c = 0; c < 2 * n; ++c) a[r][c] -= fct * a[col][c];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) Ainv[r][c] = a[r][c + n];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Equilibrium (second-order Maxwellian expansion, c_s^2 = 1/3).             */
/* ------------------------------------------------------------------------ */
static void feq(const lattice_t *L, real_t rho, const real_t u[3], real_t out[MAXQ])
{
    real_t uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < L->q; ++i) {
        real_t eu = L->e[i][0] * u[0] + L->e[i][1] * u[1] + L->e[i][2] * u[2];
        out[i] = L->w[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    }
}

/* Carnahan-Starling pressure, eta = b rho / 4 (Eq. 12 uses p_EOS). */
static real_t p_cs(real_t rho, double a, double b, double R, real_t T)
{
    real_t eta = b * rho / 4.0;
    real_t one_m = 1.0 - eta;
    return rho * R * T * (1.0 + eta + eta * eta - eta * eta * eta) /
               (one_m * one_m * one_m) -
           a * rho * rho;
}

/* psi and U of Eq. 12 for component k; the square-root argument is clamped
 * at zero where the EOS leaves the range in which it is non-negative. */
static void pseudopotential(const oref_params *p, int k, real_t rho, real_t *psi, real_t *U)
{
    if (p->psi_kind[k] == 1) {
        *psi = rho;
        *U = 0.0;
        return;
    }
    real_t T = p->eos_T[k];
#ifdef ORACLE_CSTEP
    T += p->eos_T_im[k] * I;
#endif
    real_t pe = p_cs(rho, p->eos_a[k], p->eos_b[k], p->eos_R[k], T);
    real_t u = p->alpha[k] * pe - rho / 3.0;
    real_t arg = 2.0 * u / p->g[k][k];
    if (RE(arg) < 0.0) arg = 0.0;
    *psi = SQRT_R(arg);
    *U = u;
}

/* ------------------------------------------------------------------------ */
/* Geometry helpers.                                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    lattice_t L;
    long N;
    int *nbr; /* nbr[i*N + n] = periodic index of n + e_i */
} geom_t;

static int geom_init(const oref_params *p, geom_t *G)
{
    build_lattice(p->lattice, &G->L);
    G->N = (long)p->nx * p->ny * p->nz;
    G->nbr = (int *)malloc(sizeof(int) * G->L.q * G->N);
    if (!G->nbr) return -1;
    for (int i = 0; i < G->L.q; ++i)
        for (int z = 0; z < p->nz; ++z)
            for (int y = 0; y < p->ny; ++y)
                for (int x = 0; x < p->nx; ++x) {
                    int xx = ((x + G->L.e[i][0]) % p->nx + p->nx) % p->nx;
                    int yy = ((y + G->L.e[i][1]) % p->ny + p->ny) % p->ny;
                    int zz = ((z + G->L.e[i][2]) % p->nz + p->nz) % p->nz;
                    long n = ((long)z * p->ny + y) * p->nx + x;
                    G->nbr[i * G->N + n] = (int)(((long)zz * p->ny + yy) * p->nx + xx);
                }
    return 0;
}

static void geom_free(geom_t *G) { free(G->nbr); }

/* ------------------------------------------------------------------------ */
/* Steps 1-4: densities, virtual densities, pseudopotentials, forces.       */
/* ------------------------------------------------------------------------ */
typedef struct {
    real_t *rho;     /* [nc][N] density at fluid nodes, virtual density at boundary solids */
    real_t *j;       /* [nc][3][N] momentum sum_i f_i e_i at fluid nodes */
    real_t *psi;     /* [nc][N] */
    real_t *U;       /* [nc][N] */
    real_t *F;       /* [nc][3][N] total force on component k */
    real_t *Q;       /* [nc][3][N] Q_xx, Q_yy, Q_xy of Eq. 16 (D2Q9 with kappa) */
    uint8_t *active; /* solid node with at least one fluid neighbour */
} work_t;

static int work_alloc(const oref_params *p, long N, work_t *W)
{
    int nc = p->nc;
    W->rho = (real_t *)calloc((size_t)nc * N, sizeof(real_t));
    W->j = (real_t *)calloc((size_t)nc * 3 * N, sizeof(real_t));
    W->psi = (real_t *)calloc((size_t)nc * N, sizeof(real_t));
    W->U = (real_t *)calloc((size_t)nc * N, sizeof(real_t));
    W->F = (real_t *)calloc((size_t)nc * 3 * N, sizeof(real_t));
    W->Q = (real_t *)calloc((size_t)nc * 3 * N, sizeof(real_t));
    W->active = (uint8_t *)calloc((size_t)N, 1);
    if (!W->rho || !W->j || !W->psi || !W->U || !W->F || !W->Q || !W->active) return -1;
    return 0;
}

static void work_free(work_t *W)
{
    free(W->rho);
    free(W->j);
    free(W->psi);
    free(W->U);
    free(W->F);
    free(W->Q);
    free(W->active);
}

static void fields(const oref_params *p, const geom_t *G, const uint8_t *solid,
                   const real_t *wet, const real_t *f, work_t *W)
{
    const lattice_t *L = &G->L;
    const long N = G->N;
    const int q = L->q, nc = p->nc;

    /* 1. rho^k and j^k at fluid nodes (Eq. 4 / Eq. 10). */
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        for (int k = 0; k < nc; ++k) {
            real_t r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
            if (IS_RES(solid[n])) r = p->res_rho[solid[n] - 2][k];
            if (solid[n] == NODE_FLUID)
                for (int i = 0; i < q; ++i) {
                    real_t fi = f[((long)k * q + i) * N + n];
                    r += fi;
                    jx += fi * L->e[i][0];
                    jy += fi * L->e[i][1];
                    jz += fi * L->e[i][2];
                }
            W->rho[(long)k * N + n] = r;
            W->j[((long)k * 3 + 0) * N + n] = jx;
            W->j[((long)k * 3 + 1) * N + n] = jy;
            W->j[((long)k * 3 + 2) * N + n] = jz;
        }
    }

    /* 1b. Convective outlet nodes: the density of the node below (zero
     * gradient along the outward normal +c), res_rho[1] if that is not fluid. */
    const long plane = p->lattice == 0 ? p->nx : (long)p->nx * p->ny;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        if (solid[n] != NODE_CONV) continue;
        long m = n - plane;
        if (m < 0) m += N;
        for (int k = 0; k < nc; ++k)
            W->rho[(long)k * N + n] = solid[m] == NODE_FLUID ? W->rho[(long)k * N + m] : p->res_rho[1][k];
    }

    /* 2. Improved virtual density (Eq. 17) at solid nodes with a fluid
     * neighbour: weighted average of fluid-neighbour densities, scaled by
     * phi or shifted by -drho, then limited to [rho_min, rho_max].  A
     * reservoir or outlet neighbour counts as fluid. */
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        W->active[n] = 0;
        if (solid[n] != NODE_SOLID) continue;
        double den = 0.0;
        for (int i = 1; i < q; ++i)
            if (solid[G->nbr[i * N + n]] != NODE_SOLID) den += L->w[i];
        if (den == 0.0) continue;
        W->active[n] = 1;
        for (int k = 0; k < nc; ++k) {
            real_t num = 0.0;
            for (int i = 1; i < q; ++i) {
                int m = G->nbr[i * N + n];
                if (solid[m] != NODE_SOLID) num += L->w[i] * W->rho[(long)k * N + m];
            }
            real_t rave = num / den;
            real_t prm = wet[(long)k * N + n];
            real_t rs = p->wet_mode[k] == 0 ? prm * rave : rave - prm;
            if (RE(rs) < p->rho_min[k]) rs = p->rho_min[k];
            if (RE(rs) > p->rho_max[k]) rs = p->rho_max[k];
            W->rho[(long)k * N + n] = rs;
        }
    }

    /* 3. psi^k, U^k at fluid nodes, reservoirs and active solids (Eq. 12). */
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n)
        for (int k = 0; k < nc; ++k) {
            real_t ps = 0.0, uu = 0.0;
            if (solid[n] != NODE_SOLID || W->active[n])
                pseudopotential(p, k, W->rho[(long)k * N + n], &ps, &uu);
            W->psi[(long)k * N + n] = ps;
            W->U[(long)k * N + n] = uu;
        }

    /* 4. Force (Eq. 13) with G_i = w_i / c_s^2 on nearest neighbours, plus
     * the body force rho^k a.  Solid neighbours enter with psi(rho_s). */
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n)
        for (int k = 0; k < nc; ++k) {
            real_t Fk[3] = {0.0, 0.0, 0.0};
            if (solid[n] == NODE_FLUID) {
                real_t zc[3] = {0.0, 0.0, 0.0}, sc[3] = {0.0, 0.0, 0.0};
                for (int i = 1; i < q; ++i) {
                    int m = G->nbr[i * N + n];
                    double Gi = 3.0 * L->w[i];
                    real_t s = 0.0;
                    for (int kk = 0; kk < nc; ++kk) s += p->g[k][kk] * W->psi[(long)kk * N + m];
                    for (int d = 0; d < 3; ++d) {
                        zc[d] += Gi * W->U[(long)k * N + m] * L->e[i][d];
                        sc[d] += Gi * s * L->e[i][d];
                    }
                }
                real_t psik = W->psi[(long)k * N + n];
                real_t rk = W->rho[(long)k * N + n];
                for (int d = 0; d < 3; ++d)
                    Fk[d] = -p->A[k] * zc[d] - (1.0 - p->A[k]) * psik * sc[d] + rk * p->body[d];
            }
            for (int d = 0; d < 3; ++d) W->F[((long)k * 3 + d) * N + n] = Fk[d];
        }

    /* 4b. Tensor Q of the surface-tension source (Eq. 16) at fluid nodes, for
     * components with kappa != 0 (D2Q9 only):
     *   Q = kappa g_kk [ (1 - A) psi(x) sum_i G_i (psi(x+e_i) - psi(x)) e_i e_i
     *                   + (A/2) sum_i G_i (psi(x+e_i)^2 - psi(x)^2) e_i e_i ]
     * with the force stencil G_i = w_i / c_s^2.  The printed Eq. 16 leaves out
     * the interaction strength; with the factor g_kk the surface tension
     * falls with kappa as Table 2 prints it (0.457 of its unmodified value at
     * 1 - kappa = 0.5, about 0.01 at 1 - kappa = 0.01), and the coexistence
     * densities stay put (Table 1). */
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n)
        for (int k = 0; k < nc; ++k) {
            real_t Qxx = 0.0, Qyy = 0.0, Qxy = 0.0;
            if (p->kappa[k] != 0.0 && solid[n] == NODE_FLUID) {
                real_t ps = W->psi[(long)k * N + n];
                real_t s_xx = 0.0, s_yy = 0.0, s_xy = 0.0, t_xx = 0.0, t_yy = 0.0, t_xy = 0.0;
                for (int i = 1; i < q; ++i) {
                    int m = G->nbr[i * N + n];
                    double Gi = 3.0 * L->w[i];
                    real_t pm = W->psi[(long)k * N + m];
                    real_t a = Gi * (pm - ps), b = Gi * (pm * pm - ps * ps);
                    double ex = L->e[i][0], ey = L->e[i][1];
                    s_xx += a * ex * ex;
                    s_yy += a * ey * ey;
                    s_xy += a * ex * ey;
                    t_xx += b * ex * ex;
                    t_yy += b * ey * ey;
                    t_xy += b * ex * ey;
                }
                double c = p->kappa[k] * p->g[k][k];
                double A = p->A[k];
                Qxx = c * ((1.0 - A) * ps * s_xx + 0.5 * A * t_xx);
                Qyy = c * ((1.0 - A) * ps * s_yy + 0.5 * A * t_yy);
                Qxy = c * ((1.0 - A) * ps * s_xy + 0.5 * A * t_xy);
            }
            W->Q[((long)k * 3 + 0) * N + n] = Qxx;
            W->Q[((long)k * 3 + 1) * N + n] = Qyy;
            W->Q[((long)k * 3 + 2) * N + n] = Qxy;
        }
}

/* ------------------------------------------------------------------------ */
/* Steps 5-7: equilibrium velocity, collision + EDM, streaming.             */
/* ------------------------------------------------------------------------ */
#ifndef ORACLE_CSTEP
/* Central-moment collision with the consistent forcing of the same moments
 * (Eq. 3 CLBM form, Eq. 7): with T = N M the central-moment transform at the
 * velocity u = (j + F/2)/rho (Eq. 8),
 *   f* = f + T^-1 [ -S T (f - f^eq) + (I - S/2) T R ],
 *   R_i = (F / rho) . (e_i - u) / c_s^2  f^eq_i,
 * and no exact-difference term. */
static void collide_clbm(const lattice_t *L, const double *rates, double rho, const double u[3],
                         const double F[3], const double *fi, double *fo)
{
    const int q = L->q;
    double T[MAXQ][MAXQ], Ti[MAXQ][MAXQ], fe[MAXQ], R[MAXQ], y[MAXQ];
    build_central(L, u, T);
    invert(q, T, Ti);
    feq(L, rho, u, fe);
    for (int i = 0; i < q; ++i) {
        double s = 0.0;
        for (int d = 0; d < 3; ++d) s += F[d] * (L->e[i][d] - u[d]);
        R[i] = 3.0 * s / rho * fe[i];
    }
    for (int a = 0; a < q; ++a) {
        double z = 0.0, w = 0.0;
        for (int i = 0; i < q; ++i) {
            z += T[a][i] * (fi[i] - fe[i]);
            w += T[a][i] * R[i];
        }
        y[a] = -rates[a] * z + (1.0 - 0.5 * rates[a]) * w;
    }
    for (int i = 0; i < q; ++i) {
        double x = 0.0;
        for (int a = 0; a < q; ++a) x += Ti[i][a] * y[a];
        fo[i] = fi[i] + x;
    }
}
#endif

static void collide(const oref_params *p, const geom_t *G, const uint8_t *solid,
                    const real_t *f, const work_t *W, double M[MAXQ][MAXQ],
                    double Minv[MAXQ][MAXQ], real_t *fpost)
{
    const lattice_t *L = &G->L;
    const long N = G->N;
    const int q = L->q, nc = p->nc;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        if (solid[n] != NODE_FLUID) {
            for (int k = 0; k < nc; ++k)
                for (int i = 0; i < q; ++i) fpost[((long)k * q + i) * N + n] = 0.0;
            continue;
        }
        /* 5. Equilibrium velocity: j/rho (one component, or per component);
         * common u' = sum_k(j^k/tau_k) / sum_k(rho^k/tau_k) otherwise. */
        real_t ucom[3] = {0.0, 0.0, 0.0};
        if (nc > 1 && p->common_velocity) {
            real_t num[3] = {0.0, 0.0, 0.0}, den = 0.0;
            for (int k = 0; k < nc; ++k) {
                for (int d = 0; d < 3; ++d) num[d] += W->j[((long)k * 3 + d) * N + n] / p->tau[k];
                den += W->rho[(long)k * N + n] / p->tau[k];
            }
            for (int d = 0; d < 3; ++d) ucom[d] = num[d] / den;
        }
        for (int k = 0; k < nc; ++k) {
            real_t rho = W->rho[(long)k * N + n];
#ifndef ORACLE_CSTEP
            if (p->collision == 2) {
                /* one component: u = (j + F/2)/rho (Eq. 8) */
                double uc[3], Fk[3], fi[MAXQ], fo[MAXQ];
                for (int d = 0; d < 3; ++d) {
                    Fk[d] = W->F[((long)k * 3 + d) * N + n];
                    uc[d] = (W->j[((long)k * 3 + d) * N + n] + 0.5 * Fk[d]) / rho;
                }
                for (int i = 0; i < q; ++i) fi[i] = f[((long)k * q + i) * N + n];
                collide_clbm(L, p->mrt_s[k], rho, uc, Fk, fi, fo);
                for (int i = 0; i < q; ++i) fpost[((long)k * q + i) * N + n] = fo[i];
                continue;
            }
#endif
            real_t u[3];
            for (int d = 0; d < 3; ++d)
                u[d] = (nc > 1 && p->common_velocity) ? ucom[d]
                                                      : W->j[((long)k * 3 + d) * N + n] / rho;
            real_t fi[MAXQ], fe[MAXQ], fo[MAXQ];
            for (int i = 0; i < q; ++i) fi[i] = f[((long)k * q + i) * N + n];
            feq(L, rho, u, fe);
            /* 6a. Collision (Eq. 3). */
            if (p->collision == 0) {
                for (int i = 0; i < q; ++i) fo[i] = fi[i] - (fi[i] - fe[i]) / p->tau[k];
            } else {
                real_t m[MAXQ];
                for (int a = 0; a < q; ++a) {
                    real_t s = 0.0;
                    for (int i = 0; i < q; ++i) s += M[a][i] * (fi[i] - fe[i]);
                    m[a] = p->mrt_s[k][a] * s;
                }
                /* surface-tension source in moment space (Eq. 15, D2Q9 rows
                 * rho, e, eps, jx, qx, jy, qy, pxx, pxy), added after the
                 * relaxation: f* = f - M^-1 (S(m - m^eq) - C) */
                if (p->kappa[k] != 0.0) {
                    real_t Qxx = W->Q[((long)k * 3 + 0) * N + n];
                    real_t Qyy = W->Q[((long)k * 3 + 1) * N + n];
                    real_t Qxy = W->Q[((long)k * 3 + 2) * N + n];
                    m[1] -= 1.5 * p->mrt_s[k][1] * (Qxx + Qyy);
                    m[2] -= -1.5 * p->mrt_s[k][2] * (Qxx + Qyy);
                    m[7] -= -p->mrt_s[k][7] * (Qxx - Qyy);
                    m[8] -= -p->mrt_s[k][8] * Qxy;
                }
                for (int i = 0; i < q; ++i) {
                    real_t s = 0.0;
                    for (int a = 0; a < q; ++a) s += Minv[i][a] * m[a];
                    fo[i] = fi[i] - s;
                }
            }
            /* 6b. Exact difference method (Eq. 5): du = F dt / rho. */
            real_t u2[3], fe2[MAXQ];
            for (int d = 0; d < 3; ++d) u2[d] = u[d] + W->F[((long)k * 3 + d) * N + n] / rho;
            feq(L, rho, u2, fe2);
            for (int i = 0; i < q; ++i)
                fpost[((long)k * q + i) * N + n] = fo[i] + (fe2[i] - fe[i]);
        }
    }
}

/* 7. Streaming (Eq. 2) with halfway bounce-back: a population that would
 * leave a fluid node toward a solid node returns to it reversed; one that
 * comes from a reservoir node is the reservoir's rest equilibrium
 * w_i res_rho. */
static void stream(const oref_params *p, const geom_t *G, const uint8_t *solid,
                   const real_t *fpost, real_t *f)
{
    const lattice_t *L = &G->L;
    const long N = G->N;
    const int q = L->q, nc = p->nc;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n)
        for (int k = 0; k < nc; ++k)
            for (int i = 0; i < q; ++i) {
                real_t v = 0.0;
                if (solid[n] == NODE_FLUID) {
                    int src = G->nbr[L->opp[i] * N + n]; /* n - e_i */
                    if (solid[src] == NODE_SOLID)
                        v = fpost[((long)k * q + L->opp[i]) * N + n];
                    else if (IS_RES(solid[src]))
                        v = 2.0 * L->w[i] * p->res_rho[solid[src] - 2][k] -
                            fpost[((long)k * q + L->opp[i]) * N + n];
                    else
                        v = fpost[((long)k * q + i) * N + src];
                }
                f[((long)k * q + i) * N + n] = v;
            }
}

/* 7b. Convective outlet (Sec. 3.4.2): a population f_i that streams into the
 * fluid node x from the outlet plane above it (e_i pointing down, -c) solves
 * d f/dt + U d f/dc = 0 by the implicit upwind step
 *   f_i(x, t+1) = (f_i(x, t) + U f_i(x - c, t+1)) / (1 + U),
 * with U = max(0, mean over the fluid nodes of the plane below the outlet of
 * the bare outward velocity sum_k j_c^k / sum_k rho^k at time t) -- the
 * average-velocity form -- and f_i(x - c, t+1) the population just streamed
 * into the node below x (f_i(x, t) again where that node is not fluid).
 * fold holds f(t), f holds f(t+1) from the plain streaming.
 * Pinned in the steady limit only (a fluid at rest, a developed flow); the
 * transient action of U is parity unpinned. */
static void convective_outlet(const oref_params *p, const geom_t *G, const uint8_t *solid,
                              const work_t *W, const real_t *fold, real_t *f)
{
    const lattice_t *L = &G->L;
    const long N = G->N;
    const int q = L->q, nc = p->nc;
    const long plane = p->lattice == 0 ? p->nx : (long)p->nx * p->ny;
    const int cax = p->lattice == 0 ? 1 : 2; /* the slowest axis: y in 2-D, z in 3-D */
    real_t usum = 0.0;
    long cnt = 0;
    for (long n = 0; n < N; ++n) {
        if (solid[n] != NODE_FLUID) continue;
        long up = n + plane;
        if (up >= N) up -= N;
        if (solid[up] != NODE_CONV) continue;
        real_t jc = 0.0, r = 0.0;
        for (int k = 0; k < nc; ++k) {
            jc += W->j[((long)k * 3 + cax) * N + n];
            r += W->rho[(long)k * N + n];
        }
        usum += jc / r;
        ++cnt;
    }
    real_t U = cnt ? usum / (double)cnt : 0.0;
    if (RE(U) < 0.0) U = 0.0;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        if (solid[n] != NODE_FLUID) continue;
        long below = n - plane;
        if (below < 0) below += N;
        for (int i = 0; i < q; ++i) {
            if (L->e[i][cax] != -1) continue;
            int src = G->nbr[L->opp[i] * N + n]; /* n - e_i, in the plane above */
            if (solid[src] != NODE_CONV) continue;
            for (int k = 0; k < nc; ++k) {
                long a = ((long)k * q + i) * N;
                real_t prev = fold[a + n];
                real_t upw = solid[below] == NODE_FLUID ? f[a + below] : prev;
                f[a + n] = (prev + U * upw) / (1.0 + U);
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Exported API.                                                            */
/* ------------------------------------------------------------------------ */

#ifndef ORACLE_CSTEP
/* Lattice tables: q, e[q][3], w[q], opp[q]. */
int oref_lattice(int lat, int *q, int *e, double *w, int *opp)
{
    lattice_t L;
    build_lattice(lat, &L);
    *q = L.q;
    for (int i = 0; i < L.q; ++i) {
        for (int d = 0; d < 3; ++d) e[i * 3 + d] = L.e[i][d];
        w[i] = L.w[i];
        opp[i] = L.opp[i];
    }
    return 0;
}

/* MRT matrix M[q][q] (rows = moments) and its inverse. */
int oref_mrt_matrix(int lat, double *Mout, double *Minvout)
{
    lattice_t L;
    double M[MAXQ][MAXQ], Mi[MAXQ][MAXQ];
    build_lattice(lat, &L);
    build_mrt(&L, M);
    if (invert(L.q, M, Mi)) return -1;
    for (int a = 0; a < L.q; ++a)
        for (int b = 0; b < L.q; ++b) {
            Mout[a * L.q + b] = M[a][b];
            Minvout[a * L.q + b] = Mi[a][b];
        }
    return 0;
}

/* Equilibrium of one node. */
void oref_feq(int lat, double rho, const double *u, double *out)
{
    lattice_t L;
    build_lattice(lat, &L);
    feq(&L, rho, u, out);
}

/* Carnahan-Starling pseudopotential of one density value for component k. */
void oref_psi(const oref_params *p, int k, double rho, double *psi, double *U)
{
    pseudopotential(p, k, rho, psi, U);
}

/* Collision + EDM of a single node (one component, velocity u given). */
void oref_collide_node(const oref_params *p, int k, const double *fin, const double *u,
                       const double *F, double *fout)
{
    lattice_t L;
    double M[MAXQ][MAXQ], Mi[MAXQ][MAXQ];
    build_lattice(p->lattice, &L);
    build_mrt(&L, M);
    invert(L.q, M, Mi);
    double rho = 0.0;
    for (int i = 0; i < L.q; ++i) rho += fin[i];
    if (p->collision == 2) {
        collide_clbm(&L, p->mrt_s[k], rho, u, F, fin, fout);
        return;
    }
    double fe[MAXQ], fe2[MAXQ], u2[3];
    feq(&L, rho, u, fe);
    if (p->collision == 0) {
        for (int i = 0; i < L.q; ++i) fout[i] = fin[i] - (fin[i] - fe[i]) / p->tau[k];
    } else {
        double m[MAXQ];
        for (int a = 0; a < L.q; ++a) {
            double s = 0.0;
            for (int i = 0; i < L.q; ++i) s += M[a][i] * (fin[i] - fe[i]);
            m[a] = p->mrt_s[k][a] * s;
        }
        for (int i = 0; i < L.q; ++i) {
            double s = 0.0;
            for (int a = 0; a < L.q; ++a) s += Mi[i][a] * m[a];
            fout[i] = fin[i] - s;
        }
    }
    for (int d = 0; d < 3; ++d) u2[d] = u[d] + F[d] / rho;
    feq(&L, rho, u2, fe2);
    for (int i = 0; i < L.q; ++i) fout[i] += fe2[i] - fe[i];
}
#endif

/* Populations f = f^eq(rho0, u0) at fluid nodes, zero at solid nodes.
 * rho0[nc][N]; u0[3][N] (shared by all components) or NULL for rest. */
/* Threads of the parallel node loops (timing only: every node is computed
 * independently, so the result does not depend on it). */
void API(set_threads)(int n) { omp_set_num_threads(n > 0 ? n : 1); }

int API(init_feq)(const oref_params *p, const uint8_t *solid, const real_t *rho0,
                  const real_t *u0, real_t *f)
{
    geom_t G;
    if (geom_init(p, &G)) return -2;
    const lattice_t *L = &G.L;
    const long N = G.N;
    for (long n = 0; n < N; ++n)
        for (int k = 0; k < p->nc; ++k) {
            real_t u[3] = {0.0, 0.0, 0.0}, fe[MAXQ];
            if (u0)
                for (int d = 0; d < 3; ++d) u[d] = u0[(long)d * N + n];
            feq(L, rho0[(long)k * N + n], u, fe);
            for (int i = 0; i < L->q; ++i)
                f[((long)k * L->q + i) * N + n] = solid[n] != NODE_FLUID ? 0.0 : fe[i];
        }
    geom_free(&G);
    return 0;
}

/* Advance nsteps full time steps in place. wet[nc][N] holds the per-node
 * wetting parameter (phi or drho, by component mode). */
int API(step)(const oref_params *p, const uint8_t *solid, const real_t *wet, real_t *f,
              int nsteps)
{
    geom_t G;
    work_t W;
    double M[MAXQ][MAXQ], Mi[MAXQ][MAXQ];
    if (p->nc < 1 || p->nc > MAXC) return -1;
    for (long n = 0; n < (long)p->nx * p->ny * p->nz; ++n)
        if (solid[n] > 4) return -5;
    for (int k = 0; k < p->nc; ++k)
        if (p->kappa[k] != 0.0 && (p->lattice != 0 || p->collision != 1)) return -4;
    if (p->collision == 2 && p->nc != 1) return -4;
#ifdef ORACLE_CSTEP
    if (p->collision == 2) return -4;
#endif
    if (geom_init(p, &G)) return -2;
    build_mrt(&G.L, M);
    if (invert(G.L.q, M, Mi)) return -3;
    if (work_alloc(p, G.N, &W)) return -2;
    real_t *fpost = (real_t *)malloc(sizeof(real_t) * p->nc * G.L.q * G.N);
    if (!fpost) return -2;
    int has_conv = 0;
    for (long n = 0; n < G.N; ++n) has_conv |= solid[n] == NODE_CONV;
    real_t *fold = has_conv ? (real_t *)malloc(sizeof(real_t) * p->nc * G.L.q * G.N) : NULL;
    if (has_conv && !fold) return -2;
    for (int s = 0; s < nsteps; ++s) {
        fields(p, &G, solid, wet, f, &W);
        collide(p, &G, solid, f, &W, M, Mi, fpost);
        if (has_conv) {
            memcpy(fold, f, sizeof(real_t) * p->nc * G.L.q * G.N);
            stream(p, &G, solid, fpost, f);
            convective_outlet(p, &G, solid, &W, fold, f);
        } else {
            stream(p, &G, solid, fpost, f);
        }
    }
    free(fold);
    free(fpost);
    work_free(&W);
    geom_free(&G);
    return 0;
}

/* Diagnostic fields of the current state (any output may be NULL):
 *   rho[nc][N]     density (virtual density at boundary solids, the fixed
 *                  density at reservoirs, 0 at other solids)
 *   F[nc][3][N]    force on each component
 *   u[nc][3][N]    per-component velocity (j^k + F^k/2)/rho^k      (Eq. 6)
 *   umix[3][N]     mixture velocity sum_k(j^k + F^k/2)/sum_k rho^k
 *   psi[nc][N]     pseudopotential
 *   U[nc][N]       Zhang-Chen potential */
int API(fields)(const oref_params *p, const uint8_t *solid, const real_t *wet,
                const real_t *f, real_t *rho, real_t *F, real_t *u, real_t *umix,
                real_t *psi, real_t *U)
{
    geom_t G;
    work_t W;
    if (geom_init(p, &G)) return -2;
    if (work_alloc(p, G.N, &W)) return -2;
    fields(p, &G, solid, wet, f, &W);
    const long N = G.N;
    const int nc = p->nc;
    if (rho) memcpy(rho, W.rho, sizeof(real_t) * nc * N);
    if (F) memcpy(F, W.F, sizeof(real_t) * nc * 3 * N);
    if (psi) memcpy(psi, W.psi, sizeof(real_t) * nc * N);
    if (U) memcpy(U, W.U, sizeof(real_t) * nc * N);
    for (long n = 0; n < N; ++n) {
        real_t num[3] = {0.0, 0.0, 0.0}, den = 0.0;
        for (int k = 0; k < nc; ++k) {
            real_t r = W.rho[(long)k * N + n];
            for (int d = 0; d < 3; ++d) {
                real_t m = W.j[((long)k * 3 + d) * N + n] + 0.5 * W.F[((long)k * 3 + d) * N + n];
                if (u) u[((long)k * 3 + d) * N + n] = solid[n] != NODE_FLUID ? 0.0 : m / r;
                num[d] += m;
            }
            den += r;
        }
        if (umix)
            for (int d = 0; d < 3; ++d) umix[(long)d * N + n] = solid[n] != NODE_FLUID ? 0.0 : num[d] / den;
        if (solid[n] == NODE_SOLID && rho)
            for (int k = 0; k < nc; ++k)
                if (!W.active[n]) rho[(long)k * N + n] = 0.0;
    }
    work_free(&W);
    geom_free(&G);
    return 0;
}

/* Streaming alone applied to a post-collision field (for invariance pins). */
int API(stream_only)(const oref_params *p, const uint8_t *solid, const real_t *fpost,
                     real_t *f)
{
    geom_t G;
    if (geom_init(p, &G)) return -2;
    stream(p, &G, solid, fpost, f);
    geom_free(&G);
    return 0;
}
