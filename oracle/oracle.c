/*
 * Plain FP64 CPU oracle for the multiphase lattice Boltzmann step of
 * arXiv 2101.06769 (Hosseini, Safari, Thevenin).  TEST INFRASTRUCTURE ONLY:
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code with the GPU library.
 *
 * Every function follows the paper's equations in the paper's order, using
 * general transforms (all Q central moments by direct sums, the full set of
 * cumulants, an arbitrary relaxation-rate vector, a dense linear solve for
 * the back-transform to populations).  Nothing is blocked, fused or
 * reordered beyond what the equations state.
 *
 * Readings of passages that are garbled or silent (each also listed in the
 * design notes):
 *  - chemical potential: mu = 2 beta phi (phi-1)(2phi-1) - kappa lap(phi)
 *    (operator missing in Sec. 2.1; this is the functional derivative of the
 *    double-well free energy).
 *  - forces F = mu grad(phi) + rho g enter the flow source with a + sign.
 *  - the phase-field source is added (discrete form of Sec. 2.2), with the
 *    factor (1 - 1/(2 taubar_phi)), taubar_phi = M/cs^2 + 1/2.
 *  - Hermite coefficients are normalised (a0 = 1, a_i = u_i, a_ij = u_i u_j)
 *    so that sum g_eq = phi and sum f'_eq = p_h.
 *  - the second K^p in the MRT collision formula is the equilibrium K^eq.
 *  - the dilatation term w cs^2 rho div(u) of the flow source is dropped
 *    (two incompressible phases).
 *  - cumulants act on h = f^p - w (P - 1), P = sum f^p, so that sum h = 1 and
 *    sum c h = u; w (P - 1) is carried through the collision unchanged.
 *  - cumulant equilibria: second-order diagonal cs^2, everything else 0;
 *    viscosity acts on the off-diagonal and deviatoric second-order
 *    cumulants with omega = 1/(nu/cs^2 + 1/2); all other rates 1.
 *  - sixth-order transforms: set-partition form (Pi_yz pairs with Pi_x2yz,
 *    the 2(...) third-order group is separate, and the 2+2+2 group enters the
 *    forward relation with + and the backward one with -).
 *  - interface normal n = grad(phi)/sqrt(|grad(phi)|^2 + 1e-24).
 *  - viscosity interpolated linearly in phi (kinematic) unless asked otherwise.
 *  - walls: half-way bounce-back for both population sets; the phi stencil
 *    mirrors the first fluid layer into the ghost layer.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CS2 (1.0 / 3.0)
#define QMAX 27

/* diag offsets (orc_collide_cell) */
#define D_U 0
#define D_RHO 3
#define D_P 4
#define D_PSTAR 5
#define D_OMEGA 6
#define D_MU 7
#define D_F 8
#define D_N 11
#define D_TAUPHI 14
#define D_XI 16
#define D_H 48
#define D_PI 80
#define D_K 112
#define D_KS 144
#define D_PIS 176
#define D_HS 208
#define D_GEQ 240
#define D_SBAR 272

/* ----------------------------------------------------------------------- */
/* Lattices (Sec. 2.3: D3Q27; D2Q9 for the two-dimensional cases)           */
/* ----------------------------------------------------------------------- */

static const int C2D[9][3] = {{0, 0, 0},  {1, 0, 0},   {0, 1, 0},  {-1, 0, 0}, {0, -1, 0},
                              {1, 1, 0},  {-1, 1, 0},  {-1, -1, 0}, {1, -1, 0}};
static const double W2D[9] = {4. / 9,  1. / 9,  1. / 9,  1. / 9, 1. / 9,
                              1. / 36, 1. / 36, 1. / 36, 1. / 36};

static const int C3D[27][3] = {
    {0, 0, 0},
    {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},   {0, 0, -1},
    {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},  {1, 0, 1},   {-1, 0, -1},
    {1, 0, -1},  {-1, 0, 1},  {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1},
    {1, 1, 1},   {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1},  {-1, 1, -1},
    {-1, 1, 1},  {1, -1, -1}};
static const double W3D[27] = {
    8. / 27,
    2. / 27,  2. / 27,  2. / 27,  2. / 27,  2. / 27,  2. / 27,
    1. / 54,  1. / 54,  1. / 54,  1. / 54,  1. / 54,  1. / 54,
    1. / 54,  1. / 54,  1. / 54,  1. / 54,  1. / 54,  1. / 54,
    1. / 216, 1. / 216, 1. / 216, 1. / 216, 1. / 216, 1. / 216, 1. / 216, 1. / 216};

typedef struct {
    int Q;
    int c[QMAX][3];
    double w[QMAX];
    int opp[QMAX];
} lat_t;

static void lat_get(int dim, lat_t *L)
{
    int a, b, i;
    L->Q = dim == 2 ? 9 : 27;
    for (a = 0; a < L->Q; a++) {
        for (i = 0; i < 3; i++) L->c[a][i] = dim == 2 ? C2D[a][i] : C3D[a][i];
        L->w[a] = dim == 2 ? W2D[a] : W3D[a];
    }
    for (a = 0; a < L->Q; a++)
        for (b = 0; b < L->Q; b++)
            if (L->c[b][0] == -L->c[a][0] && L->c[b][1] == -L->c[a][1] && L->c[b][2] == -L->c[a][2])
                L->opp[a] = b;
}

int orc_Q(int dim) { return dim == 2 ? 9 : (dim == 3 ? 27 : -1); }

void orc_lattice(int dim, int *c, double *w, int *opp)
{
    lat_t L;
    int a, i;
    lat_get(dim, &L);
    for (a = 0; a < L.Q; a++) {
        for (i = 0; i < 3; i++) c[3 * a + i] = L.c[a][i];
        w[a] = L.w[a];
        opp[a] = L.opp[a];
    }
}

void orc_set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int check_params(const orc_params *p)
{
    if (p->dim != 2 && p->dim != 3) return -1;
    if (p->n[0] <= 0 || p->n[1] <= 0 || p->n[2] <= 0) return -1;
    if (p->dim == 2 && p->n[2] != 1) return -1;
    if (p->cac_edf != 0 && p->cac_edf != 1) return -1;
    return 0;
}

static long ncells(const orc_params *p) { return (long)p->n[0] * p->n[1] * p->n[2]; }

/* ----------------------------------------------------------------------- */
/* Hermite expansion (Appendix A): sum_{n=nmin}^{2} H_n : a_n / (n! cs^2n)   */
/* with the normalised coefficients a0 = 1, a_i = u_i, a_ij = u_i u_j.      */
/* ----------------------------------------------------------------------- */
static double hermite_sum(const int *c, const double *u, int nmin)
{
    double s = 0.0, h1 = 0.0, h2 = 0.0;
    int i, j;
    if (nmin <= 0) s += 1.0;
    for (i = 0; i < 3; i++) h1 += c[i] * u[i];
    s += h1 / CS2;
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++) h2 += (c[i] * c[j] - CS2 * (i == j)) * u[i] * u[j];
    s += h2 / (2.0 * CS2 * CS2);
    return s;
}

/* The same expansion truncated after the first-order term (Sec. 2.2, the
 * first-order equilibrium): 1 + c.u / cs^2. */
static double hermite_sum_first(const int *c, const double *u)
{
    double h1 = 0.0;
    int i;
    for (i = 0; i < 3; i++) h1 += c[i] * u[i];
    return 1.0 + h1 / CS2;
}

/* ----------------------------------------------------------------------- */
/* Isotropic finite differences (Sec. 2.2)                                 */
/* ----------------------------------------------------------------------- */

/* neighbour index along one axis for the phi stencil: periodic wrap, or the
 * ghost layer mirrors the first fluid layer at walls and symmetry planes */
static int stencil_coord(int x, int d, int n, int bc)
{
    int s = x + d;
    if (s >= 0 && s < n) return s;
    if (bc == ORC_BC_PERIODIC) return (s + n) % n;
    return s < 0 ? 0 : n - 1;
}

static long cell_index(const orc_params *p, int x, int y, int z)
{
    return ((long)z * p->n[1] + y) * p->n[0] + x;
}

static double phi_from_g(const lat_t *L, const double *g, long N, long idx)
{
    double s = 0.0;
    int a;
    for (a = 0; a < L->Q; a++) s += g[(long)a * N + idx];
    return s;
}

/* gradient = (1/cs^2) sum w c phi(x+c); laplacian = (2/cs^2) sum w [phi(x+c) - phi(x)].
 * phi values come from the field when given, otherwise from sum_a g_a at each neighbour. */
static void stencil(const orc_params *p, const lat_t *L, const double *phi_field, const double *g,
                    int x, int y, int z, double *phi0, double *grad, double *lap)
{
    long N = ncells(p);
    long i0 = cell_index(p, x, y, z);
    double p0 = phi_field ? phi_field[i0] : phi_from_g(L, g, N, i0);
    double gr[3] = {0, 0, 0}, lp = 0.0;
    int a, i;
    for (a = 0; a < L->Q; a++) {
        int xs = stencil_coord(x, L->c[a][0], p->n[0], p->bc[0]);
        int ys = stencil_coord(y, L->c[a][1], p->n[1], p->bc[1]);
        int zs = stencil_coord(z, L->c[a][2], p->n[2], p->bc[2]);
        long j = cell_index(p, xs, ys, zs);
        double pn = phi_field ? phi_field[j] : phi_from_g(L, g, N, j);
        for (i = 0; i < 3; i++) gr[i] += L->w[a] * L->c[a][i] * pn;
        lp += L->w[a] * (pn - p0);
    }
    for (i = 0; i < 3; i++) grad[i] = gr[i] / CS2;
    *lap = 2.0 * lp / CS2;
    *phi0 = p0;
}

int orc_gradients(const orc_params *p, const double *phi, double *grad, double *lap)
{
    lat_t L;
    long N, row;
    if (check_params(p)) return -1;
    lat_get(p->dim, &L);
    N = ncells(p);
#pragma omp parallel for schedule(static)
    for (row = 0; row < (long)p->n[1] * p->n[2]; row++) {
        int x, i, y = (int)(row % p->n[1]), z = (int)(row / p->n[1]);
        for (x = 0; x < p->n[0]; x++) {
            double p0, gr[3], lp;
            long idx = cell_index(p, x, y, z);
            stencil(p, &L, phi, NULL, x, y, z, &p0, gr, &lp);
            for (i = 0; i < 3; i++) grad[(long)i * N + idx] = gr[i];
            lap[idx] = lp;
        }
    }
    return 0;
}

/* ----------------------------------------------------------------------- */
/* Central moments and cumulants (Sec. 2.3)                                 */
/* Pi27[a*9 + b*3 + c] holds the central moment x^a y^b z^c.               */
/* ----------------------------------------------------------------------- */
#define IX(a, b, c) ((a) * 9 + (b) * 3 + (c))

/* x^k for the small non-negative exponents of the moment basis */
static double ipow(double x, int k)
{
    double r = 1.0;
    while (k-- > 0) r *= x;
    return r;
}

void orc_central_moments(int dim, const double *h, const double *u, double *Pi27)
{
    lat_t L;
    int a, b, c, al;
    lat_get(dim, &L);
    for (a = 0; a < 27; a++) Pi27[a] = 0.0;
    for (a = 0; a < 3; a++)
        for (b = 0; b < 3; b++)
            for (c = 0; c < (dim == 2 ? 1 : 3); c++) {
                double s = 0.0;
                for (al = 0; al < L.Q; al++)
                    s += ipow(L.c[al][0] - u[0], a) * ipow(L.c[al][1] - u[1], b) *
                         ipow(L.c[al][2] - u[2], c) * h[al];
                Pi27[IX(a, b, c)] = s;
            }
}

/* Central moments -> cumulants for a unit-mass set with zero first central
 * moments: orders <= 3 equal the central moments; orders 4-6 subtract the
 * products of lower-order moments over the set partitions (Sec. 2.3). */
void orc_cumulants_from_central(int dim, const double *P, double *K)
{
    int i;
    for (i = 0; i < 27; i++) K[i] = P[i];
    if (dim == 2) {
        K[IX(2, 2, 0)] = P[IX(2, 2, 0)] - (P[IX(2, 0, 0)] * P[IX(0, 2, 0)] + 2.0 * P[IX(1, 1, 0)] * P[IX(1, 1, 0)]);
        return;
    }
    /* fourth order: x^2yz and permutations */
    K[IX(2, 1, 1)] = P[IX(2, 1, 1)] - (P[IX(2, 0, 0)] * P[IX(0, 1, 1)] + 2.0 * P[IX(1, 1, 0)] * P[IX(1, 0, 1)]);
    K[IX(1, 2, 1)] = P[IX(1, 2, 1)] - (P[IX(0, 2, 0)] * P[IX(1, 0, 1)] + 2.0 * P[IX(1, 1, 0)] * P[IX(0, 1, 1)]);
    K[IX(1, 1, 2)] = P[IX(1, 1, 2)] - (P[IX(0, 0, 2)] * P[IX(1, 1, 0)] + 2.0 * P[IX(1, 0, 1)] * P[IX(0, 1, 1)]);
    /* fourth order: x^2y^2 and permutations */
    K[IX(2, 2, 0)] = P[IX(2, 2, 0)] - (P[IX(2, 0, 0)] * P[IX(0, 2, 0)] + 2.0 * P[IX(1, 1, 0)] * P[IX(1, 1, 0)]);
    K[IX(2, 0, 2)] = P[IX(2, 0, 2)] - (P[IX(2, 0, 0)] * P[IX(0, 0, 2)] + 2.0 * P[IX(1, 0, 1)] * P[IX(1, 0, 1)]);
    K[IX(0, 2, 2)] = P[IX(0, 2, 2)] - (P[IX(0, 2, 0)] * P[IX(0, 0, 2)] + 2.0 * P[IX(0, 1, 1)] * P[IX(0, 1, 1)]);
    /* fifth order: xy^2z^2 and permutations */
    K[IX(1, 2, 2)] = P[IX(1, 2, 2)] - (P[IX(0, 0, 2)] * P[IX(1, 2, 0)] + P[IX(0, 2, 0)] * P[IX(1, 0, 2)] +
                                       4.0 * P[IX(0, 1, 1)] * P[IX(1, 1, 1)] +
                                       2.0 * (P[IX(1, 0, 1)] * P[IX(0, 2, 1)] + P[IX(1, 1, 0)] * P[IX(0, 1, 2)]));
    K[IX(2, 1, 2)] = P[IX(2, 1, 2)] - (P[IX(0, 0, 2)] * P[IX(2, 1, 0)] + P[IX(2, 0, 0)] * P[IX(0, 1, 2)] +
                                       4.0 * P[IX(1, 0, 1)] * P[IX(1, 1, 1)] +
                                       2.0 * (P[IX(0, 1, 1)] * P[IX(2, 0, 1)] + P[IX(1, 1, 0)] * P[IX(1, 0, 2)]));
    K[IX(2, 2, 1)] = P[IX(2, 2, 1)] - (P[IX(2, 0, 0)] * P[IX(0, 2, 1)] + P[IX(0, 2, 0)] * P[IX(2, 0, 1)] +
                                       4.0 * P[IX(1, 1, 0)] * P[IX(1, 1, 1)] +
                                       2.0 * (P[IX(1, 0, 1)] * P[IX(1, 2, 0)] + P[IX(0, 1, 1)] * P[IX(2, 1, 0)]));
    /* sixth order */
    {
        double pairs4 = P[IX(2, 0, 0)] * P[IX(0, 2, 2)] + P[IX(0, 2, 0)] * P[IX(2, 0, 2)] +
                        P[IX(0, 0, 2)] * P[IX(2, 2, 0)] +
                        4.0 * (P[IX(0, 1, 1)] * P[IX(2, 1, 1)] + P[IX(1, 0, 1)] * P[IX(1, 2, 1)] +
                               P[IX(1, 1, 0)] * P[IX(1, 1, 2)]);
        double triples = 4.0 * P[IX(1, 1, 1)] * P[IX(1, 1, 1)] +
                         2.0 * (P[IX(1, 2, 0)] * P[IX(1, 0, 2)] + P[IX(2, 1, 0)] * P[IX(0, 1, 2)] +
                                P[IX(2, 0, 1)] * P[IX(0, 2, 1)]);
        double pairs222 = 16.0 * P[IX(1, 1, 0)] * P[IX(1, 0, 1)] * P[IX(0, 1, 1)] +
                          4.0 * (P[IX(1, 0, 1)] * P[IX(1, 0, 1)] * P[IX(0, 2, 0)] +
                                 P[IX(0, 1, 1)] * P[IX(0, 1, 1)] * P[IX(2, 0, 0)] +
                                 P[IX(1, 1, 0)] * P[IX(1, 1, 0)] * P[IX(0, 0, 2)]) +
                          2.0 * P[IX(2, 0, 0)] * P[IX(0, 2, 0)] * P[IX(0, 0, 2)];
        K[IX(2, 2, 2)] = P[IX(2, 2, 2)] - pairs4 - triples + pairs222;
    }
}

/* Cumulants -> central moments, the inverse of the relations above, each
 * higher order built from the already reconstructed lower orders. */
void orc_central_from_cumulants(int dim, const double *K, double *P)
{
    int i;
    for (i = 0; i < 27; i++) P[i] = K[i];
    if (dim == 2) {
        P[IX(2, 2, 0)] = K[IX(2, 2, 0)] + (P[IX(2, 0, 0)] * P[IX(0, 2, 0)] + 2.0 * P[IX(1, 1, 0)] * P[IX(1, 1, 0)]);
        return;
    }
    P[IX(2, 1, 1)] = K[IX(2, 1, 1)] + (P[IX(2, 0, 0)] * P[IX(0, 1, 1)] + 2.0 * P[IX(1, 1, 0)] * P[IX(1, 0, 1)]);
    P[IX(1, 2, 1)] = K[IX(1, 2, 1)] + (P[IX(0, 2, 0)] * P[IX(1, 0, 1)] + 2.0 * P[IX(1, 1, 0)] * P[IX(0, 1, 1)]);
    P[IX(1, 1, 2)] = K[IX(1, 1, 2)] + (P[IX(0, 0, 2)] * P[IX(1, 1, 0)] + 2.0 * P[IX(1, 0, 1)] * P[IX(0, 1, 1)]);
    P[IX(2, 2, 0)] = K[IX(2, 2, 0)] + (P[IX(2, 0, 0)] * P[IX(0, 2, 0)] + 2.0 * P[IX(1, 1, 0)] * P[IX(1, 1, 0)]);
    P[IX(2, 0, 2)] = K[IX(2, 0, 2)] + (P[IX(2, 0, 0)] * P[IX(0, 0, 2)] + 2.0 * P[IX(1, 0, 1)] * P[IX(1, 0, 1)]);
    P[IX(0, 2, 2)] = K[IX(0, 2, 2)] + (P[IX(0, 2, 0)] * P[IX(0, 0, 2)] + 2.0 * P[IX(0, 1, 1)] * P[IX(0, 1, 1)]);
    P[IX(1, 2, 2)] = K[IX(1, 2, 2)] + (P[IX(0, 0, 2)] * P[IX(1, 2, 0)] + P[IX(0, 2, 0)] * P[IX(1, 0, 2)] +
                                       4.0 * P[IX(0, 1, 1)] * P[IX(1, 1, 1)] +
                                       2.0 * (P[IX(1, 0, 1)] * P[IX(0, 2, 1)] + P[IX(1, 1, 0)] * P[IX(0, 1, 2)]));
    P[IX(2, 1, 2)] = K[IX(2, 1, 2)] + (P[IX(0, 0, 2)] * P[IX(2, 1, 0)] + P[IX(2, 0, 0)] * P[IX(0, 1, 2)] +
                                       4.0 * P[IX(1, 0, 1)] * P[IX(1, 1, 1)] +
                                       2.0 * (P[IX(0, 1, 1)] * P[IX(2, 0, 1)] + P[IX(1, 1, 0)] * P[IX(1, 0, 2)]));
    P[IX(2, 2, 1)] = K[IX(2, 2, 1)] + (P[IX(2, 0, 0)] * P[IX(0, 2, 1)] + P[IX(0, 2, 0)] * P[IX(2, 0, 1)] +
                                       4.0 * P[IX(1, 1, 0)] * P[IX(1, 1, 1)] +
                                       2.0 * (P[IX(1, 0, 1)] * P[IX(1, 2, 0)] + P[IX(0, 1, 1)] * P[IX(2, 1, 0)]));
    {
        double pairs4 = P[IX(2, 0, 0)] * P[IX(0, 2, 2)] + P[IX(0, 2, 0)] * P[IX(2, 0, 2)] +
                        P[IX(0, 0, 2)] * P[IX(2, 2, 0)] +
                        4.0 * (P[IX(0, 1, 1)] * P[IX(2, 1, 1)] + P[IX(1, 0, 1)] * P[IX(1, 2, 1)] +
                               P[IX(1, 1, 0)] * P[IX(1, 1, 2)]);
        double triples = 4.0 * P[IX(1, 1, 1)] * P[IX(1, 1, 1)] +
                         2.0 * (P[IX(1, 2, 0)] * P[IX(1, 0, 2)] + P[IX(2, 1, 0)] * P[IX(0, 1, 2)] +
                                P[IX(2, 0, 1)] * P[IX(0, 2, 1)]);
        double pairs222 = 16.0 * P[IX(1, 1, 0)] * P[IX(1, 0, 1)] * P[IX(0, 1, 1)] +
                          4.0 * (P[IX(1, 0, 1)] * P[IX(1, 0, 1)] * P[IX(0, 2, 0)] +
                                 P[IX(0, 1, 1)] * P[IX(0, 1, 1)] * P[IX(2, 0, 0)] +
                                 P[IX(1, 1, 0)] * P[IX(1, 1, 0)] * P[IX(0, 0, 2)]) +
                          2.0 * P[IX(2, 0, 0)] * P[IX(0, 2, 0)] * P[IX(0, 0, 2)];
        P[IX(2, 2, 2)] = K[IX(2, 2, 2)] + pairs4 + triples - pairs222;
    }
}

/* Populations with prescribed central moments about u: solve the dense
 * Q x Q system  sum_a (c_ax-ux)^a (c_ay-uy)^b (c_az-uz)^c h_a = Pi_abc
 * by Gaussian elimination with partial pivoting. */
int orc_populations_from_central(int dim, const double *Pi27, const double *u, double *h)
{
    lat_t L;
    double A[QMAX][QMAX + 1];
    int rows = 0, a, b, c, al, i, j, k;
    lat_get(dim, &L);
    for (a = 0; a < 3; a++)
        for (b = 0; b < 3; b++)
            for (c = 0; c < (dim == 2 ? 1 : 3); c++) {
                for (al = 0; al < L.Q; al++)
                    A[rows][al] = ipow(L.c[al][0] - u[0], a) * ipow(L.c[al][1] - u[1], b) *
                                  ipow(L.c[al][2] - u[2], c);
                A[rows][L.Q] = Pi27[IX(a, b, c)];
                rows++;
            }
    for (k = 0; k < L.Q; k++) {
        int piv = k;
        for (i = k + 1; i < L.Q; i++)
            if (fabs(A[i][k]) > fabs(A[piv][k])) piv = i;
        if (fabs(A[piv][k]) < 1e-300) return -1;
        if (piv != k)
            for (j = 0; j <= L.Q; j++) {
                double t = A[k][j];
                A[k][j] = A[piv][j];
                A[piv][j] = t;
            }
        for (i = k + 1; i < L.Q; i++) {
            double m = A[i][k] / A[k][k];
            for (j = k; j <= L.Q; j++) A[i][j] -= m * A[k][j];
        }
    }
    for (i = L.Q - 1; i >= 0; i--) {
        double s = A[i][L.Q];
        for (j = i + 1; j < L.Q; j++) s -= A[i][j] * h[j];
        h[i] = s / A[i][i];
    }
    return 0;
}

/* Cumulant relaxation.  Viscous modes (off-diagonal and deviatoric second
 * order) relax with omega toward 0; the trace relaxes with rate_bulk toward
 * dim*cs^2; orders 3..6 relax with their rates toward 0. */
static void relax_cumulants(const orc_params *p, double omega, const double *K, double *Ks)
{
    int a, b, c, i;
    for (i = 0; i < 27; i++) Ks[i] = K[i];
    if (p->dim == 2) {
        double A = K[IX(2, 0, 0)] - K[IX(0, 2, 0)];
        double S = K[IX(2, 0, 0)] + K[IX(0, 2, 0)];
        double As = (1.0 - omega) * A;
        double Ss = S + p->rate_bulk * (2.0 * CS2 - S);
        Ks[IX(2, 0, 0)] = (Ss + As) / 2.0;
        Ks[IX(0, 2, 0)] = (Ss - As) / 2.0;
        Ks[IX(1, 1, 0)] = (1.0 - omega) * K[IX(1, 1, 0)];
    } else {
        double A = K[IX(2, 0, 0)] - K[IX(0, 2, 0)];
        double B = K[IX(2, 0, 0)] - K[IX(0, 0, 2)];
        double S = K[IX(2, 0, 0)] + K[IX(0, 2, 0)] + K[IX(0, 0, 2)];
        double As = (1.0 - omega) * A, Bs = (1.0 - omega) * B;
        double Ss = S + p->rate_bulk * (3.0 * CS2 - S);
        Ks[IX(2, 0, 0)] = (Ss + As + Bs) / 3.0;
        Ks[IX(0, 2, 0)] = (Ss - 2.0 * As + Bs) / 3.0;
        Ks[IX(0, 0, 2)] = (Ss + As - 2.0 * Bs) / 3.0;
        Ks[IX(1, 1, 0)] = (1.0 - omega) * K[IX(1, 1, 0)];
        Ks[IX(1, 0, 1)] = (1.0 - omega) * K[IX(1, 0, 1)];
        Ks[IX(0, 1, 1)] = (1.0 - omega) * K[IX(0, 1, 1)];
    }
    for (a = 0; a < 3; a++)
        for (b = 0; b < 3; b++)
            for (c = 0; c < 3; c++) {
                int ord = a + b + c;
                double r = ord == 3 ? p->rate3 : ord == 4 ? p->rate4 : ord == 5 ? p->rate5 : ord == 6 ? p->rate6 : -1.0;
                if (r >= 0.0) Ks[IX(a, b, c)] = (1.0 - r) * K[IX(a, b, c)];
            }
}

/* ----------------------------------------------------------------------- */
/* One cell: closure, flow collision (Sec. 2.3), phase-field collision      */
/* (Sec. 2.2).                                                              */
/* ----------------------------------------------------------------------- */
int orc_collide_cell(const orc_params *p, const double *f, const double *g, double phi,
                     const double *grad, double lap, double *fo, double *go, double *diag,
                     const double *phiu_prev, double *phiu_out)
{
    lat_t L;
    double rho, grad_rho[3], beta, kappa, mu, F[3], nrm, n[3], nu, tau, omega;
    double u[3], Gam[QMAX], Xi[QMAX], fp[QMAX], h[QMAX], P, pstar;
    double Pi[27], K[27], Ks[27], Pis[27], hs[QMAX];
    double tau_phi, tpb, geq[QMAX], Sbar[QMAX];
    int a, i, Q;
    double dg[ORC_DIAG_SIZE];
    double gr[3], gv[3];
    lat_get(p->dim, &L);
    Q = L.Q;
    memset(dg, 0, sizeof(dg));
    /* in 2-D only the in-plane components exist */
    for (i = 0; i < 3; i++) {
        gr[i] = i < p->dim ? grad[i] : 0.0;
        gv[i] = i < p->dim ? p->g[i] : 0.0;
    }
    grad = gr;

    /* density interpolation and its gradient (Sec. 2.3) */
    rho = p->rho_l + (p->rho_h - p->rho_l) * phi;
    for (i = 0; i < 3; i++) grad_rho[i] = (p->rho_h - p->rho_l) * grad[i];
    /* chemical potential and free parameters (Sec. 2.1) */
    beta = 12.0 * p->sigma / p->W;
    kappa = 1.5 * p->sigma * p->W;
    mu = 2.0 * beta * phi * (phi - 1.0) * (2.0 * phi - 1.0) - kappa * lap;
    /* forces: surface tension mu grad(phi) plus body force rho g */
    for (i = 0; i < 3; i++) F[i] = mu * grad[i] + rho * gv[i];
    /* interface normal */
    nrm = sqrt(grad[0] * grad[0] + grad[1] * grad[1] + grad[2] * grad[2] + 1e-24);
    for (i = 0; i < 3; i++) n[i] = grad[i] / nrm;
    /* viscosity and relaxation: tau = nu/cs^2, taubar = tau + 1/2 */
    if (p->visc_interp == 1)
        nu = (p->rho_l * p->nu_l + (p->rho_h * p->nu_h - p->rho_l * p->nu_l) * phi) / rho;
    else
        nu = p->nu_l + (p->nu_h - p->nu_l) * phi;
    tau = nu / CS2;
    omega = 1.0 / (tau + 0.5);

    /* velocity: first moment of the preconditioned populations */
    for (i = 0; i < 3; i++) {
        double s = 0.0;
        for (a = 0; a < Q; a++) s += L.c[a][i] * f[a];
        u[i] = s / (rho * CS2) + F[i] / (2.0 * rho);
    }
    /* Gamma = f_eq / rho, and the source Xi (dilatation term dropped) */
    for (a = 0; a < Q; a++) {
        double cu_grad = 0.0, cu_F = 0.0;
        Gam[a] = L.w[a] * hermite_sum(L.c[a], u, 0);
        for (i = 0; i < 3; i++) {
            cu_grad += (L.c[a][i] - u[i]) * grad_rho[i];
            cu_F += (L.c[a][i] - u[i]) * F[i];
        }
        Xi[a] = CS2 * (Gam[a] - L.w[a]) * cu_grad + cu_F * Gam[a];
    }

    if (p->collision == ORC_COLL_SRT) {
        /* BGK form of the flow collision, discretised with the half source */
        double s0 = 0.0, sxi = 0.0;
        for (a = 0; a < Q; a++) {
            s0 += f[a];
            sxi += Xi[a];
        }
        pstar = s0 + 0.5 * sxi;
        P = pstar / (rho * CS2);
        for (a = 0; a < Q; a++) {
            double feq = L.w[a] * pstar + L.w[a] * rho * CS2 * hermite_sum(L.c[a], u, 1);
            fo[a] = f[a] - omega * (f[a] - feq) + (1.0 - 0.5 * omega) * Xi[a];
        }
    } else {
        /* preconditioning: f^p = f'/(rho cs^2) + Xi/(2 rho cs^2) */
        P = 0.0;
        for (a = 0; a < Q; a++) {
            fp[a] = f[a] / (rho * CS2) + Xi[a] / (2.0 * rho * CS2);
            P += fp[a];
        }
        pstar = rho * CS2 * P;
        /* unit-mass set carried through the cumulant transforms */
        for (a = 0; a < Q; a++) h[a] = fp[a] - L.w[a] * (P - 1.0);
        orc_central_moments(p->dim, h, u, Pi);
        orc_cumulants_from_central(p->dim, Pi, K);
        relax_cumulants(p, omega, K, Ks);
        orc_central_from_cumulants(p->dim, Ks, Pis);
        if (orc_populations_from_central(p->dim, Pis, u, hs)) return -2;
        /* f'* = rho cs^2 f^p* + Xi/2 with f^p* = h* + w (P - 1) */
        for (a = 0; a < Q; a++) fo[a] = rho * CS2 * (hs[a] + L.w[a] * (P - 1.0)) + 0.5 * Xi[a];
        for (a = 0; a < Q; a++) {
            dg[D_H + a] = h[a];
            dg[D_HS + a] = hs[a];
        }
        for (i = 0; i < 27; i++) {
            dg[D_PI + i] = Pi[i];
            dg[D_K + i] = K[i];
            dg[D_KS + i] = Ks[i];
            dg[D_PIS + i] = Pis[i];
        }
    }

    /* conservative Allen-Cahn: BGK toward the equilibrium, plus the discrete
     * antidiffusion source (Sec. 2.2).  With the first-order equilibrium the
     * discrete correction term Cbar = (1 - 1/(2 taubar)) (w / cs^2) c.d(phi u)/dt
     * is added; the time derivative is the backward difference over one step
     * (zero when no previous (phi u) is given). */
    tau_phi = p->M / CS2;
    tpb = tau_phi + 0.5;
    {
        double phiu[3], dphiu[3];
        for (i = 0; i < 3; i++) {
            phiu[i] = phi * u[i];
            dphiu[i] = (p->cac_edf == 1 && phiu_prev) ? phiu[i] - phiu_prev[i] : 0.0;
            if (phiu_out) phiu_out[i] = phiu[i];
        }
        for (a = 0; a < Q; a++) {
            double cn = 0.0, cd = 0.0, Cbar = 0.0;
            for (i = 0; i < 3; i++) {
                cn += L.c[a][i] * n[i];
                cd += L.c[a][i] * dphiu[i];
            }
            if (p->cac_edf == 1) {
                geq[a] = L.w[a] * phi * hermite_sum_first(L.c[a], u);
                Cbar = (1.0 - 1.0 / (2.0 * tpb)) * L.w[a] / CS2 * cd;
            } else {
                geq[a] = L.w[a] * phi * hermite_sum(L.c[a], u, 0);
            }
            Sbar[a] = (1.0 - 1.0 / (2.0 * tpb)) * L.w[a] * cn * 4.0 * phi * (1.0 - phi) / p->W;
            go[a] = (1.0 - 1.0 / tpb) * g[a] + geq[a] / tpb + Sbar[a] + Cbar;
        }
    }

    if (diag) {
        for (i = 0; i < 3; i++) {
            dg[D_U + i] = u[i];
            dg[D_F + i] = F[i];
            dg[D_N + i] = n[i];
        }
        dg[D_RHO] = rho;
        dg[D_P] = P;
        dg[D_PSTAR] = pstar;
        dg[D_OMEGA] = omega;
        dg[D_MU] = mu;
        dg[D_TAUPHI] = tpb;
        for (a = 0; a < Q; a++) {
            dg[D_XI + a] = Xi[a];
            dg[D_GEQ + a] = geq[a];
            dg[D_SBAR + a] = Sbar[a];
        }
        memcpy(diag, dg, sizeof(dg));
    }
    return 0;
}

/* ----------------------------------------------------------------------- */
/* Initial state.  The scheme's velocity is the first moment of f' plus half */
/* the force, and its pressure is the zeroth moment plus half the source, so */
/* the populations are the equilibria at velocity u - F/(2 rho) and pressure */
/* p - sum(Xi)/2: the velocity and pressure the scheme reports at t = 0 are  */
/* then exactly the prescribed ones.  g = g_eq(phi, u).                      */
/* ----------------------------------------------------------------------- */
int orc_init(const orc_params *p, const double *phi, const double *u, const double *ph,
             double *f, double *g)
{
    lat_t L;
    long N, row;
    if (check_params(p)) return -1;
    lat_get(p->dim, &L);
    N = ncells(p);
#pragma omp parallel for schedule(static)
    for (row = 0; row < (long)p->n[1] * p->n[2]; row++) {
        int x, a, i, y = (int)(row % p->n[1]), z = (int)(row / p->n[1]);
        for (x = 0; x < p->n[0]; x++) {
            long idx = cell_index(p, x, y, z);
            double uu[3], upop[3], p0, gr[3], lp, rho, beta, kappa, mu, F[3], sxi = 0.0, ppop;
            stencil(p, &L, phi, NULL, x, y, z, &p0, gr, &lp);
            for (i = 0; i < 3; i++) {
                uu[i] = i < p->dim ? u[(long)i * N + idx] : 0.0;
                if (i >= p->dim) gr[i] = 0.0;
            }
            rho = p->rho_l + (p->rho_h - p->rho_l) * p0;
            beta = 12.0 * p->sigma / p->W;
            kappa = 1.5 * p->sigma * p->W;
            mu = 2.0 * beta * p0 * (p0 - 1.0) * (2.0 * p0 - 1.0) - kappa * lp;
            for (i = 0; i < 3; i++) {
                F[i] = mu * gr[i] + rho * (i < p->dim ? p->g[i] : 0.0);
                upop[i] = uu[i] - F[i] / (2.0 * rho);
            }
            for (a = 0; a < L.Q; a++) {
                double Gam = L.w[a] * hermite_sum(L.c[a], uu, 0), cg = 0.0, cf = 0.0;
                for (i = 0; i < 3; i++) {
                    cg += (L.c[a][i] - uu[i]) * (p->rho_h - p->rho_l) * gr[i];
                    cf += (L.c[a][i] - uu[i]) * F[i];
                }
                sxi += CS2 * (Gam - L.w[a]) * cg + cf * Gam;
            }
            ppop = ph[idx] - 0.5 * sxi;
            for (a = 0; a < L.Q; a++) {
                f[(long)a * N + idx] = L.w[a] * ppop + L.w[a] * rho * CS2 * hermite_sum(L.c[a], upop, 1);
                g[(long)a * N + idx] = L.w[a] * p0 * hermite_sum(L.c[a], uu, 0);
            }
        }
    }
    return 0;
}

/* ----------------------------------------------------------------------- */
/* Streaming: f_a(x, t+1) = f*_a(x - c_a).  If the source lies beyond a     */
/* wall, the population is the bounced-back f*_{opp(a)}(x).  A source beyond */
/* a symmetry plane is mirrored: same cell on that axis, that velocity       */
/* component reversed.  Periodic axes wrap.                                  */
/* ----------------------------------------------------------------------- */
static void stream_source(const orc_params *p, const lat_t *L, int x, int y, int z, int a,
                          long *src_cell, int *src_dir)
{
    int xs[3] = {x, y, z}, s[3], cdir[3], i, b, wall = 0;
    for (i = 0; i < 3; i++) {
        cdir[i] = L->c[a][i];
        s[i] = xs[i] - L->c[a][i];
        if (s[i] < 0 || s[i] >= p->n[i]) {
            if (p->bc[i] == ORC_BC_PERIODIC)
                s[i] = (s[i] + p->n[i]) % p->n[i];
            else if (p->bc[i] == ORC_BC_WALL)
                wall = 1;
            else {
                s[i] = xs[i];
                cdir[i] = -cdir[i];
            }
        }
    }
    if (wall) {
        *src_cell = cell_index(p, x, y, z);
        *src_dir = L->opp[a];
        return;
    }
    *src_cell = cell_index(p, s[0], s[1], s[2]);
    for (b = 0; b < L->Q; b++)
        if (L->c[b][0] == cdir[0] && L->c[b][1] == cdir[1] && L->c[b][2] == cdir[2]) *src_dir = b;
}

static void gather_cell(const double *arr, long N, int Q, long idx, double *out)
{
    int a;
    for (a = 0; a < Q; a++) out[a] = arr[(long)a * N + idx];
}

int orc_step(const orc_params *p, const double *f, const double *g, double *fo, double *go)
{
    return orc_step_hist(p, f, g, fo, go, NULL, 0);
}

int orc_step_hist(const orc_params *p, const double *f, const double *g, double *fo, double *go,
                  double *phiu, int have_prev)
{
    lat_t L;
    long N;
    double *phi, *fs, *gs;
    long row;
    int z, err = 0;
    if (check_params(p)) return -1;
    lat_get(p->dim, &L);
    N = ncells(p);
    phi = (double *)malloc(sizeof(double) * N);
    fs = (double *)malloc(sizeof(double) * N * L.Q);
    gs = (double *)malloc(sizeof(double) * N * L.Q);
    if (!phi || !fs || !gs) {
        free(phi);
        free(fs);
        free(gs);
        return -3;
    }
    /* order parameter: zeroth moment of the phase-field populations */
#pragma omp parallel for schedule(static)
    for (z = 0; z < p->n[2]; z++) {
        long idx;
        for (idx = (long)z * p->n[0] * p->n[1]; idx < (long)(z + 1) * p->n[0] * p->n[1]; idx++)
            phi[idx] = phi_from_g(&L, g, N, idx);
    }
    /* collision at every cell */
#pragma omp parallel for schedule(static) reduction(| : err)
    for (row = 0; row < (long)p->n[1] * p->n[2]; row++) {
        int x, a, y = (int)(row % p->n[1]), z = (int)(row / p->n[1]);
        for (x = 0; x < p->n[0]; x++) {
            double fc[QMAX], gc[QMAX], fpost[QMAX], gpost[QMAX], p0, gr[3], lp;
            long idx = cell_index(p, x, y, z);
            stencil(p, &L, phi, NULL, x, y, z, &p0, gr, &lp);
            gather_cell(f, N, L.Q, idx, fc);
            gather_cell(g, N, L.Q, idx, gc);
            {
                double prev[3], cur[3];
                int i;
                if (phiu && have_prev)
                    for (i = 0; i < 3; i++) prev[i] = phiu[(long)i * N + idx];
                err |= orc_collide_cell(p, fc, gc, p0, gr, lp, fpost, gpost, NULL,
                                        (phiu && have_prev) ? prev : NULL, cur);
                /* each cell reads only its own previous value: update in place */
                if (phiu)
                    for (i = 0; i < 3; i++) phiu[(long)i * N + idx] = cur[i];
            }
            for (a = 0; a < L.Q; a++) {
                fs[(long)a * N + idx] = fpost[a];
                gs[(long)a * N + idx] = gpost[a];
            }
        }
    }
    /* streaming */
#pragma omp parallel for schedule(static)
    for (row = 0; row < (long)p->n[1] * p->n[2]; row++) {
        int x, a, sd, y = (int)(row % p->n[1]), z = (int)(row / p->n[1]);
        long sc;
        for (x = 0; x < p->n[0]; x++) {
            long idx = cell_index(p, x, y, z);
            for (a = 0; a < L.Q; a++) {
                stream_source(p, &L, x, y, z, a, &sc, &sd);
                fo[(long)a * N + idx] = fs[(long)sd * N + sc];
                go[(long)a * N + idx] = gs[(long)sd * N + sc];
            }
        }
    }
    free(phi);
    free(fs);
    free(gs);
    return err ? -2 : 0;
}

/* One step evaluated only at the listed cells: each streamed population is
 * obtained by colliding its source cell, with phi recomputed from g. */
int orc_step_sampled(const orc_params *p, const double *f, const double *g, const long *cells,
                     long m, double *fo, double *go)
{
    lat_t L;
    long N, k;
    int err = 0;
    if (check_params(p)) return -1;
    lat_get(p->dim, &L);
    N = ncells(p);
#pragma omp parallel for schedule(dynamic, 4) reduction(| : err)
    for (k = 0; k < m; k++) {
        long idx = cells[k], sc;
        int x = (int)(idx % p->n[0]);
        int y = (int)((idx / p->n[0]) % p->n[1]);
        int z = (int)(idx / ((long)p->n[0] * p->n[1]));
        int a, sd;
        for (a = 0; a < L.Q; a++) {
            double fc[QMAX], gc[QMAX], fpost[QMAX], gpost[QMAX], p0, gr[3], lp;
            int sx, sy, sz;
            stream_source(p, &L, x, y, z, a, &sc, &sd);
            sx = (int)(sc % p->n[0]);
            sy = (int)((sc / p->n[0]) % p->n[1]);
            sz = (int)(sc / ((long)p->n[0] * p->n[1]));
            stencil(p, &L, NULL, g, sx, sy, sz, &p0, gr, &lp);
            gather_cell(f, N, L.Q, sc, fc);
            gather_cell(g, N, L.Q, sc, gc);
            err |= orc_collide_cell(p, fc, gc, p0, gr, lp, fpost, gpost, NULL, NULL, NULL);
            fo[k * L.Q + a] = fpost[sd];
            go[k * L.Q + a] = gpost[sd];
        }
    }
    return err ? -2 : 0;
}

/* Macroscopic fields of the pre-collision state: phi, rho, u (with the half
 * force) and p_h = sum f' + sum Xi / 2. */
int orc_fields(const orc_params *p, const double *f, const double *g, double *phi, double *rho,
               double *u, double *ph)
{
    lat_t L;
    long N, row;
    int z, err = 0;
    double *phf;
    if (check_params(p)) return -1;
    lat_get(p->dim, &L);
    N = ncells(p);
    phf = (double *)malloc(sizeof(double) * N);
    if (!phf) return -3;
    for (z = 0; z < p->n[2]; z++) {
        long idx;
        for (idx = (long)z * p->n[0] * p->n[1]; idx < (long)(z + 1) * p->n[0] * p->n[1]; idx++)
            phf[idx] = phi_from_g(&L, g, N, idx);
    }
#pragma omp parallel for schedule(static) reduction(| : err)
    for (row = 0; row < (long)p->n[1] * p->n[2]; row++) {
        int x, i, y = (int)(row % p->n[1]), z = (int)(row / p->n[1]);
        for (x = 0; x < p->n[0]; x++) {
            double fc[QMAX], gc[QMAX], fpost[QMAX], gpost[QMAX], p0, gr[3], lp;
            double dg[ORC_DIAG_SIZE];
            long idx = cell_index(p, x, y, z);
            stencil(p, &L, phf, NULL, x, y, z, &p0, gr, &lp);
            gather_cell(f, N, L.Q, idx, fc);
            gather_cell(g, N, L.Q, idx, gc);
            err |= orc_collide_cell(p, fc, gc, p0, gr, lp, fpost, gpost, dg, NULL, NULL);
            if (phi) phi[idx] = p0;
            if (rho) rho[idx] = dg[D_RHO];
            if (u)
                for (i = 0; i < 3; i++) u[(long)i * N + idx] = dg[D_U + i];
            if (ph) ph[idx] = dg[D_PSTAR];
        }
    }
    free(phf);
    return err ? -2 : 0;
}

/* sum phi, sum rho u (3 components), max |u| over the lattice; serial and
 * in cell order */
int orc_reduce(const orc_params *p, const double *f, const double *g, double *out5)
{
    long N = ncells(p), idx;
    double *phi, *rho, *u;
    int i, err;
    if (check_params(p)) return -1;
    phi = (double *)malloc(sizeof(double) * N);
    rho = (double *)malloc(sizeof(double) * N);
    u = (double *)malloc(sizeof(double) * N * 3);
    if (!phi || !rho || !u) {
        free(phi);
        free(rho);
        free(u);
        return -3;
    }
    err = orc_fields(p, f, g, phi, rho, u, NULL);
    for (i = 0; i < 5; i++) out5[i] = 0.0;
    for (idx = 0; idx < N; idx++) {
        double m = 0.0;
        out5[0] += phi[idx];
        for (i = 0; i < 3; i++) {
            out5[1 + i] += rho[idx] * u[(long)i * N + idx];
            m += u[(long)i * N + idx] * u[(long)i * N + idx];
        }
        m = sqrt(m);
        if (m > out5[4]) out5[4] = m;
    }
    free(phi);
    free(rho);
    free(u);
    return err;
}
