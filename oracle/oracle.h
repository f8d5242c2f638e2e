/*
 * Plain FP64 CPU oracle for the multiphase lattice Boltzmann step of
 * Hosseini, Safari & Thevenin (arXiv 2101.06769): pressure-based low-Mach
 * flow populations under the cumulant collision operator (Sec. 2.3), coupled
 * to conservative Allen-Cahn phase-field populations (Sec. 2.2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code; it exists so that the GPU path can be checked against a
 * slow, literal transcription of the method.  It shares no source with the
 * GPU library.
 *
 * Layout of every population array: [Q][nz][ny][nx] doubles, x fastest,
 * in this file's own velocity ordering (see orc_lattice).  The state held in
 * the arrays is the pre-collision (post-streaming) population set at time n.
 * Scalar fields: [nz][ny][nx]; vector fields: [3][nz][ny][nx].
 */
#ifndef MPLB_ORACLE_H
#define MPLB_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BC_PERIODIC = 0, ORC_BC_WALL = 1, ORC_BC_SYMMETRY = 2 };
enum { ORC_COLL_CUMULANT = 0, ORC_COLL_SRT = 1 };

typedef struct {
    int dim;            /* 2 (D2Q9) or 3 (D3Q27) */
    int n[3];           /* nx, ny, nz; nz = 1 in 2-D */
    int bc[3];          /* per axis, both faces */
    double rho_h, rho_l;
    double nu_h, nu_l;  /* kinematic viscosities */
    double W, M, sigma; /* interface width, mobility, surface tension */
    double g[3];        /* body-force acceleration, F_b = rho g */
    int visc_interp;    /* 0: nu linear in phi; 1: dynamic viscosity linear in phi */
    int collision;      /* ORC_COLL_* */
    /* relaxation rates of the non-viscous cumulant groups (all 1 in the paper) */
    double rate_bulk, rate3, rate4, rate5, rate6;
    /* phase-field equilibrium: 0 second-order (the paper's choice); 1
     * first-order plus the correction term of Sec. 2.2 */
    int cac_edf;
} orc_params;

/* number of diag doubles written by orc_collide_cell */
#define ORC_DIAG_SIZE 320

int  orc_Q(int dim);
void orc_lattice(int dim, int *c /* Q*3 */, double *w /* Q */, int *opp /* Q */);
void orc_set_threads(int nthreads);
int  orc_num_threads(void);

int orc_gradients(const orc_params *p, const double *phi, double *grad, double *lap);
int orc_init(const orc_params *p, const double *phi, const double *u, const double *ph,
             double *f, double *g);
int orc_step(const orc_params *p, const double *f, const double *g, double *fo, double *go);
/* One step with the history the first-order phase-field equilibrium needs:
 * phiu holds (phi u) per cell ([3][N]) of the previous step when have_prev
 * is non-zero, and receives this step's; without history the time
 * derivative of (phi u) is taken as zero. */
int orc_step_hist(const orc_params *p, const double *f, const double *g, double *fo, double *go,
                  double *phiu, int have_prev);
int orc_step_sampled(const orc_params *p, const double *f, const double *g,
                     const long *cells, long m, double *fo, double *go);
int orc_fields(const orc_params *p, const double *f, const double *g,
               double *phi, double *rho, double *u, double *ph);
int orc_reduce(const orc_params *p, const double *f, const double *g, double *out5);

int  orc_collide_cell(const orc_params *p, const double *f, const double *g, double phi,
                      const double *grad, double lap, double *fo, double *go, double *diag,
                      const double *phiu_prev, double *phiu_out);
void orc_central_moments(int dim, const double *h, const double *u, double *Pi27);
void orc_cumulants_from_central(int dim, const double *Pi27, double *K27);
void orc_central_from_cumulants(int dim, const double *K27, double *Pi27);
int  orc_populations_from_central(int dim, const double *Pi27, const double *u, double *h);

#ifdef __cplusplus
}
#endif
#endif
