/*
 * mplb.h -- C ABI of the MI355X (gfx950) multiphase lattice Boltzmann library.
 *
 * One time step advances two coupled population sets on a regular lattice
 * (arXiv 2101.06769):
 *   - conservative Allen-Cahn phase-field populations g (Sec. 2.2): BGK
 *     collision toward a second-order equilibrium plus the antidiffusion
 *     source, order parameter phi = sum_a g_a;
 *   - pressure-based low-Mach flow populations f' (Sec. 2.3): preconditioned
 *     populations, cumulant collision (viscosity on the second-order
 *     off-diagonal and deviatoric cumulants, all other rates unity), source
 *     Xi carrying the density gradient, surface tension mu grad(phi) and the
 *     body force;
 * coupled through isotropic finite-difference gradients and Laplacians of
 * phi (Sec. 2.2) and the linear density interpolation rho(phi) (Sec. 2.3).
 * Lattices: D2Q9 (dim 2) and D3Q27 (dim 3).  Lattice units: dt = dx = 1,
 * cs^2 = 1/3, heavy density 1 (Sec. 3).
 *
 * Conventions
 *   - Every function returns an int status (MPLB_OK = 0, negative on error)
 *     unless stated; none throws.  mplb_last_error() gives a message for the
 *     most recent failure on the calling thread.
 *   - Host arrays are double precision, C order with x fastest:
 *     scalar fields [nz][ny][nx]; vector fields [dim][nz][ny][nx];
 *     populations [Q][nz][ny][nx].
 *   - Population order a = (cx+1) + 3 (cy+1) [+ 9 (cz+1)]: velocity
 *     components are read off the base-3 digits of a.  Opposite: Q-1-a.
 *   - "State at time n" means the pre-collision populations at every cell
 *     (after streaming).  The library stores post-collision values and
 *     streams by pulling, but every exchange through this header uses the
 *     pre-collision view.
 *   - Ownership: the caller owns the device arena (any device allocation of
 *     at least mplb_state_bytes() bytes, e.g. a torch uint8 tensor) and all
 *     host buffers.  The library carves the arena and never allocates or
 *     frees device memory; it owns only its handle and, once the handle has
 *     stepped, its step graph and capture stream (mplb_step).
 *   - Stream: all device work is queued on the hipStream_t given at create
 *     time (NULL = the null stream).  Calls are asynchronous unless stated;
 *     calls that return host data synchronise that stream.
 *   - One handle per stream; handles are not thread-safe.
 */
#ifndef MPLB_H
#define MPLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPLB_VERSION 1

enum {
    MPLB_OK = 0,
    MPLB_EINVAL = -1,    /* invalid argument or parameter */
    MPLB_ENOMEM = -2,    /* arena smaller than mplb_state_bytes() */
    MPLB_EDEVICE = -3,   /* HIP runtime error (message in mplb_last_error) */
    MPLB_EUNSTABLE = -4, /* non-finite value found by mplb_reduce or mplb_batch_status */
    MPLB_ESTATE = -5     /* call not valid in the handle's current state */
};

/* Boundary type per axis (both faces of that axis). */
enum {
    MPLB_BC_PERIODIC = 0,
    MPLB_BC_WALL = 1,    /* half-way bounce-back no-slip wall (Sec. 3.2, 3.4);
                            phi ghost layer mirrors the first fluid layer */
    MPLB_BC_SYMMETRY = 2 /* specular free-slip plane (Sec. 3.4, side walls) */
};

/* Population storage format.  Arithmetic is FP64 for MPLB_STORE_FP64 and
 * FP32 otherwise; global reductions are always FP64. */
enum {
    MPLB_STORE_FP64 = 0,
    MPLB_STORE_FP32 = 1,
    MPLB_STORE_FP16S = 2,    /* f': per moving direction the FP16 code
                                q = (f'/w - P)/s against the writing cell's
                                references P = fp16(p*), s = rho(fp16(phi)) cs^2,
                                rest direction FP32; g FP32 */
    MPLB_STORE_FP16S_ALL = 3 /* f' as above; g: the FP16 code q = g/w - F against
                                the reading cell's F = fp16(phi), rest direction
                                FP32 */
};

/* Flow collision operator. */
enum {
    MPLB_COLL_CUMULANT = 0, /* the paper's operator (Sec. 2.3) */
    MPLB_COLL_SRT = 1       /* single-relaxation-time form of the same kinetic
                               equation (Sec. 2.3, BGK collision), for comparison */
};

/* Fields for mplb_read. */
enum {
    MPLB_FIELD_PHI = 0, /* order parameter, sum_a g_a */
    MPLB_FIELD_RHO = 1, /* rho_l + (rho_h - rho_l) phi */
    MPLB_FIELD_UX = 2,  /* velocity: first moment of f'/(rho cs^2) plus F/(2 rho) */
    MPLB_FIELD_UY = 3,
    MPLB_FIELD_UZ = 4,
    MPLB_FIELD_P = 5    /* hydrodynamic pressure: sum f' + sum Xi / 2 */
};

/* Problem statement (Sec. 2.1-2.3, Sec. 3): lattice, densities, viscosities,
 * interface width, mobility, surface tension, gravity, boundaries. */
typedef struct mplb_params {
    int32_t dim;          /* 2 -> D2Q9, 3 -> D3Q27 */
    int32_t n[3];         /* nx, ny, nz (nz = 1 in 2-D); each >= 1 */
    int32_t bc[3];        /* MPLB_BC_* per axis; z ignored in 2-D */
    double rho_heavy;     /* rho_h > 0 (1 in the paper's units) */
    double rho_light;     /* rho_l > 0 */
    double nu_heavy;      /* kinematic viscosity of the heavy phase, > 0 */
    double nu_light;      /* kinematic viscosity of the light phase, > 0;
                             tau = nu/cs^2, omega = 1/(tau + 1/2) */
    double W;             /* interface thickness, >= 1 (cells) */
    double mobility;      /* M > 0; tau_phi = M/cs^2, taubar_phi = tau_phi + 1/2 */
    double sigma;         /* surface tension >= 0; beta = 12 sigma/W, kappa = 3 sigma W/2 */
    double gravity[3];    /* body-force acceleration, F_b = rho g; g[2] = 0 in 2-D */
    int32_t storage;      /* MPLB_STORE_* */
    int32_t visc_interp;  /* 0: nu = nu_l + (nu_h - nu_l) phi; 1: rho nu linear in phi */
    int32_t collision;    /* MPLB_COLL_* */
    int32_t cac_edf;      /* phase-field equilibrium (Sec. 2.2): 0 second-order (the
                             paper's); 1 first-order plus the correction term
                             (1 - 1/(2 taubar_phi)) (w/cs^2) c.d(phi u)/dt, the time
                             derivative the backward difference over one step (zero on
                             the first step after mplb_init / mplb_set_populations) */
} mplb_params;

typedef struct mplb_solver mplb_solver;

/* Library version (MPLB_VERSION) and the device architecture it was built
 * for.  Design, not in the paper. */
int32_t mplb_version(void);
const char *mplb_arch(void);

/* Bytes of device memory a solver with these parameters needs (0 if the
 * parameters are invalid; mplb_last_error says why).  The parameters are the
 * paper's statement of the problem (Sec. 2.1: densities, viscosities,
 * interface thickness W, mobility M, surface tension sigma; Sec. 3: lattice,
 * gravity, boundary types); the memory layout is this library's design. */
size_t mplb_state_bytes(const mplb_params *p);

/* Validate p and bind a solver to the caller's arena and stream.
 * dev_arena: device pointer, 256-byte aligned, at least mplb_state_bytes(p)
 * bytes, owned by the caller for the solver's lifetime.
 * hip_stream: a hipStream_t (NULL for the null stream).
 * Errors: EINVAL (bad parameters, see mplb_last_error), ENOMEM (arena too
 * small).  Design, not in the paper. */
int mplb_create(const mplb_params *p, void *dev_arena, size_t arena_bytes, void *hip_stream,
                mplb_solver **out);

/* Initial state from macroscopic fields (host, double): phi [N], u [dim][N],
 * p [N] (NULL = zero pressure).  Populations become the equilibria of
 * Sec. 2.2 (phase field, Eq. LBM_AC with the Hermite terms of Appendix A)
 * and Sec. 2.3 (flow, Eq. LMNA_distribution), taken at the velocity
 * u - F/(2 rho) and pressure p - sum(Xi)/2, so that mplb_read returns exactly
 * phi, u and p before the first step.  Resets the step counter and the
 * history.  Synchronises the stream.  Errors: EINVAL, ESTATE (attached to a
 * batch), EDEVICE. */
int mplb_init(mplb_solver *s, const double *phi, const double *u, const double *p);

/* Advance nsteps >= 0 time steps (asynchronous).  One step is the paper's
 * scheme from time n to n + 1: the order parameter as the zeroth moment of
 * the phase-field populations (Sec. 2.2), its isotropic gradient and
 * Laplacian (Sec. 2.2), density, chemical potential and forces (Sec. 2.1),
 * the flow collision with its source term (Sec. 2.3, Eqs. LMNA_LBM to
 * LMNA_distribution, cumulant relaxation), the phase-field collision with
 * the antidiffusion source (Sec. 2.2, Eqs. LBM_AC and
 * phase_source_post_discretization), and streaming with the boundary rules
 * of Sec. 3 (half-way bounce-back walls, symmetry planes, periodic axes).
 * Runs of 16 steady-state steps are launched as one captured HIP graph (the
 * same kernels and arguments, the same results; design, not in the paper):
 * the graph is captured on a stream of the handle's own at the first such
 * run and again when the level parity, the block or the step form changes.
 * Errors: EINVAL, ESTATE (not initialised, or attached to a batch),
 * EDEVICE. */
int mplb_step(mplb_solver *s, int64_t nsteps);

/* As mplb_step, but records HIP events around every kernel launch on the
 * solver's stream and returns the summed device time of the two launches of
 * each step (ms_phi: order-parameter stage; ms_collide: cell update) in
 * milliseconds.  Synchronises the stream.  For profiling; the events add a
 * few microseconds per step.  Design, not in the paper.  Errors: as
 * mplb_step. */
int mplb_step_timed(mplb_solver *s, int64_t nsteps, double *ms_phi, double *ms_collide);

/* Block until all queued work on the solver's stream has finished. */
int mplb_sync(mplb_solver *s);

/* Steps taken since mplb_init / mplb_set_populations (kept by mplb_load). */
int64_t mplb_steps_done(const mplb_solver *s);

/* One macroscopic field (MPLB_FIELD_*) of the state at time n into host_out[N]:
 * phi = sum g (Sec. 2.2), rho(phi) linear (Sec. 2.3), u the first moment of
 * f'/(rho cs^2) plus F/(2 rho) (Sec. 2.3), p = sum f' + sum(Xi)/2, the zeroth
 * moment of Eq. LMNA_distribution with half the source (the reading this
 * library takes of the pressure field).  Synchronises the stream.  Errors:
 * EINVAL, ESTATE, EDEVICE. */
int mplb_read(mplb_solver *s, int32_t field, double *host_out);

/* FP64 reductions over the lattice, deterministic (fixed summation order):
 * out[0] = sum phi (the phase mass Sec. 2.2's conservative form keeps),
 * out[1..3] = sum rho u, out[4] = max |u|.  Returns MPLB_EUNSTABLE if any
 * phi, rho u or |u| is not finite.  Synchronises the stream.  The FP64
 * reductions are this library's design, not in the paper. */
int mplb_reduce(mplb_solver *s, double out[5]);

/* mplb_reduce for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same reductions, same results, with the partial sums and the result in a
 * static device array of the library instead of the solver's arena, so the
 * call makes no allocation of any kind.  The array holds the partials of up
 * to 1024 reduction blocks (every lattice fits: the reduction uses at most
 * 1024 blocks; a larger need returns EINVAL with the sizes in the message)
 * and is looked up once per device: call with the solver's device current.
 * Every call on one device shares that array, so calls that overlap on one
 * device (other threads, other streams) race; serialise them.  Synchronises
 * the stream.  Errors: EINVAL, ESTATE, EDEVICE; EUNSTABLE as mplb_reduce. */
int mplb_reduce_noalloc(mplb_solver *s, double out[5]);

/* Pre-collision populations of the state at time n (which: 0 = f', 1 = g),
 * host_out[Q][N] in the population order above, decoded to double.
 * Synchronises the stream. */
int mplb_get_populations(mplb_solver *s, int32_t which, double *host_out);

/* Replace one population set of the state at time n (which: 0 = f', 1 = g)
 * with host_in[Q][N] (pre-collision values, population order above),
 * rounded to the storage format.  Synchronises the stream.  This is a state
 * edit, not a resume: it resets the step counter, drops the (phi u) history
 * of the first-order phase-field equilibrium and the partial sums of phi,
 * and FP16 formats re-encode against the current references.  Use
 * mplb_save / mplb_load to checkpoint and resume.  Errors: EINVAL, ESTATE
 * (FP16 formats before mplb_init; attached to a batch), EDEVICE. */
int mplb_set_populations(mplb_solver *s, int32_t which, const double *host_in);

/* Checkpoint and resume.  mplb_save_bytes: size of the host blob mplb_save
 * writes for the solver's current state (0 for a NULL solver).  mplb_save
 * copies into host_blob (at least that many bytes, caller-owned) everything
 * a following step reads, in the stored representation: the population
 * buffers of the current level, the per-cell references of the FP16
 * formats, the (phi u) history, the partial sums of phi if the last update
 * wrote them, the step counter and the launch settings, with a hash of the
 * parameters.  mplb_load restores such a blob into a solver created with
 * equal parameters (any arena); the loaded solver's later steps are bit for
 * bit those the saved one would have taken.  Both synchronise the stream.
 * Errors: EINVAL (NULL arguments, blob too small, another format or other
 * parameters), ESTATE (save before mplb_init; load into an attached
 * solver), EDEVICE.  Design, not in the paper. */
size_t mplb_save_bytes(const mplb_solver *s);
int mplb_save(mplb_solver *s, void *host_blob, size_t bytes);
int mplb_load(mplb_solver *s, const void *host_blob, size_t bytes);

/* Threads per block of the cell update (x, y, z); (0, 0, 0) = library
 * default (as wide in x as the lattice, up to 256).  Between 1 and 256
 * threads; bz = 1 in 2-D.  Blocks a multiple of 64 wide in x on lattices
 * periodic in x take wavefront-uniform (row-form) addressing; results do not
 * depend on the shape.  Errors: EINVAL.  Design, not in the paper. */
int mplb_set_block(mplb_solver *s, int32_t bx, int32_t by, int32_t bz);

/* Next order parameter from partial sums.  phi at a cell is the zeroth
 * moment of the phase-field populations pulled there (Sec. 2.2); on 3-D
 * lattices periodic in x with nx a multiple of 64 up to 256 (or 512 with
 * FP32 storage), y and z periodic or walls, and plain phase-field storage
 * (FP64, FP32, FP16S), the update kernel works on tiles of whole rows (as
 * many rows as 512 threads, 256 with FP64 and FP16S, allow, dividing ny),
 * sums each cell's stored phase-field values towards the cells they stream
 * to while it holds them, and the next step merges a few partial sums per
 * cell instead of re-reading all Q pulled values.  The sums run in another
 * order than the pull sum, so results agree with mode 0 to round-off, not
 * bit for bit (they do not depend on the block shape set by
 * mplb_set_block).  The first step after mplb_init, mplb_set_populations or
 * a step in mode 0 uses the pull sum.  A batch (mplb_batch_*) steps such a
 * solver the same way, with the same bits; partial sums carry into and out
 * of a batch run.  mode 0: never; 1 (default): wherever it applies.
 * Errors: EINVAL, ESTATE (attached to a batch).  Design, not in the paper. */
int mplb_set_phi_partials(mplb_solver *s, int32_t mode);

/* Rows per tile (>= 1) if the next update of this solver writes partial
 * sums of phi, 0 if not; <0 on error. */
int mplb_uses_phi_partials(const mplb_solver *s);

/* Autotuner: time candidate block shapes for the step kernels (each over
 * `steps` steps after two warm-up steps, device time from HIP events), select
 * the fastest, and write it to best[3].  The solver is advanced by the timed
 * steps, so tune on a scratch solver of representative size.  candidates is
 * an array of ncand (bx, by, bz) triples, or NULL for the built-in list.
 * Errors: EINVAL, ESTATE (attached to a batch), EDEVICE.  Design, not in
 * the paper. */
int mplb_tune_block(mplb_solver *s, int32_t steps, const int32_t *candidates, int32_t ncand,
                    int32_t best[3], double *best_ms_per_step);

/* Release the handle, its step graph and its capture stream (the arena stays
 * the caller's).  Waits for the handle's stream when a step graph exists, so
 * that no replay is in flight when the graph goes. */
void mplb_destroy(mplb_solver *s);

/* ---------------------------------------------------------------------------
 * Batches (design, not in the paper): many independent solvers of one
 * dimension and storage format advance together.  The small ones share
 * launches over a tile list that covers every such lattice, one block per
 * tile: per step a phi launch and an update launch, plus one launch per row
 * length (64, 128, 192, 256, 512) for the solvers whose update sums the next
 * phi (mplb_set_phi_partials); large ones step with their own kernels beside
 * them (mplb_batch_set_solo_cells).  Each
 * attached solver has its own parameters, lattice size and activity window;
 * a solver's result is identical whether it is stepped alone or in a batch
 * (same per-cell arithmetic, same step form).  Steps are replayed from a
 * captured hipGraph in chunks of `graph_chunk` steps.  max_tiles bounds the
 * tile list: per solver about N / (block threads) block tiles, plus
 * ny nz / rows tiles where the update sums phi.
 * ------------------------------------------------------------------------- */
typedef struct mplb_batch mplb_batch;

/* Device bytes of the batch tables for `capacity` solvers and `max_tiles`
 * tiles in total. */
size_t mplb_batch_table_bytes(int32_t capacity, int64_t max_tiles);

/* dev_table: 256-byte aligned device memory of mplb_batch_table_bytes(),
 * caller-owned; hip_stream: a created (non-NULL) stream, which must also be
 * the stream of every solver that will be attached (step chunks are captured
 * from it).  Errors: EINVAL, ENOMEM (table too small), EDEVICE. */
int mplb_batch_create(int32_t dim, int32_t storage, int32_t capacity, int64_t max_tiles,
                      void *dev_table, size_t table_bytes, void *hip_stream, mplb_batch **out);

/* Block (= tile) shape of the batched kernels; at most 256 threads.
 * Rebuilds the tile list.  Errors: EINVAL, ENOMEM (tile list full). */
int mplb_batch_set_block(mplb_batch *b, int32_t bx, int32_t by, int32_t bz);

/* Graph chunk in steps (>= 1), or 0 to launch every step directly. */
int mplb_batch_set_graph_chunk(mplb_batch *b, int32_t chunk);

/* Autotuner: time `steps` batch steps (after one warm-up step) for each
 * candidate block shape (candidates = ncand triples bx, by, bz; NULL = a
 * built-in list), keep the fastest and report it in best[3] and its time per
 * step.  Timing needs real work, so every attached domain whose window is
 * open advances by up to ncand * (steps + 1) steps: tune on a copy of the
 * workload.  Errors: EINVAL (steps < 1, no valid candidate, no attached
 * domain), EDEVICE. */
int mplb_batch_tune_block(mplb_batch *b, int32_t steps, const int32_t *candidates, int32_t ncand,
                          int32_t best[3], double *best_ms_per_step);

/* Attach an initialised solver for the next nsteps batch steps; *slot
 * receives its slot (and its status flag is cleared).  The solver must not
 * step, be re-initialised or loaded on its own while attached (those calls
 * return ESTATE).  Errors: EINVAL (dimension/storage/stream mismatch),
 * ENOMEM (no free slot or tile list full), ESTATE (solver not initialised
 * or already attached). */
int mplb_batch_attach(mplb_batch *b, mplb_solver *s, int64_t nsteps, int32_t *slot);

/* Detach the solver in `slot` (its state stays valid and readable). */
int mplb_batch_detach(mplb_batch *b, int32_t slot);

/* Advance the batch by nsteps (asynchronous): every attached solver whose
 * window covers a step is advanced by it. */
int mplb_batch_step(mplb_batch *b, int64_t nsteps);

/* Domains of at least min_cells cells (default 2^20) fill the GPU on their
 * own: a batch steps each with its solver's own kernels (the same ones
 * mplb_step launches, same results), on the solvers' stream, while the
 * smaller domains share the batched launches, replayed from the captured
 * graph on a second stream of the batch, so that the two overlap.  0: every
 * domain steps alone; a value above every domain's size: all share.
 * Applies to solvers attached after the call.  mplb_batch_is_solo: 1 if the
 * solver in `slot` steps alone, 0 if it shares the batched launches, <0 on
 * error.  Errors: EINVAL. */
int mplb_batch_set_solo_cells(mplb_batch *b, int64_t min_cells);
int mplb_batch_is_solo(const mplb_batch *b, int32_t slot);

/* Steps the solver in `slot` still has to take (0 = finished or retired). */
int mplb_batch_remaining(const mplb_batch *b, int32_t slot, int64_t *remaining);

/* Health of every slot, status[capacity]: MPLB_OK for an attached solver
 * whose order parameter has stayed finite, MPLB_EUNSTABLE for one whose
 * order parameter held a non-finite value at some batch step (checked by
 * the batch's phi stage at every step, inside the captured graph; a
 * non-finite population of either set reaches phi within a step),
 * MPLB_ESTATE for an empty slot.  An unstable solver is retired by this call:
 * its window closes, so it takes no further batch steps; detach it to free
 * the slot.  Synchronises the batch stream.  Errors: EINVAL, EDEVICE. */
int mplb_batch_status(mplb_batch *b, int32_t *status);

/* Batch steps taken so far. */
int64_t mplb_batch_steps_done(const mplb_batch *b);

/* Release the batch handle and its graph (attached solvers are detached). */
void mplb_batch_destroy(mplb_batch *b);

/* Message describing the last failed call on this thread ("" if none). */
const char *mplb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
