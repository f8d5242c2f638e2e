// Host-side interface between the C ABI (api.cpp) and the kernel launchers
// (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.hpp"

namespace mplb {

enum { ST_FP64 = 0, ST_FP32 = 1, ST_FP16S = 2, ST_FP16S_ALL = 3 };

// Physical parameters in the form the kernels use (double on the host,
// converted to the arithmetic type at launch).
struct PhysD {
    double rho_l, drho;    // rho = rho_l + drho phi
    double nu_l, dnu;      // nu = nu_l + dnu phi            (visc_interp 0)
    double rnu_l, drnu;    // nu = (rnu_l + drnu phi) / rho  (visc_interp 1)
    double beta, kappa;    // chemical potential coefficients
    double gx, gy, gz;     // body-force acceleration
    double inv_tpb;        // 1 / taubar_phi
    double src_pre;        // 1 - 1/(2 taubar_phi)
    double four_W;         // 4 / W
    double scl_l, dscl;    // FP16 flow codes' scale rho cs^2 = scl_l + dscl phi
    int visc_interp;
    int collision;         // 0 cumulant, 1 SRT
    int cac_edf;           // phase-field equilibrium: 0 second-order, 1 first-order + correction
};

// Device buffers one launch works on.  "in" buffers hold the post-collision
// state of the previous step (pre-collision values are pulled from them);
// "out" buffers receive the new post-collision state.
struct Ptrs {
    const void *Fin;
    void *Fout;
    const void *Gin;
    void *Gout;
    // order parameter of the current time level: [np] in the arithmetic
    // type; FP16 formats: [np] 8-byte records (phi, packed references of the
    // values the cell wrote a step earlier), see device.hpp "FP16 storage"
    void *phi;
    // FP16 formats: the packed references the update writes for the values
    // it stores ([np]), and the rest-direction values of the FP16 sets in
    // FP32 ([np] each, null for a set in plain storage)
    unsigned *ref;
    const float *frest_in, *grest_in;
    float *frest_out, *grest_out;
    // first-order phase-field equilibrium: (phi u) per cell, [3][np], of the
    // previous step (valid when have_prev) and of this step
    const void *phiu_in;
    void *phiu_out;
    int have_prev;
};

struct Ctx {
    int dim;
    int storage;
    Geom g;
    PhysD ph;
    dim3 block;
    hipStream_t stream;
    Ptrs p;
};

hipError_t launch_phi(const Ctx &c);
hipError_t launch_collide(const Ctx &c);
// Partial sums of the next order parameter, written by launch_collide_nphi
// for launch_phi_merge of the following step: part [3][np], edge
// [2][3][ny / by][nz][nx] in the arithmetic type; by = tile rows,
// nphi_rows(nx, ny, storage format).
struct NextPhi {
    void *part;
    void *edge;
    int by;
};
// The update kernel that also sums the next order parameter from the values
// it stores, tile by tile (3-D, x periodic, nx as nphi_width_ok, y and z
// periodic or walls); nphi_ok tells whether it
// applies.  Its tiles are whole rows by nphi_rows rows, whatever
// the block shape of the other kernels.
bool nphi_ok(const Ctx &c);
int nphi_rows(int nx, int ny, int storage);
// Row lengths the phi-summing update takes: multiples of 64 up to 256, and
// 512 with FP32 arithmetic (one row per 512-thread tile).
bool nphi_width_ok(int nx, int storage);
// Groups of the batched phi-summing update by row length 64, 128, 192, 256, 512.
constexpr int NPHI_GROUPS = 5;
constexpr int nphi_group_width(int k) { return k < 4 ? 64 * (k + 1) : 512; }
constexpr int nphi_group(int nx) { return nx == 512 ? 4 : nx / 64 - 1; }
hipError_t launch_collide_nphi(const Ctx &c, const NextPhi &q);
// phi of the current level from the partial sums of the previous update.
hipError_t launch_phi_merge(const Ctx &c, const NextPhi &q);
// Equilibrium initial state from device FP64 fields (phi[N], u[dim][N], p[N])
// written into the Fout/Gout buffers in pull layout.
hipError_t launch_init(const Ctx &c, const double *phi, const double *u, const double *pr);
// Pre-collision populations a0..a1-1 of set `which` (0 f', 1 g) from the
// Fin/Gin buffers into dst[(a-a0)][N] (FP64).
hipError_t launch_get_pop(const Ctx &c, int which, int a0, int a1, double *dst);
// The inverse: src[(a-a0)][N] into the Fout/Gout buffers in pull layout.
hipError_t launch_set_pop(const Ctx &c, int which, int a0, int a1, const double *src);
// References of the FP16 formats (the ref array) for an initial state, from
// FP64 order-parameter and pressure fields.
hipError_t launch_set_refs(const Ctx &c, const double *phi, const double *pr);
// One macroscopic field of the state held in Fin/Gin (phi must be current).
hipError_t launch_field(const Ctx &c, int field, double *dst);
// Deterministic FP64 reduction: partials (at least reduce_blocks() x 8
// doubles), out[8] = {sum phi, sum rho ux, uy, uz, max|u|, nonfinite count}.
hipError_t launch_reduce(const Ctx &c, double *partials, double *out);
int reduce_blocks(const Ctx &c);
// launch_reduce with the partials and the result in the library's static
// device scratch (of the current device); *result receives the device
// address of the 8 results.  hipErrorInvalidValue if the reduction needs
// more partial blocks than the scratch holds (reduce_scratch_max_blocks).
hipError_t launch_reduce_static(const Ctx &c, double **result);
int reduce_scratch_max_blocks();

// One domain of a batch, as the batched kernels read it from device memory.
struct BatchDom {
    Geom g;
    PhysD ph;
    void *F[2], *G[2], *phi;
    unsigned *ref;
    float *frest[2], *grest[2];
    void *phiu[2];
    long long first, last;  // active for batch steps first <= t < last
    long long hist_from;    // (phi u) of the previous step valid for t >= hist_from
    // phi-summing update (see NextPhi): tile rows, 0 if the domain's update
    // does not sum phi; the partial sums; the phi stage of steps t >=
    // nphi_from merges them (earlier ones sum the pulled populations)
    int nphi_by;
    void *npart, *nedge;
    long long nphi_from;
};

// A tile of a batch: domain index, origin cell (x0, y0, z0), end of its
// plane range z1 and width w: w cells in x by (threads per block) / w rows,
// one plane.
struct BatchTile {
    int dom, x0, y0, z0, z1, w;
};

// True when the row-form kernels apply: block a multiple of 64 wide in x,
// x periodic, population arrays of fewer than 2^31 elements.
bool row_form_ok(int dim, const Geom &g, dim3 block);
// row: every attached domain satisfies row_form_ok with this block.
// One batch step over the tile list (*ntiles entries), batch step index
// *tbase + step_off.  collision: operator code, bit 0 the flow collision, bit
// 1 the first-order phase-field equilibrium (shared by all domains).  The
// phi pass and the update run over block tiles (row: every domain takes the
// row form).  grid blocks stride over the tiles (at least one per tile:
// hardware scheduling).
// Tile list: ntiles[0] block tiles of the domains the block kernels update,
// then block tiles of the phi-summing domains up to ntiles[1] (their phi
// stage merges partial sums), then the tiles of the phi-summing update
// (domains with nphi_by > 0: whole rows of one plane), grouped by row length
// (nphi_group): group k starts at ntiles[2 + 2k] and holds ntiles[3 + 2k]
// tiles.  grid[0], grid[1]: blocks of the phi stage and the update;
// grid[2 + k]: of group k's update (0: not launched); 2 + NPHI_GROUPS entries.
// status[dom] is or-ed with 1 when the phi stage finds a non-finite order
// parameter in that domain.
hipError_t launch_batch_step(int dim, int storage, int collision, bool row,
                             const BatchDom *doms, const BatchTile *tiles, const int *ntiles,
                             const long long *tbase, int step_off, dim3 block, const int *grid,
                             int *status, hipStream_t stream);
// Threads per block of the phi-summing update for a storage format and row length.
int nphi_block_threads(int storage, int nx);
hipError_t launch_set_i64(long long *ptr, long long v, hipStream_t stream);
// *flag |= 1 if the order parameter of the context's current level (phi
// array, as the phi stage left it) holds a non-finite value.
hipError_t launch_flag_nonfinite(const Ctx &c, int *flag);
// ptr[0 .. n) = v by a kernel (no memset node when captured into a graph).
hipError_t launch_fill_i32(int *ptr, int n, int v, hipStream_t stream);

}  // namespace mplb
